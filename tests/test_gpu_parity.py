"""GPU path against the oracle, through the C ABI.

Force parity (one evaluation on identical inputs) uses the relative error
M1 = max_i |a_gpu,i - a_oracle,i| / scale_i, with scale_i the sum of the
magnitudes of every contribution to a_i (oracle.accel_scale).  Bars: 1e-12 for
LION_FP64, 1e-6 for the FP32 pair modes.  Trajectory checks compare short runs,
centre-of-mass motion (exact for a linear trap), energies and bitwise
reproducibility.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import lion_inputs as li
from tests import trajectory_bar as tb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6, "mixed_kahan": 1e-6}


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _oracle_trap(oracle, spec):
    V0, U0 = oracle.voltages_for(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                 spec.r0, spec.z0, spec.kappa)
    return oracle.Trap(V0=V0, Omega=spec.omega, U0=U0, R0=spec.r0, Z0=spec.z0, kappa=spec.kappa)


def _sim(w, prec, oracle, **cfg):
    """Simulation fed the oracle's trap voltages (same doubles on both sides).
    Asking for the all-pairs kernels (symmetric=1) means the pair kernel and
    its epilogue (step_launches=2) unless the one-launch step is asked for."""
    from paper_1907_10514_amd import Simulation

    if cfg.get("symmetric") == 1:
        cfg.setdefault("step_launches", 2)
    batched = w.n_traps > 1
    sim = Simulation(w.mass, w.charge, prec, n_per_trap=np.diff(w.offsets) if batched else None)
    if cfg:
        sim.set_config(**cfg)
    for k, spec in enumerate(w.traps):
        tr = _oracle_trap(oracle, spec)
        sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa, trap=k if batched else -1)
        sim.set_damping(spec.gamma, trap=k if batched else -1)
    sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.0)
    return sim


def _m1(a, r, scale):
    return float(np.max(np.sqrt((a[0] - r[0]) ** 2 + (a[1] - r[1]) ** 2 + (a[2] - r[2]) ** 2)
                        / scale))


SIZES = [1, 2, 3, 5, 8, 63, 64, 65, 100, 257, 1000, 1025, 4097]


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("launches", [0, 1, 2])
def test_accel_parity_sizes(torch_gpu, oracle_mod, n, prec, launches):
    """One force evaluation, mixed species, several tiles and ragged tails, on
    the built-in path (the one-workgroup kernel up to 128 ions, one launch per
    step up to 2048, the pair kernels above), the one-launch step and the pair
    kernel with its epilogue (the last two on the multi-workgroup kernels)."""
    w = li.random_cloud(n, seed=100 + n, sigma=60e-6, light_fraction=0.2)
    cfg = dict(small_trap=1, step_launches=launches) if launches else {}
    sim = _sim(w, prec, oracle_mod, **cfg)
    if launches:
        assert sim.config()["step_launches"] == launches
    a = sim.compute_accel()
    tr = _oracle_trap(oracle_mod, w.traps[0])
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    err = _m1(a, r, sc)
    print(f"n={n} {prec} M1={err:.3e}")
    assert err <= TOL[prec]
    sim.close()


def test_accel_parity_multiple_charges(torch_gpu, oracle_mod):
    """Ions of charge -1, +1, +2, +3 e (positive and negative sources)."""
    rng = np.random.default_rng(5)
    w = li.random_cloud(700, seed=6, sigma=50e-6, charge_e=rng.choice([-1, 1, 2, 3], 700))
    tr = _oracle_trap(oracle_mod, w.traps[0])
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 2.5e-8)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 2.5e-8)
    for prec in TOL:
        sim = _sim(w, prec, oracle_mod)
        sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 2.5e-8)
        assert _m1(sim.compute_accel(), r, sc) <= TOL[prec], prec
        sim.close()


@pytest.mark.parametrize("prec,cfgs", [
    ("fp64", [dict(i_per_lane=i, j_split=j) for i in (1, 2, 4) for j in (1, 3, 7, 64)]),
    ("mixed", [dict(i_per_lane=i, j_split=j, flush_len=l) for i in (1, 2, 4) for j in (1, 9, 64)
               for l in (4, 8, 16)]),
    ("mixed_kahan", [dict(i_per_lane=i, j_split=j) for i in (1, 2, 4) for j in (1, 64)]),
    ("fp64", [dict(j_split=64, update_waves=u) for u in (4, 8, 16)]),
])
def test_accel_parity_launch_shapes(torch_gpu, oracle_mod, prec, cfgs):
    """Every launch shape the tuner may pick gives the same forces within the bar."""
    w = li.random_cloud(2113, seed=77, sigma=80e-6, light_fraction=0.2)
    tr = _oracle_trap(oracle_mod, w.traps[0])
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sim = _sim(w, prec, oracle_mod)
    for cfg in cfgs:
        sim.set_config(**cfg)
        err = _m1(sim.compute_accel(), r, sc)
        assert err <= TOL[prec], (cfg, err)
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_accel_parity_full_size_sampled(torch_gpu, oracle_mod, prec):
    """The 16384-ion mixed-species cloud in the default (benchmarked) launch
    shape: 768 sampled targets against the oracle, every source counted."""
    w = li.mixed16384()
    sim = _sim(w, prec, oracle_mod)
    a = sim.compute_accel()
    tr = _oracle_trap(oracle_mod, w.traps[0])
    idx = np.random.default_rng(0).choice(w.n, 768, replace=False)
    rx, ry, rz, sc = oracle_mod.accel_at(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0, idx)
    err = _m1((a[0][idx], a[1][idx], a[2][idx]), (rx, ry, rz), sc)
    print(f"N=16384 {prec} sampled M1={err:.3e} config={sim.config()}")
    assert err <= TOL[prec]
    sim.close()


SYM_SIZES = [1, 2, 3, 100, 255, 256, 257, 1000, 4097, 8191]


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("n", SYM_SIZES)
def test_accel_parity_pair_once(torch_gpu, oracle_mod, n, prec):
    """The kernels that evaluate each unordered pair once (tile pairs, reaction
    sums through LDS) meet the same bars, for full and ragged tiles."""
    w = li.random_cloud(n, seed=300 + n, sigma=60e-6, light_fraction=0.2,
                        charge_e=np.random.default_rng(n).choice([1, 1, 2, -1], n))
    sim = _sim(w, prec, oracle_mod, symmetric=2)
    assert sim.config()["symmetric"] == 2
    a = sim.compute_accel()
    tr = _oracle_trap(oracle_mod, w.traps[0])
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    err = _m1(a, r, sc)
    print(f"pair-once n={n} {prec} M1={err:.3e}")
    assert err <= TOL[prec]
    sim.close()


COINCIDENT = ((1, 2), (10, 500), (999, 3), (256, 257), (0, 255))


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("sym", [1, 2])
def test_coincident_ions(torch_gpu, oracle_mod, prec, sym):
    """Exactly coincident ions (within a tile, across tiles, at tile edges) add
    nothing to each other's field, a select and not softening, on the
    all-pairs and the pair-once kernels; every other term meets the bar."""
    w = li.random_cloud(1000, seed=61, sigma=60e-6,
                        charge_e=np.random.default_rng(62).choice([1, 2, -1], 1000))
    for i, j in COINCIDENT:
        w.x[j], w.y[j], w.z[j] = w.x[i], w.y[i], w.z[i]
    sim = _sim(w, prec, oracle_mod, symmetric=sym)
    a = sim.compute_accel()
    tr = _oracle_trap(oracle_mod, w.traps[0])
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    assert all(np.all(np.isfinite(c)) for c in a)
    err = _m1(a, r, sc)
    print(f"coincident ions {prec} symmetric={sym}: M1={err:.3e}")
    assert err <= TOL[prec]
    sim.close()


def test_coincident_ions_batched(torch_gpu, oracle_mod):
    """The same in the batched kernel, for every precision."""
    w = _large_trap_batch()
    for k, (i, j) in enumerate(((5, 6), (700, 1023), (1030, 1500))):
        w.x[j], w.y[j], w.z[j] = w.x[i], w.y[i], w.z[i]
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    r = oracle_mod.accel_batch(w.offsets, w.x, w.y, w.z, w.charge, w.mass, traps,
                               np.zeros(w.n_traps))
    for prec in TOL:
        sim = _sim(w, prec, oracle_mod)
        a = sim.compute_accel()
        assert all(np.all(np.isfinite(c)) for c in a)
        for k in range(w.n_traps):
            o, e = w.offsets[k], w.offsets[k + 1]
            sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e],
                                        w.mass[o:e], traps[k], 0.0)
            assert _m1([c[o:e] for c in a], [c[o:e] for c in r], sc) <= TOL[prec], (prec, k)
        sim.close()


def test_lost_ion_check(torch_gpu, oracle_mod):
    """Ions farther than r_lost from the trap centre are counted, for any
    radius; a trap beyond the first stability region (q = 1.2) loses its
    cloud within 20 rf periods while the stable one (q = 0.3) keeps it."""
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    w = li.random_cloud(500, seed=71, sigma=30e-6)
    w.x[:7] = 2e-3  # seven ions placed far out
    r = np.sqrt(w.x ** 2 + w.y ** 2 + w.z ** 2)
    sim = _sim(w, "fp64", oracle_mod)
    for rl in (1e-4, 5e-4, 1.5e-3, 3e-3):
        assert sim.count_lost(rl) == int(np.sum(r > rl)), rl
    with pytest.raises(LionError) as ei:
        sim.count_lost(0.0)
    assert ei.value.code == L.LION_ERR_ARG
    sim.close()
    w = li.random_cloud(500, seed=72, sigma=30e-6)
    spec = w.traps[0]
    lost = {}
    for q in (0.3, 1.2):
        V0, U0 = oracle_mod.voltages_for(q, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                         spec.r0, spec.z0, spec.kappa)
        sim = _sim(w, "fp64", oracle_mod)
        sim.set_trap(V0, spec.omega, U0, spec.r0, spec.z0, spec.kappa)
        sim.step(400, spec.dt)  # 20 rf periods
        lost[q] = sim.count_lost(1e-3)
        sim.close()
    print(f"lost beyond 1 mm after 20 rf periods: {lost}")
    assert lost[0.3] == 0 and lost[1.2] > 250


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_pair_once_full_size_and_steps(torch_gpu, oracle_mod, prec):
    """Pair-once kernels at 16384 ions: sampled targets against the oracle;
    45 steps bitwise reproducible; and the first SEGMENT steps of the pair-once
    and of the all-pairs kernels against the oracle, ion by ion within 10x the
    envelope of the oracle's own run under per-step kicks of dt M1 A_i (M1 the
    larger measured force error of the two).  FP64 also compares 45 steps of
    the two kernels within max(1e-12 x extent, 10x the one-ulp envelope)."""
    w = li.mixed16384()
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    sim = _sim(w, prec, oracle_mod, symmetric=2)
    a = sim.compute_accel()
    idx = np.random.default_rng(1).choice(w.n, 512, replace=False)
    rx, ry, rz, sc = oracle_mod.accel_at(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0, idx)
    err = _m1((a[0][idx], a[1][idx], a[2][idx]), (rx, ry, rz), sc)
    print(f"pair-once N=16384 {prec} sampled M1={err:.3e}")
    assert err <= TOL[prec]
    sim.close()
    # the segment against the oracle, both kernels
    ref_a = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    scale = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    segs, m1 = {}, 0.0
    for sym in (2, 1):
        s2 = _sim(w, prec, oracle_mod, symmetric=sym)
        m1 = max(m1, tb.m1(s2.compute_accel(), ref_a, scale))
        s2.step(tb.SEGMENT, spec.dt)
        segs[sym] = s2.get_state()[0]
        s2.close()
    ref = oracle_mod.step(w.state(), w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, tb.SEGMENT)
    kicked = tb.kicked_run(
        lambda st, k: oracle_mod.step(st, w.charge, w.mass, tr, spec.gamma, k * spec.dt, spec.dt, 1),
        tb.nudge(w.state()), tb.SEGMENT, tb.kick(scale, max(m1, tb.M1_FLOOR), spec.dt))
    for sym, got in segs.items():
        r = (tb.ratio(got, ref, kicked, tb.X), tb.ratio(got, ref, kicked, tb.V))
        print(f"N=16384 {prec} symmetric={sym}: {tb.SEGMENT} steps, M1 {m1:.2e}, "
              f"|dx| {r[0]:.2f} bars, |dv| {r[1]:.2f} bars")
        assert r[0] <= 1 and r[1] <= 1, sym
    if prec != "fp64":
        assert m1 <= tb.M1_REF
    # 45 steps: reproducible bits; FP64 also equal across kernels to roundoff growth
    outs = []
    for sym in (2, 2, 1):
        s2 = _sim(w, prec, oracle_mod, symmetric=sym)
        s2.step(45, spec.dt)
        outs.append(s2.get_state()[0])
        s2.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k
    if prec == "fp64":
        ext = np.max(np.abs(w.x))
        err = tb.divergence(outs[0], outs[2], tb.X)
        bar = 1e-12 * ext
        if err >= bar:
            env, _ = tb.ulp_envelope(
                lambda st: oracle_mod.step(st, w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, 45),
                w.state())
            print(f"pair-once N=16384 fp64: 45-step |dx| {err:.3e} > {bar:.3e}; envelope {env:.3e}")
            bar = max(bar, 10 * env)
        assert err < bar


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_pair_once_variants(torch_gpu, oracle_mod, prec, variant):
    """Every pair-once kernel variant the tuner may pick meets the bar, on full
    and ragged tiles, with one common charge (the charge factored out of the
    sums) and with mixed charges (per-source charges in the sums)."""
    for n, mixed_q in ((255, False), (1000, False), (4097, False), (1000, True), (4097, True)):
        q = np.random.default_rng(n).choice([1, 1, 2, -1], n) if mixed_q else None
        w = li.random_cloud(n, seed=500 + n, sigma=60e-6, light_fraction=0.2, charge_e=q)
        sim = _sim(w, prec, oracle_mod, symmetric=2, sym_variant=variant)
        assert sim.config()["sym_variant"] == variant
        tr = _oracle_trap(oracle_mod, w.traps[0])
        r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
        sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
        err = _m1(sim.compute_accel(), r, sc)
        assert err <= TOL[prec], (n, err)
        sim.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("q", [-1, 3])
def test_pair_once_uniform_charge(torch_gpu, oracle_mod, prec, q):
    """All ions of one charge other than +1 e: tile pairs without padding take
    the loop with the charge factored out of the sums, the last ragged tile the
    general loop; both meet the bar with the right sign and scale."""
    for n in (1000, 4096):
        w = li.random_cloud(n, seed=700 + n, sigma=60e-6, light_fraction=0.2,
                            charge_e=np.full(n, q))
        sim = _sim(w, prec, oracle_mod, symmetric=2)
        tr = _oracle_trap(oracle_mod, w.traps[0])
        r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
        sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
        err = _m1(sim.compute_accel(), r, sc)
        assert err <= TOL[prec], (n, q, err)
        sim.close()


def test_pair_once_rejected_where_unsupported(torch_gpu, oracle_mod):
    """Batched handles have no pair-once kernels: asking for them is refused."""
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    b = _small_batch(n_traps=3, seed=5, n_max=20)
    sim = _sim(b, "mixed", oracle_mod)
    with pytest.raises(LionError) as ei:
        sim.set_config(symmetric=2)
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    sim.close()


def test_crystal8_full_run_matches_oracle(torch_gpu, oracle_mod):
    """8 ions, q=0.3, gamma=1e5/s, 20000 steps in FP64: the final state of the
    GPU run equals the oracle's to roundoff growth."""
    w = li.crystal8()
    spec = w.traps[0]
    sim = _sim(w, "fp64", oracle_mod)
    sim.step(w.nsteps, spec.dt)
    st, t = sim.get_state()
    ref = oracle_mod.step(w.state(), w.charge, w.mass, _oracle_trap(oracle_mod, spec), spec.gamma,
                          0.0, spec.dt, w.nsteps)
    assert t == ref["t"]
    ext = np.max(np.abs(ref["z"]))
    for k in ("x", "y", "z"):
        assert np.max(np.abs(st[k] - ref[k])) < 1e-9 * ext, k
    sim.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-5), ("mixed_kahan", 1e-5)])
def test_crystal1024_short_run(torch_gpu, oracle_mod, prec, tol):
    """1024 ions, 200 steps: positions agree with the FP64 oracle."""
    w = li.crystal1024()
    spec = w.traps[0]
    sim = _sim(w, prec, oracle_mod)
    sim.step(200, spec.dt)
    st, _ = sim.get_state()
    ref = oracle_mod.step(w.state(), w.charge, w.mass, _oracle_trap(oracle_mod, spec), spec.gamma,
                          0.0, spec.dt, 200)
    disp = np.max(np.abs(ref["x"] - w.x))
    err = max(np.max(np.abs(st[k] - ref[k])) for k in ("x", "y", "z"))
    print(f"{prec}: max |dx| {err:.3e} m after 200 steps (max displacement {disp:.3e} m)")
    assert err < tol * disp
    sim.close()


def test_crystal1024_observables_match_oracle(torch_gpu, oracle_mod):
    """The 1024-ion cooling run (gamma = 2e5/s, 50000 steps, FP64) forms a
    crystal; its trajectories are chaotic, so its label-free observables are
    compared (section "Verifications / Cooling mechanisms"): the kinetic
    temperature every 1000 steps (every 50 rf periods) and the final energy
    per ion, against the oracle's run stored in tests/golden (written by
    make_crystal1024_observables.py) and its 16 twins.  A twin is the oracle's
    run perturbed as an FP64 force path perturbs it: a one-ulp start shift and,
    after every step, the velocity kick dt M1 A_i xi_i with M1 the FP64 path's
    largest measured force error (start shifts alone decay in the damped
    cloud; a path's rounding enters at every step).  Stated tolerances, from
    the twins' spread: the mean temperature over each stretch of ten samples
    within 3x the twins' largest deviation of that mean; each sample within 3x
    the twins' largest deviation over the samples within five of it (the
    spread of a chaotic observable moves slowly; 16 draws at one sample alone
    underestimate it), and at least 0.5 % of the temperature; energies per ion
    within 3x the twins' largest deviation."""
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "crystal1024_observables.json")
    with open(path) as fh:
        gold = json.load(fh)
    w = li.crystal1024()
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    sim = _sim(w, "fp64", oracle_mod)
    every = gold["every"]
    temps = [float(np.sum(0.5 * w.mass * (w.vx ** 2 + w.vy ** 2 + w.vz ** 2))
                   / (1.5 * w.n * li.K_B))]
    for _ in range(w.nsteps // every):
        sim.step(every, spec.dt)
        st, t = sim.get_state()
        v2 = st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2
        temps.append(float(np.sum(0.5 * w.mass * v2) / (1.5 * w.n * li.K_B)))
    assert t == pytest.approx(gold["base"]["t_end"], rel=1e-15, abs=0)
    temps = np.array(temps)
    base = np.array(gold["base"]["temperature_K"])
    twins = np.array([tw["temperature_K"] for tw in gold["twins"]])
    for a in range(0, base.size, 10):
        b = min(a + 10, base.size)
        spread = np.max(np.abs(twins[:, a:b].mean(1) - base[a:b].mean()))
        dev = abs(temps[a:b].mean() - base[a:b].mean())
        print(f"temperature, mean of samples {a}-{b - 1}: GPU {temps[a:b].mean():.5e} K, oracle "
              f"{base[a:b].mean():.5e} K, deviation {dev / (3 * spread):.2f} of the tolerance")
        assert dev <= 3 * spread, (a, b)
    d = np.max(np.abs(twins - base), axis=0)
    near = np.array([d[max(0, k - 5):k + 6].max() for k in range(d.size)])
    tol = np.maximum(3 * near, 5e-3 * base)
    dev = np.abs(temps - base)
    k = int(np.argmax(dev / tol))
    print(f"temperature: worst sample {k * every} steps, GPU {temps[k]:.5e} K, oracle "
          f"{base[k]:.5e} K, deviation {dev[k] / tol[k]:.2f} of the tolerance; final "
          f"{temps[-1]:.5e} K against {base[-1]:.5e} K")
    assert np.all(dev <= tol)
    kin, coul, dc = sim.energy()
    for name, val in (("kinetic", kin), ("coulomb", coul), ("dc_trap", dc)):
        ref = gold["base"]["energy_per_ion_J"][name]
        spread = max(abs(tw["energy_per_ion_J"][name] - ref) for tw in gold["twins"])
        print(f"energy per ion {name}: GPU {val / w.n:.6e} J, oracle {ref:.6e} J, "
              f"twin spread {spread:.2e}")
        assert abs(val / w.n - ref) <= 3 * spread, name
    sim.close()


def test_centre_of_mass_follows_single_ion_on_gpu(torch_gpu, oracle_mod):
    """Kohn: with one species the centre of mass of the GPU run follows the
    oracle's single-ion trajectory (full rf, damping)."""
    w = li.random_cloud(512, seed=3, sigma=40e-6)
    spec = w.traps[0]
    for prec in ("fp64", "mixed"):
        sim = _sim(w, prec, oracle_mod)
        sim.step(2000, spec.dt)
        st, _ = sim.get_state()
        com0 = {k: np.array([np.mean(getattr(w, k))]) for k in ("x", "y", "z", "vx", "vy", "vz")}
        one = oracle_mod.step(com0, [li.E_CHARGE], [li.REF_MASS], _oracle_trap(oracle_mod, spec),
                              spec.gamma, 0.0, spec.dt, 2000)
        for k in ("x", "y", "z"):
            amp = np.max(np.abs(getattr(w, k)))
            tol = 1e-9 if prec == "fp64" else 1e-6
            assert abs(np.mean(st[k]) - one[k][0]) < tol * amp, (prec, k)
        sim.close()


def test_free_ion_damping_exact(torch_gpu, oracle_mod):
    """Single ion, no field: v decays as exp(-gamma t) (cooling verification)."""
    from paper_1907_10514_amd import Simulation

    sim = Simulation([li.REF_MASS], [li.E_CHARGE], "fp64")
    sim.set_damping(1e6)
    sim.set_state([0.0], [0.0], [0.0], [3.0], [-1.0], [0.5], 0.0)
    sim.step(1000, li.DT)
    st, _ = sim.get_state()
    assert st["vx"][0] == pytest.approx(3.0 * math.exp(-1e6 * 1000 * li.DT), rel=1e-12, abs=0)
    sim.close()


def test_energy_matches_oracle(torch_gpu, oracle_mod):
    w = li.random_cloud(900, seed=8, sigma=40e-6, light_fraction=0.3)
    tr = _oracle_trap(oracle_mod, w.traps[0])
    sim = _sim(w, "fp64", oracle_mod)
    k, c, d = sim.energy()
    ko, co, do = oracle_mod.energy(w.state(), w.charge, w.mass, tr)
    assert k == pytest.approx(ko, rel=1e-13, abs=0)
    assert c == pytest.approx(co, rel=1e-12, abs=0)
    assert d == pytest.approx(do, rel=1e-12, abs=0)
    sim.close()


def test_bitwise_reproducible_and_launch_mode_independent(torch_gpu, oracle_mod):
    """Fixed-order reductions: reruns, graph vs plain launches and chunk sizes
    give identical bits (one launch shape throughout: a tuned shape for this
    size may differ from the built-in one)."""
    w = li.random_cloud(3000, seed=9, sigma=60e-6)
    spec = w.traps[0]
    outs = []
    base = dict(i_per_lane=2, j_split=16, flush_len=8)
    for cfg in (base, base, dict(base, use_graph=2), dict(base, chunk_steps=7)):
        sim = _sim(w, "mixed", oracle_mod, **cfg)
        sim.step(45, spec.dt)
        outs.append(sim.get_state()[0])
        sim.close()
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k


def test_checkpoint_resume_is_bit_identical(torch_gpu, oracle_mod):
    """get_state + set_state + step equals stepping straight through (with a
    binary time step, so both paths see identical times)."""
    w = li.random_cloud(600, seed=10, sigma=50e-6)
    dt = 2.0 ** -26
    a = _sim(w, "fp64", oracle_mod)
    a.step(100, dt)
    sa, ta = a.get_state()
    b = _sim(w, "fp64", oracle_mod)
    b.step(60, dt)
    sb, tb = b.get_state()
    b.set_state(sb["x"], sb["y"], sb["z"], sb["vx"], sb["vy"], sb["vz"], tb)
    b.step(40, dt)
    sc, tc = b.get_state()
    assert tc == ta
    for k in sa:
        assert np.array_equal(sa[k], sc[k]), k
    a.close()
    b.close()


def _small_batch(n_traps=24, seed=13, n_max=300):
    return li.batch512(n_traps=n_traps, n_min=2, n_max=n_max, seed=seed, nsteps=0)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("charges", ["common", "mixed"])
def test_batch_accel_parity(torch_gpu, oracle_mod, prec, charges):
    """Batched field against the oracle for every launch shape the tuner may
    pick (workgroup size x targets per thread), with one common charge (sums
    scaled by it once) and with per-ion charges."""
    w = _small_batch()
    if charges == "mixed":
        w.charge = np.random.default_rng(7).choice([1, 2, -1], w.n) * li.E_CHARGE
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    r = oracle_mod.accel_batch(w.offsets, w.x, w.y, w.z, w.charge, w.mass, traps,
                               np.zeros(w.n_traps))
    from paper_1907_10514_amd import tune

    for cfg in tune.batch_candidates():  # every shape the tuner may pick
        sim = _sim(w, prec, oracle_mod, **cfg)
        a = sim.compute_accel()
        for k in range(w.n_traps):
            o, e = w.offsets[k], w.offsets[k + 1]
            sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e], w.mass[o:e],
                                        traps[k], 0.0)
            err = _m1([c[o:e] for c in a], [c[o:e] for c in r], sc)
            assert err <= TOL[prec], (cfg, k, err)
        sim.close()


def test_batch_max_trap_parity(torch_gpu, oracle_mod):
    """Traps of 1 and of the maximum 1024 ions."""
    w = li.batch512(n_traps=3, n_min=1, n_max=1024, seed=1, nsteps=0)
    sizes = np.array([1, 1024, 513])
    rng = np.random.default_rng(2)
    w.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(w.offsets[-1])
    w.mass = np.full(n, li.REF_MASS)
    w.charge = np.full(n, li.E_CHARGE)
    w.x, w.y, w.z = rng.normal(0, 30e-6, (3, n))
    w.vx, w.vy, w.vz = rng.normal(0, 1.0, (3, n))
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    r = oracle_mod.accel_batch(w.offsets, w.x, w.y, w.z, w.charge, w.mass, traps, np.zeros(3))
    for prec in TOL:
        for block in (256, 1024):
            sim = _sim(w, prec, oracle_mod, batch_block=block)
            a = sim.compute_accel()
            for k in range(3):
                o, e = w.offsets[k], w.offsets[k + 1]
                sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e],
                                            w.mass[o:e], traps[k], 0.0)
                assert _m1([c[o:e] for c in a], [c[o:e] for c in r], sc) <= TOL[prec]
            sim.close()


def test_batch_trajectory_matches_oracle(torch_gpu, oracle_mod):
    w = _small_batch(n_traps=16, seed=21, n_max=200)
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    g = np.array([s.gamma for s in w.traps])
    dts = np.array([s.dt for s in w.traps]) * np.linspace(0.8, 1.2, w.n_traps)
    ref = oracle_mod.step_batch(w.offsets, w.state(), w.charge, w.mass, traps, g,
                                np.zeros(w.n_traps), dts, 150)
    sim = _sim(w, "fp64", oracle_mod, chunk_steps=40)
    sim.step(150, dts)
    st, _ = sim.get_state()
    for k in range(w.n_traps):
        o, e = w.offsets[k], w.offsets[k + 1]
        disp = np.max(np.abs(ref["x"][o:e] - w.x[o:e])) + 1e-12
        for c in ("x", "y", "z"):
            assert np.max(np.abs(st[c][o:e] - ref[c][o:e])) < 1e-10 * disp, (k, c)
    sim.close()


@pytest.mark.parametrize("n", [161, 1000, 2048, 2049])
def test_one_launch_step_matches_oracle(torch_gpu, oracle_mod, n):
    """One launch per step (each workgroup ends the step for its targets, the
    positions alternating between two buffers): 61 FP64 steps against the
    oracle, in chunks of 25 (odd and even chunk lengths, so the last step of a
    chunk finds the positions in either buffer), bit for bit the same in chunks
    of 7, as plain launches, and in calls that stop and resume between chunks
    (a binary time step, so that resumed calls see identical times).  2049
    ions take the path on request (above the built-in limit)."""
    w = li.random_cloud(n, seed=500 + n, sigma=80e-6, light_fraction=0.2)
    spec = w.traps[0]
    dt = 2.0 ** -26
    tr = _oracle_trap(oracle_mod, spec)
    ref = oracle_mod.step(w.state(), w.charge, w.mass, tr, spec.gamma, 0.0, dt, 61)
    runs = []
    for cfg, calls in ((dict(chunk_steps=25), (61,)), (dict(chunk_steps=7), (61,)),
                       (dict(chunk_steps=25, use_graph=2), (61,)),
                       (dict(chunk_steps=25), (13, 30, 18))):
        sim = _sim(w, "fp64", oracle_mod, step_launches=1, **cfg)
        assert sim.config()["step_launches"] == 1
        for c in calls:
            sim.step(c, dt)
        runs.append(sim.get_state())
        sim.close()
    st, t = runs[0]
    assert t == 61 * dt
    disp = np.max(np.abs(ref["x"] - w.x))
    for c in ("x", "y", "z"):
        assert np.max(np.abs(st[c] - ref[c])) < 1e-10 * disp, c
    vs = np.max(np.abs(ref["vx"]))
    for c in ("vx", "vy", "vz"):
        assert np.max(np.abs(st[c] - ref[c])) < 1e-9 * vs, c
    for other, _ in runs[1:]:
        for c in st:
            assert np.array_equal(st[c], other[c]), c


@pytest.mark.parametrize("prec", ["mixed", "mixed_kahan"])
def test_one_launch_step_fp32_forces_along_a_run(torch_gpu, oracle_mod, prec):
    """FP32 pairs on the one-launch step: forces against the oracle at the
    start and at the state reached after 75 steps (the kernel that steps also
    evaluates them), and the built-in shape of a 1000-ion trap is this path."""
    w = li.random_cloud(1000, seed=71, sigma=80e-6, light_fraction=0.2)
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    sim = _sim(w, prec, oracle_mod, chunk_steps=30)
    assert sim.config()["step_launches"] == 1
    for k in (0, 75):
        if k:
            sim.step(k, spec.dt)
        st, t = sim.get_state()
        r = oracle_mod.accel(st["x"], st["y"], st["z"], w.charge, w.mass, tr, t)
        sc = oracle_mod.accel_scale(st["x"], st["y"], st["z"], w.charge, w.mass, tr, t)
        assert _m1(sim.compute_accel(), r, sc) <= TOL[prec], k
    sim.close()


def _tiny_trap_batch(sizes, seed):
    w = li.batch512(n_traps=len(sizes), n_min=2, n_max=12, seed=seed, nsteps=0)
    rng = np.random.default_rng(seed + 1)
    w.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(w.offsets[-1])
    w.mass = rng.choice([li.REF_MASS, 17 * li.AMU], n)
    w.charge = rng.choice([1, 1, 2], n) * li.E_CHARGE
    w.x, w.y, w.z = rng.normal(0, 15e-6, (3, n))
    w.vx, w.vy, w.vz = rng.normal(0, 1.0, (3, n))
    return w


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_one_wave_traps_match_oracle(torch_gpu, oracle_mod, prec):
    """Traps of at most 16 ions step on one wave (the one-wave kernel, the
    built-in shape).  Forces of every trap against the oracle before and after
    a 130-step run (three launches of 50 steps, so the per-launch table of RF
    phases is refilled within a launch and across launches); in FP64 the run
    itself against the oracle's batched steps."""
    sizes = np.array([1, 2, 3, 5, 7, 8, 9, 11, 12, 12, 4, 6, 13, 16])
    w = _tiny_trap_batch(sizes, seed=61)
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    sim = _sim(w, prec, oracle_mod, chunk_steps=50)
    assert sim.config()["batch_block"] == 64
    r = oracle_mod.accel_batch(w.offsets, w.x, w.y, w.z, w.charge, w.mass, traps,
                               np.zeros(w.n_traps))
    a = sim.compute_accel()
    for k in range(w.n_traps):
        o, e = w.offsets[k], w.offsets[k + 1]
        sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e], w.mass[o:e],
                                    traps[k], 0.0)
        assert _m1([c[o:e] for c in a], [c[o:e] for c in r], sc) <= TOL[prec], k
    g = np.array([s.gamma for s in w.traps])
    dts = np.array([s.dt for s in w.traps]) * np.linspace(0.8, 1.2, w.n_traps)
    sim.step(130, dts)
    st, _ = sim.get_state()
    t = 130 * dts
    r = oracle_mod.accel_batch(w.offsets, st["x"], st["y"], st["z"], w.charge, w.mass, traps, t)
    a = sim.compute_accel()
    for k in range(w.n_traps):
        o, e = w.offsets[k], w.offsets[k + 1]
        sc = oracle_mod.accel_scale(st["x"][o:e], st["y"][o:e], st["z"][o:e], w.charge[o:e],
                                    w.mass[o:e], traps[k], t[k])
        assert _m1([c[o:e] for c in a], [c[o:e] for c in r], sc) <= TOL[prec], k
    if prec == "fp64":
        ref = oracle_mod.step_batch(w.offsets, w.state(), w.charge, w.mass, traps, g,
                                    np.zeros(w.n_traps), dts, 130)
        for k in range(w.n_traps):
            o, e = w.offsets[k], w.offsets[k + 1]
            disp = np.max(np.abs(ref["x"][o:e] - w.x[o:e])) + 1e-12
            for c in ("x", "y", "z"):
                assert np.max(np.abs(st[c][o:e] - ref[c][o:e])) < 1e-10 * disp, (k, c)
    sim.close()


@pytest.mark.parametrize("n", [13, 40, 64])
def test_one_wave_shape_up_to_64_ions(torch_gpu, oracle_mod, n):
    """The 64-thread shape, asked for explicitly, on lone traps above the
    built-in threshold: forces and a 60-step FP64 run against the oracle."""
    w = li.random_cloud(n, seed=300 + n, sigma=20e-6, light_fraction=0.2)
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    sim = _sim(w, "fp64", oracle_mod, small_trap=2, batch_block=64)
    assert sim.config()["batch_block"] == 64
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    assert _m1(sim.compute_accel(), r, sc) <= TOL["fp64"]
    ref = oracle_mod.step(w.state(), w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, 60)
    sim.step(60, spec.dt)
    st, _ = sim.get_state()
    disp = np.max(np.abs(ref["x"] - w.x)) + 1e-12
    for c in ("x", "y", "z"):
        assert np.max(np.abs(st[c] - ref[c])) < 1e-10 * disp, c
    sim.close()


@pytest.mark.parametrize("n,block", [(17, 256), (24, 256), (33, 512), (48, 512), (40, 1024),
                                     (56, 1024), (64, 1024)])
@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_owner_parts_split_up_to_64_ions(torch_gpu, oracle_mod, n, block, prec):
    """Traps of <= 64 ions on 256 to 1024 threads: up to 48 ions (and block / 8)
    the wave kernel on block / 64 waves with 8 parts per target, above that the
    batched kernel's m owners followed by at most 8 source parts (48 ions on 512
    threads would take 10 without the cap). Forces against the oracle, then
    forces after 60 steps; in FP64 the run itself against the oracle's steps."""
    w = li.random_cloud(n, seed=500 + n, sigma=20e-6, light_fraction=0.2)
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    sim = _sim(w, prec, oracle_mod, small_trap=2, batch_block=block)
    assert sim.config()["batch_block"] == block
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    assert _m1(sim.compute_accel(), r, sc) <= TOL[prec]
    sim.step(60, spec.dt)
    st, t = sim.get_state()
    r = oracle_mod.accel(st["x"], st["y"], st["z"], w.charge, w.mass, tr, t)
    sc = oracle_mod.accel_scale(st["x"], st["y"], st["z"], w.charge, w.mass, tr, t)
    assert _m1(sim.compute_accel(), r, sc) <= TOL[prec]
    if prec == "fp64":
        ref = oracle_mod.step(w.state(), w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, 60)
        disp = np.max(np.abs(ref["x"] - w.x)) + 1e-12
        for c in ("x", "y", "z"):
            assert np.max(np.abs(st[c] - ref[c])) < 1e-10 * disp, c
    sim.close()


def test_one_wave_shape_refused_above_64_ions(torch_gpu, oracle_mod):
    from paper_1907_10514_amd.lion import LionError

    w = li.random_cloud(65, seed=7, sigma=20e-6)
    sim = _sim(w, "fp64", oracle_mod)
    with pytest.raises(LionError, match="at most 64"):
        sim.set_config(batch_block=64)
    sim.close()


def _large_trap_batch():
    """Traps of the maximum 1024 ions down to 2, with a ragged one of 257 and
    mixed charges."""
    w = li.batch512(n_traps=7, n_min=2, n_max=512, seed=37, nsteps=0)
    sizes = np.array([1024, 600, 257, 256, 255, 40, 2])
    rng = np.random.default_rng(38)
    w.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(w.offsets[-1])
    w.mass = np.full(n, li.REF_MASS)
    w.charge = rng.choice([1, 1, 2], n) * li.E_CHARGE
    w.x, w.y, w.z = rng.normal(0, 30e-6, (3, n))
    w.vx, w.vy, w.vz = rng.normal(0, 1.0, (3, n))
    return w


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-4), ("mixed_kahan", 1e-4)])
@pytest.mark.parametrize("block", [256, 1024])
def test_batch_large_traps_run(torch_gpu, oracle_mod, prec, tol, block):
    """Traps up to the 1024-ion maximum in the batched kernel: forces, and a
    60-step run of every trap (4 targets per thread at 256 threads, 2 at 1024)
    against the oracle."""
    w = _large_trap_batch()
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    dts = np.array([s.dt for s in w.traps])
    sim = _sim(w, prec, oracle_mod, batch_block=block, chunk_steps=25)
    a = sim.compute_accel()
    r = oracle_mod.accel_batch(w.offsets, w.x, w.y, w.z, w.charge, w.mass, traps,
                               np.zeros(w.n_traps))
    for k in range(w.n_traps):
        o, e = w.offsets[k], w.offsets[k + 1]
        sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e], w.mass[o:e],
                                    traps[k], 0.0)
        assert _m1([c[o:e] for c in a], [c[o:e] for c in r], sc) <= TOL[prec], k
    sim.step(60, dts)
    st, _ = sim.get_state()
    assert sim.check_finite() == 0
    sim.close()
    ref = oracle_mod.step_batch(w.offsets, w.state(), w.charge, w.mass, traps,
                                np.array([s.gamma for s in w.traps]), np.zeros(w.n_traps), dts,
                                60)
    for k in range(w.n_traps):
        o, e = int(w.offsets[k]), int(w.offsets[k + 1])
        disp = np.max(np.abs(ref["x"][o:e] - w.x[o:e])) + 1e-12
        for c in ("x", "y", "z"):
            assert np.max(np.abs(st[c][o:e] - ref[c][o:e])) < tol * disp, (k, c)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("block,tpt", [(256, 1), (256, 2), (256, 4), (512, 1), (512, 2),
                                       (512, 4), (1024, 1), (1024, 2)])
def test_batch_tuner_shapes_accel_parity(torch_gpu, oracle_mod, prec, block, tpt):
    """Every (threads per trap, targets per thread) shape the batch tuner may
    pick, forced on traps of 2 to 1024 ions (the FP32 runs of the threads with
    several targets included), with mixed charges and with one common charge
    (factored out of the sums): forces against the oracle trap by trap."""
    w = _large_trap_batch()
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    for charge in (w.charge, np.full(w.n, li.E_CHARGE)):
        w.charge = charge
        sim = _sim(w, prec, oracle_mod, batch_block=block, batch_tpt=tpt)
        a = sim.compute_accel()
        sim.close()
        r = oracle_mod.accel_batch(w.offsets, w.x, w.y, w.z, w.charge, w.mass, traps,
                                   np.zeros(w.n_traps))
        for k in range(w.n_traps):
            o, e = w.offsets[k], w.offsets[k + 1]
            sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e],
                                        w.mass[o:e], traps[k], 0.0)
            assert _m1([c[o:e] for c in a], [c[o:e] for c in r], sc) <= TOL[prec], k


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("n", [100, 300, 700, 1024])
def test_lone_trap_workgroup_shapes_parity(torch_gpu, oracle_mod, prec, n):
    """A single trap stepped inside one workgroup, in every workgroup size and
    targets-per-thread count it accepts: forces against the oracle, then (FP64)
    a 30-step run against the oracle's steps."""
    w = li.random_cloud(n, seed=900 + n, sigma=30e-6, light_fraction=0.2)
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    ref = (oracle_mod.step(w.state(), w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, 30)
           if prec == "fp64" else None)
    for block in (256, 512, 1024):
        for tpt in (1, 2, 4):
            if block == 1024 and tpt == 4:
                continue
            sim = _sim(w, prec, oracle_mod, small_trap=2, batch_block=block, batch_tpt=tpt)
            assert sim.config()["batch_block"] == block
            assert _m1(sim.compute_accel(), r, sc) <= TOL[prec], (block, tpt)
            if ref is not None:
                sim.step(30, spec.dt)
                st, _ = sim.get_state()
                disp = np.max(np.abs(ref["x"] - w.x)) + 1e-12
                for c in ("x", "y", "z"):
                    assert np.max(np.abs(st[c] - ref[c])) < 1e-10 * disp, (block, tpt, c)
            sim.close()


def test_batch_equals_single_trap_path(torch_gpu, oracle_mod):
    """One trap run through the batched kernel and through the single-trap
    kernels gives the same trajectory (FP64, to roundoff)."""
    w = li.random_cloud(333, seed=31, sigma=30e-6)
    from paper_1907_10514_amd import Simulation

    tr = _oracle_trap(oracle_mod, w.traps[0])
    out = []
    for npt in (None, [333]):
        sim = Simulation(w.mass, w.charge, "fp64", n_per_trap=npt)
        sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)
        sim.set_damping(1e5)
        sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.0)
        sim.step(120, li.DT)
        out.append(sim.get_state()[0])
        sim.close()
    # two FP64 paths of different summation order: within max(1e-12 x extent,
    # 10x the oracle's divergence under a one-ulp start shift) over 120 steps
    ext = np.max(np.abs(w.x))
    err = tb.divergence(out[0], out[1], tb.X)
    bar = 1e-12 * ext
    if err >= bar:
        env, _ = tb.ulp_envelope(
            lambda st: oracle_mod.step(st, w.charge, w.mass, tr, 1e5, 0.0, li.DT, 120), w.state())
        print(f"batched vs single-trap kernels: 120-step |dx| {err:.3e}, ulp envelope {env:.3e}")
        bar = max(bar, 10 * env)
    assert err < bar


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
@pytest.mark.parametrize("n", [1, 8, 100, 128, 160, 300])
def test_small_trap_path_equals_multi_workgroup_path(torch_gpu, oracle_mod, n, prec, tol):
    """A single trap stepped inside one workgroup (many steps per launch) and by
    the multi-workgroup kernels gives the same trajectory to rounding, with a
    beam, a bath and the velocity time average switched on; force evaluations
    after the run see the updated positions in both paths."""
    w = li.random_cloud(n, seed=600 + n, sigma=20e-6 * max(1, n / 8) ** (1 / 3),
                        light_fraction=0.3)
    sp = (w.mass < 30 * li.AMU).astype(np.int32)
    out = []
    for small in (1, 2):
        sim = _sim(w, prec, oracle_mod, small_trap=small, chunk_steps=40)
        assert sim.config()["small_trap"] == small
        sim.set_species(sp)
        sim.set_beam(0, (0.3, 0.2, 1.0), 2e5, species=0)
        sim.set_bath(0, 1e-3, 50e-6, 11, species=1)
        sim.set_time_average(20)
        sim.step(150, w.traps[0].dt)
        st, t = sim.get_state()
        avg, end = sim.time_average()
        out.append((st, t, avg, end, np.array(sim.compute_accel())))
        sim.close()
    (a, ta, va, ea, fa), (b, tb, vb, eb, fb) = out
    assert ta == tb and ea == eb == 140
    ext = max(np.max(np.abs(w.x)), 1e-6)
    for k in ("x", "y", "z"):
        assert np.max(np.abs(a[k] - b[k])) < tol * 1e3 * ext, k
    vs = max(np.max(np.abs(a["vx"])), 1e-3)
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(a[k] - b[k])) < tol * 1e3 * vs, k
    assert np.max(np.abs(fa - fb)) <= tol * 1e3 * np.max(np.abs(fa))


SMALL_SIZES = [1, 2, 3, 8, 31, 32, 33, 63, 64, 65, 100, 128, 129, 160]


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("charges", ["common", "mixed"])
def test_small_trap_accel_parity(torch_gpu, oracle_mod, prec, charges):
    """A single trap stepped inside one workgroup evaluates its forces with that
    kernel (lone trap: one target per thread, sources split over the parts);
    at every size up to the default limit the force meets the bar."""
    for n in SMALL_SIZES:
        q = None if charges == "common" else np.random.default_rng(n).choice([1, 2, -1], n)
        w = li.random_cloud(n, seed=900 + n, sigma=20e-6 * max(1, n / 8) ** (1 / 3),
                            light_fraction=0.3, charge_e=q)
        sim = _sim(w, prec, oracle_mod, small_trap=2)
        assert sim.config()["small_trap"] == 2
        tr = _oracle_trap(oracle_mod, w.traps[0])
        r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
        sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
        err = _m1(sim.compute_accel(), r, sc)
        assert err <= TOL[prec], (n, err)
        sim.close()


@pytest.mark.parametrize("prec", ["mixed", "mixed_kahan"])
@pytest.mark.parametrize("n", [8, 64, 100, 160])
def test_small_trap_fp32_run_matches_oracle(torch_gpu, oracle_mod, n, prec):
    """The one-workgroup stepping path (the default for <= 128 ions) in the FP32
    modes over 200 steps: at steps 0, 100 and 190 the run is re-anchored and
    its next SEGMENT steps are compared with the oracle's run from the GPU's
    state, ion by ion within 10x the envelope of the oracle's own segment under
    per-step kicks of dt M1 A_i, M1 measured on that kernel's force there."""
    w = li.random_cloud(n, seed=800 + n, sigma=20e-6 * max(1, n / 8) ** (1 / 3),
                        light_fraction=0.3)
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    sim = _sim(w, prec, oracle_mod, small_trap=2)
    assert sim.config()["small_trap"] == 2
    anchors = (0, 100, 190)
    states, done = {0: (w.state(), 0.0, sim.compute_accel())}, 0
    for k in (10, 100, 110, 190, 200):
        sim.step(k - done, spec.dt)
        done = k
        st, t = sim.get_state()
        states[k] = (st, t, sim.compute_accel() if k in anchors else None)
    for k0 in anchors:
        s0, t0, a0 = states[k0]
        ra = oracle_mod.accel(s0["x"], s0["y"], s0["z"], w.charge, w.mass, tr, t0)
        sc = oracle_mod.accel_scale(s0["x"], s0["y"], s0["z"], w.charge, w.mass, tr, t0)
        m1 = tb.m1(a0, ra, sc)
        ref = oracle_mod.step(s0, w.charge, w.mass, tr, spec.gamma, t0, spec.dt, tb.SEGMENT)
        kicked = tb.kicked_run(
            lambda st, k: oracle_mod.step(st, w.charge, w.mass, tr, spec.gamma, t0 + k * spec.dt,
                                          spec.dt, 1),
            tb.nudge(s0), tb.SEGMENT, tb.kick(sc, max(m1, tb.M1_FLOOR), spec.dt))
        got = states[k0 + tb.SEGMENT][0]
        rx, rv = tb.ratio(got, ref, kicked, tb.X), tb.ratio(got, ref, kicked, tb.V)
        print(f"n={n} {prec} from step {k0}: M1 {m1:.2e}, |dx| {rx:.2f} bars, |dv| {rv:.2f} bars")
        assert m1 <= min(TOL[prec], tb.M1_REF), (k0, m1)
        assert rx <= 1 and rv <= 1, (k0, rx, rv)
    sim.close()


def test_crystal8_full_run_matches_oracle_on_both_paths(torch_gpu, oracle_mod):
    w = li.crystal8()
    spec = w.traps[0]
    ref = oracle_mod.step(w.state(), w.charge, w.mass, _oracle_trap(oracle_mod, spec),
                          spec.gamma, 0.0, spec.dt, w.nsteps)
    ext = np.max(np.abs(ref["z"]))
    for small in (1, 2):
        sim = _sim(w, "fp64", oracle_mod, small_trap=small)
        sim.step(w.nsteps, spec.dt)
        st, t = sim.get_state()
        assert t == ref["t"]
        for k in ("x", "y", "z"):
            assert np.max(np.abs(st[k] - ref[k])) < 1e-9 * ext, (small, k)
        sim.close()


def test_error_paths_on_gpu(torch_gpu, oracle_mod):
    from paper_1907_10514_amd import LionError, Simulation
    from paper_1907_10514_amd import lion as L

    sim = Simulation([li.REF_MASS] * 4, [li.E_CHARGE] * 4, "fp64")
    with pytest.raises(LionError) as ei:
        sim.step(10, li.DT)
    assert ei.value.code == L.LION_ERR_STATE
    with pytest.raises(LionError) as ei:
        sim.set_trap(1.0, 0.0, 0.1, 1e-3, 1e-3, 0.25)  # rf without frequency
    assert ei.value.code == L.LION_ERR_ARG
    with pytest.raises(LionError) as ei:
        sim.set_state([0, 0, 0, math.nan], [0] * 4, [0] * 4, [0] * 4, [0] * 4, [0] * 4)
    assert ei.value.code == L.LION_ERR_ARG
    sim.set_state([1e-5, -1e-5, 0, 2e-5], [0] * 4, [0] * 4, [0] * 4, [0] * 4, [0] * 4)
    with pytest.raises(LionError) as ei:
        sim.step(-1, li.DT)
    assert ei.value.code == L.LION_ERR_ARG
    with pytest.raises(LionError) as ei:
        sim.step(1, 0.0)
    assert ei.value.code == L.LION_ERR_ARG
    sim.step(0, li.DT)  # no-op
    assert sim.check_finite() == L.LION_OK
    # a finite but absurd position overflows the trap field: reported, not hidden
    sim.set_trap(9.0, li.OMEGA, 0.24, li.R0, li.Z0, li.KAPPA)
    sim.set_state([1e300, 0, 0, 0], [0] * 4, [0, 0, 1e-5, -1e-5], [0] * 4, [0] * 4, [0] * 4)
    sim.step(2, li.DT)
    assert sim.check_finite() == L.LION_ERR_NONFINITE
    sim.close()


# ------------------------------------------------------------ rigid bodies

def _body_cloud(n, seed, contiguous=True):
    rng = np.random.default_rng(seed)
    w = li.random_cloud(n, seed=seed, sigma=40e-6, light_fraction=0.2)
    body = np.full(n, -1, dtype=np.int32)
    if contiguous:
        for b, start in enumerate(range(0, n // 2, 37)):
            body[start:start + 20] = b
    else:
        body[rng.permutation(n)[: n // 3]] = rng.integers(0, 7, n // 3)
    return w, body


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("contiguous", [True, False])
def test_body_exclusion_parity(torch_gpu, oracle_mod, prec, contiguous):
    """Pairs inside a rigid body are left out, for bodies laid out in runs of
    consecutive ions (fast path) and scattered (per-pair test everywhere)."""
    w, body = _body_cloud(1500, 41 if contiguous else 43, contiguous)
    tr = _oracle_trap(oracle_mod, w.traps[0])
    rx, ry, rz, sc = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, body, tr, 0.0)
    sim = _sim(w, prec, oracle_mod)
    sim.set_bodies(body)
    cfgs = [dict()] + [dict(i_per_lane=i, j_split=j, lds_sources=l, symmetric=1)
                       for i in (1, 4) for j in (1, 7) for l in (1, 2)]
    if prec != "mixed_kahan":
        cfgs.append(dict(symmetric=2))  # pair-once kernels with the per-pair body test
    for cfg in cfgs:
        if cfg:
            sim.set_config(**cfg)
        err = _m1(sim.compute_accel(), (rx, ry, rz), sc)
        assert err <= TOL[prec], (cfg, err)
    # clearing the mask restores the all-pairs field
    sim.set_bodies(None)
    r2 = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc2 = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    assert _m1(sim.compute_accel(), r2, sc2) <= TOL[prec]
    sim.close()


def _tile_body_cloud(n, seed, charge_e=None):
    """Cloud whose bodies fill whole 256-ion tiles: body 0 = tile 0, body 1 =
    tiles 1-2, body 2 = tile 3; the rest free (last tile ragged)."""
    w = li.random_cloud(n, seed=seed, sigma=40e-6, light_fraction=0.2, charge_e=charge_e)
    body = np.full(n, -1, dtype=np.int32)
    body[:256] = 0
    body[256:768] = 1
    body[768:1024] = 2
    return w, body


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("charges", ["uniform", "mixed"])
def test_pair_once_tile_aligned_bodies(torch_gpu, oracle_mod, prec, charges):
    """Bodies that fill whole 256-ion tiles on the pair-once kernels: tile pairs
    inside one body are skipped, everything else is evaluated once; the field
    meets the bar against the oracle and the all-pairs kernels with the mask."""
    q = None if charges == "uniform" else np.random.default_rng(3).choice([1, 2, -1], 3000)
    w, body = _tile_body_cloud(3000, 51, q)
    tr = _oracle_trap(oracle_mod, w.traps[0])
    rx, ry, rz, sc = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, body, tr, 0.0)
    sym = _sim(w, prec, oracle_mod, symmetric=2)
    sym.set_bodies(body)
    assert sym.config()["symmetric"] == 2
    a = sym.compute_accel()
    err = _m1(a, (rx, ry, rz), sc)
    allp = _sim(w, prec, oracle_mod, symmetric=1)
    allp.set_bodies(body)
    err_all = _m1(a, allp.compute_accel(), sc)
    print(f"tile bodies {prec} {charges}: M1={err:.3e} vs masked all-pairs {err_all:.3e}")
    assert err <= TOL[prec]
    assert err_all <= 2 * TOL[prec]
    sym.close()
    allp.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_pair_once_bodies_sharing_tiles(torch_gpu, oracle_mod, prec):
    """13000 ions (pair-once by default) with clusters that straddle tile
    edges: tile pairs inside one body are skipped, pairs of tiles whose bodies
    may meet take the per-pair test, the rest the plain loop.  Sampled
    targets against the oracle, the field against the masked all-pairs
    kernels, and (FP64) 20 rigid steps against them."""
    n = 13000
    w = li.random_cloud(n, seed=57, sigma=200e-6, light_fraction=0.2)
    body = np.full(n, -1, dtype=np.int32)
    for k, start in enumerate(range(100, 100 + 12 * 600, 600)):
        body[start:start + 512] = k  # 512-ion clusters starting off tile edges
    body[9000:9040] = 99             # a small body inside one tile
    tr = _oracle_trap(oracle_mod, w.traps[0])
    sym = _sim(w, prec, oracle_mod)
    sym.set_bodies(body)
    assert sym.config()["symmetric"] == 2
    a = sym.compute_accel()
    idx = np.concatenate([np.arange(95, 105), np.arange(600, 620), np.arange(9000, 9040),
                          np.random.default_rng(8).choice(n, 128, replace=False)])
    rx, ry, rz, sc = oracle_mod.accel_bodies_at(w.x, w.y, w.z, w.charge, w.mass, body, tr, 0.0,
                                                idx)
    err = _m1((a[0][idx], a[1][idx], a[2][idx]), (rx, ry, rz), sc)
    allp = _sim(w, prec, oracle_mod, symmetric=1)
    allp.set_bodies(body)
    b = allp.compute_accel()
    scale = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, body, tr, 0.0)[3]
    err_all = _m1(a, b, scale)
    print(f"bodies sharing tiles {prec}: M1={err:.3e} vs masked all-pairs {err_all:.3e}")
    assert err <= TOL[prec]
    assert err_all <= 2 * TOL[prec]
    if prec == "fp64":  # rigid stepping on both kernels agrees to round-off
        outs = []
        for s2 in (sym, allp):
            s2.set_rigid_bodies(body)
            s2.step(20, w.traps[0].dt)
            outs.append(s2.get_state()[0])
        ext = np.max(np.abs(w.x))
        for k in ("x", "y", "z"):
            assert np.max(np.abs(outs[0][k] - outs[1][k])) < 1e-11 * ext, k
    sym.close()
    allp.close()


def test_pair_once_rigid_steps(torch_gpu, oracle_mod):
    """Rigid integration over the pair-once kernels (tile-aligned bodies)
    follows the masked all-pairs run to round-off over 30 FP64 steps."""
    w, body = _tile_body_cloud(1600, 53)
    dt = w.traps[0].dt
    outs = []
    for sym in (2, 1):
        sim = _sim(w, "fp64", oracle_mod, symmetric=sym)
        sim.set_rigid_bodies(body)
        sim.step(30, dt)
        outs.append(sim.get_state()[0])
        sim.close()
    ext = np.max(np.abs(w.x))
    for k in ("x", "y", "z"):
        assert np.max(np.abs(outs[0][k] - outs[1][k])) < 1e-11 * ext, k


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("n", [40000, 100000])
def test_pair_once_above_32768(torch_gpu, oracle_mod, prec, n):
    """Pair-once kernels at 40000 and 100000 ions (157 and 391 tiles, one
    partial per tile): sampled targets against the oracle, and 5 steps against
    all-pairs."""
    w = li.random_cloud(n, seed=55, sigma=200e-6, light_fraction=0.2)
    tr = _oracle_trap(oracle_mod, w.traps[0])
    sim = _sim(w, prec, oracle_mod, symmetric=2)
    assert sim.config()["symmetric"] == 2
    a = sim.compute_accel()
    idx = np.random.default_rng(6).choice(w.n, 256, replace=False)
    rx, ry, rz, sc = oracle_mod.accel_at(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0, idx)
    err = _m1((a[0][idx], a[1][idx], a[2][idx]), (rx, ry, rz), sc)
    print(f"pair-once N={n} {prec} sampled M1={err:.3e}")
    assert err <= TOL[prec]
    outs = []
    for s2 in (sim, _sim(w, prec, oracle_mod, symmetric=1)):
        s2.step(5, w.traps[0].dt)
        outs.append(s2.get_state()[0])
        s2.close()
    ext = np.max(np.abs(w.x))
    tol = 1e-12 if prec == "fp64" else 1e-6
    for k in ("x", "y", "z"):
        assert np.max(np.abs(outs[0][k] - outs[1][k])) < tol * ext


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pair_once_at_maximum_size(torch_gpu, oracle_mod, prec):
    """131072 ions (512 tiles, the most the pair-once kernels take) run them by
    default and meet the bar on sampled targets; one ion more falls back to
    the all-pairs kernels, meets the bar too, and refuses the pair-once ones."""
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    for n, sym in ((131072, 2), (131073, 1)):
        w = li.random_cloud(n, seed=59, sigma=300e-6, light_fraction=0.2)
        tr = _oracle_trap(oracle_mod, w.traps[0])
        sim = _sim(w, prec, oracle_mod)
        assert sim.config()["symmetric"] == sym, n
        a = sim.compute_accel()
        idx = np.concatenate([[0, n - 1], np.random.default_rng(7).choice(n, 126, replace=False)])
        rx, ry, rz, sc = oracle_mod.accel_at(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0, idx)
        err = _m1((a[0][idx], a[1][idx], a[2][idx]), (rx, ry, rz), sc)
        print(f"N={n} {prec} symmetric={sym} sampled M1={err:.3e}")
        assert err <= TOL[prec], n
        if sym == 1:
            with pytest.raises(LionError) as ei:
                sim.set_config(symmetric=2)
            assert ei.value.code == L.LION_ERR_UNSUPPORTED
        sim.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("sym", [1, 2])
def test_clusters65536_sampled(torch_gpu, oracle_mod, prec, sym):
    """64 rigid clusters of 512 + 32768 free ions (65536): sampled targets in
    clusters and free, every source counted, intra-cluster pairs left out, on
    the all-pairs kernels (mask) and on the pair-once kernels (whole tile
    pairs skipped)."""
    w = li.clusters65536()
    body = w.notes["body"]
    tr = _oracle_trap(oracle_mod, w.traps[0])
    sim = _sim(w, prec, oracle_mod, symmetric=sym)
    sim.set_bodies(body)
    assert sim.config()["symmetric"] == sym
    a = sim.compute_accel()
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(32768, 96, replace=False),
                          32768 + rng.choice(32768, 96, replace=False)])
    rx, ry, rz, sc = oracle_mod.accel_bodies_at(w.x, w.y, w.z, w.charge, w.mass, body, tr, 0.0,
                                                idx)
    err = _m1((a[0][idx], a[1][idx], a[2][idx]), (rx, ry, rz), sc)
    print(f"clusters65536 {prec} sampled M1={err:.3e} config={sim.config()}")
    assert err <= TOL[prec]
    sim.step(3, w.traps[0].dt)
    assert sim.check_finite() == 0
    sim.close()


def test_bodies_rejected_where_unsupported(torch_gpu, oracle_mod):
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    w = li.random_cloud(300, seed=2)
    shared = np.full(300, -1, dtype=np.int32)
    shared[:100] = 0  # body 0 shares the first 256-ion tile with free ions
    sim = _sim(w, "mixed", oracle_mod, symmetric=2)
    sim.set_bodies(shared)  # per-pair test inside the pair-once kernels
    assert sim.config()["symmetric"] == 2
    sim.set_bodies(np.zeros(300, dtype=np.int32))  # whole tiles: tile pairs skipped
    assert sim.config()["symmetric"] == 2
    sim.set_config(symmetric=1)
    with pytest.raises(LionError) as ei:
        sim.set_bodies(np.full(300, -2, dtype=np.int32))
    assert ei.value.code == L.LION_ERR_ARG
    sim.close()
    k = _sim(w, "mixed_kahan", oracle_mod)
    k.set_bodies(shared)
    k.set_config(symmetric=2)  # the compensated mode has the per-pair test too
    assert k.config()["symmetric"] == 2
    k.close()
    b = _small_batch(n_traps=3, seed=5, n_max=20)
    bs = _sim(b, "fp64", oracle_mod)
    with pytest.raises(LionError) as ei:
        bs.set_bodies(np.zeros(b.n, dtype=np.int32))
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    bs.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch512_full_size_sampled(torch_gpu, oracle_mod, prec):
    """The full 512-trap batch (130408 ions) in the benchmarked launch shape:
    forces and a 20-step run of 12 sampled traps (including the largest)
    against the oracle."""
    from paper_1907_10514_amd import runner

    w = li.batch512(nsteps=0)
    sim = runner.simulation_for(w, precision=prec)
    a = sim.compute_accel()
    sizes = np.diff(w.offsets)
    rng = np.random.default_rng(7)
    pick = sorted(set([int(np.argmax(sizes))] + list(rng.choice(w.n_traps, 11, replace=False))))
    traps = [_oracle_trap(oracle_mod, s) for s in w.traps]
    for k in pick:
        o, e = int(w.offsets[k]), int(w.offsets[k + 1])
        r = oracle_mod.accel(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e], w.mass[o:e], traps[k],
                             0.0)
        sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e], w.mass[o:e],
                                    traps[k], 0.0)
        assert _m1([c[o:e] for c in a], r, sc) <= TOL[prec], k
    dts = np.array([s.dt for s in w.traps])
    sim.step(20, dts)
    st, _ = sim.get_state()
    for k in pick:
        o, e = int(w.offsets[k]), int(w.offsets[k + 1])
        sub = {c: v[o:e] for c, v in w.state().items()}
        ref = oracle_mod.step(sub, w.charge[o:e], w.mass[o:e], traps[k], w.traps[k].gamma, 0.0,
                              dts[k], 20)
        disp = np.max(np.abs(ref["x"] - sub["x"])) + 1e-12
        tol = 1e-9 if prec == "fp64" else 1e-4
        for c in ("x", "y", "z"):
            assert np.max(np.abs(st[c][o:e] - ref[c])) < tol * disp, (k, c)
    sim.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_mixed16384_full_size_steps(torch_gpu, oracle_mod, prec, tol):
    """Ten steps of the full 16384-ion cloud in the benchmarked launch shape
    against the oracle, every ion compared."""
    from paper_1907_10514_amd import runner

    w = li.mixed16384()
    spec = w.traps[0]
    sim = runner.simulation_for(w, precision=prec)
    sim.step(10, spec.dt)
    st, _ = sim.get_state()
    ref = oracle_mod.step(w.state(), w.charge, w.mass, _oracle_trap(oracle_mod, spec), spec.gamma,
                          0.0, spec.dt, 10)
    disp = np.max(np.abs(ref["x"] - w.x))
    err = max(np.max(np.abs(st[k] - ref[k])) for k in ("x", "y", "z"))
    print(f"{prec}: max |dx| {err:.2e} after 10 steps (displacement {disp:.2e}), "
          f"config {sim.config()}")
    assert err < tol * disp
    sim.close()
