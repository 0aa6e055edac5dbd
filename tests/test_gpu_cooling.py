"""Cooling beams and Langevin baths on the GPU against the oracle.

Both sides draw the bath kicks from Philox4x32-10 with the same counter
(ion, run-wide step, bath and half-step) and key (seed), each from its own
implementation; the Box-Muller transcendental functions may differ in the last
bit between the device and host math libraries, so trajectories agree to
roundoff growth, not bit for bit.  Beams involve no random numbers and match
the oracle to the last few bits.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import lion_inputs as li
from tests import trajectory_bar as tb

pytestmark = pytest.mark.gpu


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


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


BEAMS = [dict(k=_unit([1.0, 1.0, 1.0]), gamma=3e5, species=0),
         dict(k=_unit([0.2, -0.5, 1.0]), gamma=1e5, species=1)]
BATHS = [dict(temperature=0.5e-3, tau=40e-6, seed=0x1234_5678_9ABC, species=1),
         dict(temperature=2e-3, tau=80e-6, seed=99, species=-1)]


def _species(w):
    return (w.mass < 30 * li.AMU).astype(np.int32)


def _cooled_sim(w, prec, oracle, species, beams=BEAMS, baths=BATHS, **cfg):
    from paper_1907_10514_amd import Simulation

    batched = w.n_traps > 1
    sim = Simulation(w.mass, w.charge, prec, n_per_trap=np.diff(w.offsets) if batched else None)
    if cfg:
        sim.set_config(**cfg)
    for k, spec in enumerate(w.traps):
        tr = _oracle_trap(oracle, spec)
        sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa, trap=k if batched else -1)
        sim.set_damping(spec.gamma, trap=k if batched else -1)
    sim.set_species(species)
    for b, B in enumerate(beams):
        sim.set_beam(b, B["k"], B["gamma"], species=B["species"])
    for c, T in enumerate(baths):
        sim.set_bath(c, T["temperature"], T["tau"], T["seed"], species=T["species"])
    sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.0)
    return sim


def _segment_ratios(oracle, w, sp, tr, spec, k0, a_gpu, s0, t0, got, ion_base=0):
    """Per-ion bar ratios (x, v) of the GPU's SEGMENT steps from the state s0 it
    reached after k0 steps (its force there a_gpu) against the oracle run from
    s0, with bars from the oracle's run under kicks of the measured M1."""
    oracle_accel = oracle.accel(s0["x"], s0["y"], s0["z"], w["charge"], w["mass"], tr, t0)
    sc = oracle.accel_scale(s0["x"], s0["y"], s0["z"], w["charge"], w["mass"], tr, t0)
    m1 = tb.m1(a_gpu, oracle_accel, sc)

    def one(st, k):
        return oracle.step_cooled(st, w["charge"], w["mass"], sp, tr, spec.gamma, beams=BEAMS,
                                  baths=BATHS, step_base=k0 + k, t_start=t0 + k * spec.dt,
                                  dt=spec.dt, nsteps=1, ion_base=ion_base)

    ref = oracle.step_cooled(s0, w["charge"], w["mass"], sp, tr, spec.gamma, beams=BEAMS,
                             baths=BATHS, step_base=k0, t_start=t0, dt=spec.dt,
                             nsteps=tb.SEGMENT, ion_base=ion_base)
    kicked = tb.kicked_run(one, tb.nudge(s0), tb.SEGMENT,
                           tb.kick(sc, max(m1, tb.M1_FLOOR), spec.dt))
    return m1, tb.ratio(got, ref, kicked, tb.X), tb.ratio(got, ref, kicked, tb.V)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("launches", [1, 2])
def test_cooled_run_matches_oracle(torch_gpu, oracle_mod, prec, launches):
    """Two species, a beam on each and two baths (one species-selective), run in
    four calls (10 + 110 + 10 + 70 steps), each continuing the draw sequence.
    The cloud is chaotic, so the GPU is compared in two re-anchored segments:
    its steps 1-10 and 121-130 (the first steps of a call) against the oracle
    started from the state the GPU reached, ion by ion within 10x the
    envelope of the oracle's own segment under per-step velocity kicks of
    dt M1 A_i (M1 the GPU's measured force error there).  The CPU controls show
    that a wrong draw, species or rate moves such a segment by >= 10 bars.
    FP64 also matches the whole 200-step run within 10x the one-ulp envelope.
    Both the one-launch step and the pair kernel + epilogue are run."""
    w = li.random_cloud(700, seed=41, sigma=200e-6, light_fraction=0.3)
    wd = dict(charge=w.charge, mass=w.mass)
    sp = _species(w)
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    sim = _cooled_sim(w, prec, oracle_mod, sp, step_launches=launches)
    assert sim.config()["step_launches"] == launches
    states = {0: (w.state(), 0.0, sim.compute_accel())}
    for k, n in ((10, 10), (120, 110), (130, 10), (200, 70)):
        sim.step(n, spec.dt)
        st, t = sim.get_state()
        states[k] = (st, t, sim.compute_accel() if k == 120 else None)
    assert sim.step_index() == 200
    for k0 in (0, 120):
        s0, t0, a0 = states[k0]
        m1, rx, rv = _segment_ratios(oracle_mod, wd, sp, tr, spec, k0, a0, s0, t0,
                                     states[k0 + tb.SEGMENT][0])
        print(f"{prec}: segment from step {k0}: M1 {m1:.2e}, |dx| {rx:.2f} bars, "
              f"|dv| {rv:.2f} bars")
        if prec != "fp64":
            assert m1 <= tb.M1_REF, (k0, m1)
        assert rx <= 1 and rv <= 1, (k0, rx, rv)
    st = states[200][0]
    ref = oracle_mod.step_cooled(w.state(), w.charge, w.mass, sp, tr, spec.gamma, beams=BEAMS,
                                 baths=BATHS, dt=spec.dt, nsteps=120)
    ref = oracle_mod.step_cooled(ref, w.charge, w.mass, sp, tr, spec.gamma, beams=BEAMS,
                                 baths=BATHS, step_base=120, t_start=ref["t"], dt=spec.dt,
                                 nsteps=80)
    if prec == "fp64":
        disp = np.max(np.abs(ref["x"] - w.x))
        env_x, env_v = tb.ulp_envelope(
            lambda s0: oracle_mod.step_cooled(s0, w.charge, w.mass, sp, tr, spec.gamma,
                                              beams=BEAMS, baths=BATHS, dt=spec.dt, nsteps=200),
            w.state())
        err = tb.divergence(st, ref, tb.X)
        verr = tb.divergence(st, ref, tb.V)
        print(f"fp64 200 steps: |dx| {err:.3e} (disp {disp:.3e}, ulp envelope {env_x:.3e}), "
              f"|dv| {verr:.3e} (envelope {env_v:.3e})")
        assert err < max(1e-10 * disp, 10 * env_x)
        assert verr < max(1e-9 * np.max(np.abs(ref["vx"])), 10 * env_v)
    # the baths did act: without them the run differs far beyond the tolerance
    vscale = np.max(np.abs(ref["vx"]))
    plain = oracle_mod.step_cooled(w.state(), w.charge, w.mass, sp, tr, spec.gamma, beams=BEAMS,
                                   dt=spec.dt, nsteps=200)
    assert np.max(np.abs(plain["vx"] - ref["vx"])) > 0.01 * vscale
    sim.close()


def test_beam_cooling_of_free_ions_is_exact(torch_gpu, oracle_mod):
    """Neutral ions with no trap field: along the beam the velocity decays as
    exp(-gamma t), across it nothing changes, and ions of the other species are
    untouched (bit for bit)."""
    from paper_1907_10514_amd import Simulation

    rng = np.random.default_rng(3)
    n = 96
    k = _unit(rng.normal(size=3))
    v = rng.normal(0, 2.0, (3, n))
    sp = (np.arange(n) % 3 == 0).astype(np.int32)
    m = np.full(n, li.REF_MASS)
    for prec in ("fp64", "mixed", "mixed_kahan"):
        sim = Simulation(m, np.zeros(n), prec)
        sim.set_species(sp)
        sim.set_beam(2, k * 7.0, 1e6, species=0)  # normalised by the library
        sim.set_state(np.zeros(n), np.zeros(n), np.zeros(n), v[0], v[1], v[2], 0.0)
        sim.step(800, li.DT)
        st, _ = sim.get_state()
        vout = np.stack([st["vx"], st["vy"], st["vz"]])
        decay = math.exp(-1e6 * 800 * li.DT)
        for i in range(n):
            par_in, par_out = k @ v[:, i], k @ vout[:, i]
            if sp[i] == 0:
                # every half-step rounds each velocity component to ~u |v|;
                # on the decayed parallel part these add up like a random walk
                # over the 1600 half-steps (~40 u |v|): bound 10x that
                assert par_out == pytest.approx(par_in * decay, rel=1e-11,
                                                abs=1e-13 * np.max(np.abs(v[:, i]))), (prec, i)
                perp = (vout[:, i] - par_out * k) - (v[:, i] - par_in * k)
                assert np.max(np.abs(perp)) < 1e-14 * np.max(np.abs(v[:, i]))
            else:
                assert np.array_equal(vout[:, i], v[:, i]), (prec, i)
        sim.close()


@pytest.mark.parametrize("n_max", [300, 32, 16])
@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_cooled_batch_matches_oracle(torch_gpu, oracle_mod, prec, n_max):
    """Batched traps draw bath kicks by run-wide ion index (trap k's first ion is
    offsets[k]).  Every trap's steps 51-60 (re-anchored at the state the GPU
    reached after 50 steps) match the oracle run with that ion_base within the
    per-ion segment bars at the measured M1 of that trap; in FP64 every trap's
    whole 100-step run also matches within max(1e-10 x displacement, 10x the
    one-ulp envelope).  Traps of up to 300 ions run in the batched kernel, traps
    of up to 32 in the wave kernel (on 256 threads, or one wave up to 16)."""
    w = li.batch512(n_traps=12, n_min=2, n_max=n_max, seed=23, nsteps=0)
    rng = np.random.default_rng(4)
    sp = rng.integers(0, 2, w.n).astype(np.int32)
    sim = _cooled_sim(w, prec, oracle_mod, sp, chunk_steps=30)
    dt = w.traps[0].dt
    sim.step(50, dt)
    s50, t50 = sim.get_state()
    a50 = sim.compute_accel()
    sim.step(tb.SEGMENT, dt)
    s60, _ = sim.get_state()
    sim.step(100 - 50 - tb.SEGMENT, dt)
    st, _ = sim.get_state()
    for k, spec in enumerate(w.traps):
        o, e = int(w.offsets[k]), int(w.offsets[k + 1])
        tr = _oracle_trap(oracle_mod, spec)
        wd = dict(charge=w.charge[o:e], mass=w.mass[o:e])
        sub0 = {c: v[o:e] for c, v in s50.items()}
        got = {c: v[o:e] for c, v in s60.items()}
        m1, rx, rv = _segment_ratios(oracle_mod, wd, sp[o:e], tr, spec, 50,
                                     [c[o:e] for c in a50], sub0, t50, got, ion_base=o)
        if prec != "fp64":
            assert m1 <= tb.M1_REF, (k, m1)
        assert rx <= 1 and rv <= 1, (k, e - o, m1, rx, rv)
        if prec == "fp64":
            sub = {c: v[o:e] for c, v in w.state().items()}

            def run(s0):
                return oracle_mod.step_cooled(s0, w.charge[o:e], w.mass[o:e], sp[o:e], tr,
                                              spec.gamma, beams=BEAMS, baths=BATHS, dt=dt,
                                              nsteps=100, ion_base=o)

            ref = run(sub)
            disp = np.max(np.abs(ref["x"] - sub["x"])) + 1e-12
            err = max(np.max(np.abs(st[c][o:e] - ref[c])) for c in tb.X)
            if err >= 1e-10 * disp:
                env_x, _ = tb.ulp_envelope(run, sub)
                assert err < 10 * env_x, (k, err, disp, env_x)
    sim.close()


def test_cooled_batch_rejects_unequal_steps(torch_gpu, oracle_mod):
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    w = li.batch512(n_traps=4, n_min=2, n_max=50, seed=5, nsteps=0)
    sim = _cooled_sim(w, "fp64", oracle_mod, np.zeros(w.n, dtype=np.int32))
    dts = np.array([s.dt for s in w.traps]) * np.array([1.0, 1.1, 1.0, 1.0])
    with pytest.raises(LionError) as ei:
        sim.step(5, dts)
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    sim.set_bath(0, 0.0, 0.0, 0)
    sim.set_bath(1, 0.0, 0.0, 0)
    sim.set_beam(0, (1, 0, 0), 0.0)
    sim.set_beam(1, (1, 0, 0), 0.0)
    sim.step(5, dts)  # no cooling left: per-trap steps are fine again
    sim.close()


def test_cooled_runs_reproducible_and_resumable(torch_gpu, oracle_mod):
    """Counter-based draws: reruns, graph vs plain launches and chunk sizes give
    identical bits, and a run resumed in a fresh handle with set_step_index
    continues the same draw sequence bit for bit (binary time step)."""
    w = li.random_cloud(1500, seed=12, sigma=60e-6, light_fraction=0.3)
    sp = _species(w)
    dt = 2.0 ** -26
    outs = []
    base = dict(i_per_lane=2, j_split=16, flush_len=8)  # one launch shape throughout
    for cfg in (base, dict(base, use_graph=2), dict(base, chunk_steps=7)):
        sim = _cooled_sim(w, "mixed", oracle_mod, sp, **cfg)
        sim.step(45, dt)
        outs.append(sim.get_state()[0])
        sim.close()
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k
    a = _cooled_sim(w, "fp64", oracle_mod, sp)
    a.step(100, dt)
    sa, ta = a.get_state()
    b = _cooled_sim(w, "fp64", oracle_mod, sp)
    b.step(60, dt)
    sb, tb = b.get_state()
    c = _cooled_sim(w, "fp64", oracle_mod, sp)
    c.set_state(sb["x"], sb["y"], sb["z"], sb["vx"], sb["vy"], sb["vz"], tb)
    c.set_step_index(b.step_index())
    c.step(40, dt)
    sc, tc = c.get_state()
    assert tc == ta and c.step_index() == 100
    for k in sa:
        assert np.array_equal(sa[k], sc[k]), k
    for s in (a, b, c):
        s.close()


def test_langevin_bath_thermalises_on_gpu(torch_gpu, oracle_mod):
    """Free neutral ions in one bath reach k_B T = M <v_x^2> (three axes, 4096
    ions, after 10 relaxation times), in the batched kernel too."""
    from paper_1907_10514_amd import Simulation

    n, T, tau, dt = 4096, 1e-3, 2e-6, 1e-7
    m = np.full(n, li.REF_MASS)
    z = np.zeros(n)
    for npt in (None, [1024] * 4):
        sim = Simulation(m, z, "fp64", n_per_trap=npt)
        sim.set_bath(3, T, tau, 2024)
        sim.set_state(z, z, z, z, z, z, 0.0)
        sim.step(200, dt)
        st, _ = sim.get_state()
        v2 = np.stack([st["vx"], st["vy"], st["vz"]]) ** 2
        temp = li.REF_MASS * v2.mean() / li.K_B
        assert abs(temp - T) < 4 * T * math.sqrt(2 / (3 * n)), temp
        sim.close()
