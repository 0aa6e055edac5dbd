"""Rigid bodies on the GPU against the oracle (oracle.step_rigid).

Both sides set the bodies up independently from the same ion state (the GPU
library with its own Jacobi eigen-solver, the oracle with numpy's eigh); the
integration scheme depends only on the space-frame inertia tensor, so the two
agree to rounding growth whatever principal axes each picks.
"""
from __future__ import annotations

import numpy as np
import pytest

import lion_inputs as li
from tests import trajectory_bar as tb

pytestmark = pytest.mark.gpu

CA = li.REF_MASS


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _trap(oracle, q_x=0.3, a_x=-0.001):
    V0, U0 = oracle.voltages_for(q_x, a_x, CA, li.E_CHARGE, li.OMEGA, li.R0, li.Z0, li.KAPPA)
    return oracle.Trap(V0=V0, Omega=li.OMEGA, U0=U0, R0=li.R0, Z0=li.Z0, kappa=li.KAPPA)


def _rod(n=9, spacing=2.5e-6):
    z = (np.arange(n) - (n - 1) / 2) * spacing
    return np.zeros(n), np.zeros(n), z


def _rod_and_cloud(n_free=30, seed=2, sigma=100e-6):
    """The paper's charged-rod example: 9 ions 2.5 um apart on the z axis among
    a cloud of free Ca-40 ions."""
    rng = np.random.default_rng(seed)
    rx, ry, rz = _rod()
    st = dict(x=np.concatenate([rng.normal(0, sigma, n_free), rx]),
              y=np.concatenate([rng.normal(0, sigma, n_free), ry]),
              z=np.concatenate([rng.normal(0, sigma, n_free), rz]))
    n = st["x"].size
    v = rng.normal(0, 1.0, (3, n))
    st.update(vx=v[0], vy=v[1], vz=v[2])
    body = np.concatenate([np.full(n_free, -1), np.zeros(9)]).astype(np.int32)
    return st, np.full(n, CA), np.full(n, li.E_CHARGE), body


def _clusters(n_bodies=8, per=20, n_free=100, seed=4, sigma=120e-6, radius=4e-6):
    rng = np.random.default_rng(seed)
    centres = rng.normal(0, sigma, (n_bodies, 3))
    d = rng.normal(size=(n_bodies, per, 3))
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    r = radius * rng.uniform(0, 1, (n_bodies, per, 1)) ** (1 / 3)
    pos = np.concatenate([(centres[:, None] + d * r).reshape(-1, 3),
                          rng.normal(0, sigma, (n_free, 3))])
    n = pos.shape[0]
    v = rng.normal(0, 1.0, (n, 3))
    st = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), vx=v[:, 0].copy(),
              vy=v[:, 1].copy(), vz=v[:, 2].copy())
    body = np.concatenate([np.repeat(np.arange(n_bodies), per) * 3 + 5,
                           np.full(n_free, -1)]).astype(np.int32)
    perm = rng.permutation(n)  # members need not be consecutive
    st = {k: v[perm] for k, v in st.items()}
    return st, np.full(n, CA), np.full(n, li.E_CHARGE), body[perm]


def _gpu(st, m, q, body, prec, trap, gamma, **cfg):
    from paper_1907_10514_amd import Simulation

    sim = Simulation(m, q, prec)
    if cfg:
        sim.set_config(**cfg)
    if trap is not None:
        sim.set_trap(trap.V0, trap.Omega, trap.U0, trap.R0, trap.Z0, trap.kappa)
    sim.set_damping(gamma)
    sim.set_state(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], 0.0)
    sim.set_rigid_bodies(body)
    return sim


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
@pytest.mark.parametrize("case", ["rod", "clusters"])
def test_rigid_run_matches_oracle(torch_gpu, oracle_mod, case, prec):
    """300 steps in three calls (170 + 10 + 120), rf trap and damping.  These
    clouds amplify small perturbations about 4000-fold over 300 steps, so the
    GPU's steps 171-180 are compared, re-anchored at the state it reached after
    170 steps (its ions, and its body state carried into the oracle's body
    frame), with the oracle's run from there: ion by ion within 10x the envelope of the oracle's own segment under
    per-step kicks of dt M1 A_i (M1 the GPU's measured force error at step 170;
    members are kicked through their body).  The CPU controls show that one
    changed body id moves such a segment by far more than 10 bars.  FP64 also
    matches the whole run within max(1e-10 x displacement, 10x the one-ulp
    envelope)."""
    st, m, q, body = _rod_and_cloud() if case == "rod" else _clusters()
    tr = _trap(oracle_mod)
    sim = _gpu(st, m, q, body, prec, tr, 1e5)
    quat0 = sim.rigid_state()["quaternion"]
    sim.step(170, li.DT)
    s0, t0 = sim.get_state()
    rg0 = tb.rigid_anchor(oracle_mod, oracle_mod.rigid_setup(st, m, body), quat0,
                          sim.rigid_state())
    a0 = sim.compute_accel()
    sim.step(tb.SEGMENT, li.DT)
    seg, _ = sim.get_state()
    sim.step(300 - 170 - tb.SEGMENT, li.DT)
    got, _ = sim.get_state()
    ox, oy, oz, sc = oracle_mod.accel_bodies(s0["x"], s0["y"], s0["z"], q, m, body, tr, t0)
    m1 = tb.m1(a0, (ox, oy, oz), sc)
    ref, apply, one, init = tb.rigid_segment(oracle_mod, s0, rg0, q, m, body, tr, 1e5, t0,
                                             li.DT)
    kicked = tb.kicked_run(one, init, tb.SEGMENT, tb.kick(sc, max(m1, tb.M1_FLOOR), li.DT),
                           apply)
    rx, rv = tb.ratio(seg, ref, kicked, tb.X), tb.ratio(seg, ref, kicked, tb.V)
    print(f"{case} {prec}: segment 171-180: M1 {m1:.2e}, |dx| {rx:.2f} bars, |dv| {rv:.2f} bars")
    if prec != "fp64":
        assert m1 <= tb.M1_REF
    assert rx <= 1 and rv <= 1
    if prec == "fp64":
        a, rg = oracle_mod.step_rigid(st, q, m, body, tr, 1e5, 0.0, li.DT, 170)
        full, _ = oracle_mod.step_rigid(a, q, m, body, tr, 1e5, a["t"], li.DT, 130, rigid=rg)
        disp = np.max(np.abs(full["x"] - st["x"]))
        err = tb.divergence(got, full, tb.X)
        bar = 1e-10 * disp
        if err >= bar:
            env, _ = tb.ulp_envelope(
                lambda s: oracle_mod.step_rigid(s, q, m, body, tr, 1e5, 0.0, li.DT, 300)[0], st)
            bar = max(bar, 10 * env)
        print(f"{case} fp64 300 steps: max |dx| {err:.3e} m (bar {bar:.3e} m)")
        assert err < bar
    sim.close()


def test_rigid_body_com_follows_single_ion_on_gpu(torch_gpu, oracle_mod):
    """Kohn for a lone rod (all members the same Q/M): its centre of mass
    follows the one-ion oracle trajectory to rounding."""
    st, m, q, body = _rod_and_cloud(n_free=0, seed=5)
    for k, off in (("x", 7e-6), ("y", -4e-6), ("z", 11e-6)):
        st[k] = st[k] + off
    tr = _trap(oracle_mod)
    for prec in ("fp64", "mixed", "mixed_kahan"):
        sim = _gpu(st, m, q, body, prec, tr, 1e5)
        sim.step(2000, li.DT)
        rs = sim.rigid_state()
        setup = oracle_mod.rigid_setup(st, m, body)
        one = {k: setup[a][0, c:c + 1].copy() for k, a, c in
               (("x", "R", 0), ("y", "R", 1), ("z", "R", 2), ("vx", "V", 0), ("vy", "V", 1),
                ("vz", "V", 2))}
        ref = oracle_mod.step(one, [li.E_CHARGE], [CA], tr, 1e5, 0.0, li.DT, 2000)
        for c, k in enumerate("xyz"):
            assert abs(rs["com"][0, c] - ref[k][0]) < 1e-10 * 11e-6, (prec, k)
        sim.close()


def test_rigid_explosion_conserves_momenta_on_gpu(torch_gpu, oracle_mod):
    """No trap, no damping: total momentum and angular momentum (orbital +
    spin) of bodies and free ions stay fixed to rounding."""
    st, m, q, body = _clusters(n_bodies=4, per=12, n_free=40, seed=9, sigma=15e-6, radius=3e-6)
    sim = _gpu(st, m, q, body, "fp64", None, 0.0)
    free = body < 0

    def invariants():
        s, _ = sim.get_state()
        rs = sim.rigid_state()
        r = np.stack([s["x"], s["y"], s["z"]], 1)
        v = np.stack([s["vx"], s["vy"], s["vz"]], 1)
        M = np.array([m[body == b].sum() for b in np.unique(body[body >= 0])])
        P = (m[free, None] * v[free]).sum(0) + (M[:, None] * rs["com_velocity"]).sum(0)
        J = (m[free, None] * np.cross(r[free], v[free])).sum(0) + \
            (M[:, None] * np.cross(rs["com"], rs["com_velocity"])).sum(0) + \
            rs["angular_momentum"].sum(0)
        return P, J, np.sum(m[:, None] * np.abs(v)), \
            np.sum(m * np.linalg.norm(r, axis=1) * np.linalg.norm(v, axis=1))

    P0, J0, _, _ = invariants()
    sim.step(400, 2e-9)
    P1, J1, ps, js = invariants()
    assert np.max(np.abs(P1 - P0)) < 1e-13 * ps
    assert np.max(np.abs(J1 - J0)) < 1e-12 * js
    sim.close()


def test_rigid_rod_spin_on_gpu(torch_gpu, oracle_mod):
    """Torque-free rod spinning about x: equals the oracle's run to rounding
    and the exact uniform rotation to the scheme's O(dt^2)."""
    omega0 = 2e5
    x, y, z = _rod()
    n = x.size
    v = np.cross([omega0, 0, 0], np.stack([x, y, z], 1))
    st = dict(x=x, y=y, z=z, vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())
    m, q, body = np.full(n, CA), np.zeros(n), np.zeros(n, dtype=np.int32)
    dt = 1.0 / omega0 / 200
    sim = _gpu(st, m, q, body, "fp64", None, 0.0)
    sim.step(200, dt)
    got, _ = sim.get_state()
    ref, _ = oracle_mod.step_rigid(st, q, m, body, oracle_mod.Trap(), 0.0, 0.0, dt, 200)
    ext = np.max(np.abs(z))
    for k in ("x", "y", "z"):
        assert np.max(np.abs(got[k] - ref[k])) < 1e-13 * ext, k
    assert np.max(np.abs(got["y"] + np.sin(1.0) * z)) < 1e-5 * ext
    sim.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_rigid_clusters65536_full_size(torch_gpu, oracle_mod, prec):
    """The 65536-ion cluster workload (64 rigid clusters of 512 ions + 32768 free
    ions) integrated with rigid bodies in the benchmarked launch shape: members
    keep their distances, everything stays finite, and two runs agree bit for
    bit."""
    from paper_1907_10514_amd import runner

    w = li.clusters65536()
    body = w.notes["body"]
    outs = []
    for _ in range(2):
        sim = runner.simulation_for(w, precision=prec)
        sim.set_rigid_bodies(body)
        sim.step(20, w.traps[0].dt)
        assert sim.check_finite() == 0
        outs.append(sim.get_state()[0])
        sim.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k
    for b in (0, 17, 63):
        idx = np.nonzero(body == b)[0][:64]
        r0 = np.stack([w.x[idx], w.y[idx], w.z[idx]], 1)
        r1 = np.stack([outs[0][k][idx] for k in ("x", "y", "z")], 1)
        d0 = np.linalg.norm(r0[:, None] - r0[None], axis=2)
        d1 = np.linalg.norm(r1[:, None] - r1[None], axis=2)
        assert np.max(np.abs(d1 - d0)) < 1e-12 * np.max(d0), b


def test_rigid_set_state_and_switches(torch_gpu, oracle_mod):
    from paper_1907_10514_amd import LionError, Simulation
    from paper_1907_10514_amd import lion as L

    st, m, q, body = _rod_and_cloud(n_free=10)
    sim = Simulation(m, q, "fp64")
    with pytest.raises(LionError) as ei:
        sim.set_rigid_bodies(body)  # no state yet
    assert ei.value.code == L.LION_ERR_STATE
    sim.set_state(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], 0.0)
    sim.set_rigid_bodies(body)
    assert sim.rigid_state()["com"].shape == (1, 3)
    # set_state re-runs the body set-up: a shifted state moves the COM
    sim.set_state(st["x"] + 1e-6, st["y"], st["z"], st["vx"], st["vy"], st["vz"], 0.0)
    assert sim.rigid_state()["com"][0, 0] == pytest.approx(1e-6, rel=1e-9, abs=0)
    sim.set_rigid_bodies(None)
    assert sim.rigid_state()["com"].shape == (0, 3)
    sim.step(3, li.DT)
    sim.close()
    bat = Simulation(np.full(4, CA), np.full(4, li.E_CHARGE), "fp64", n_per_trap=[2, 2])
    with pytest.raises(LionError) as ei:
        bat.set_rigid_bodies([0, 0, -1, -1])
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    bat.close()
