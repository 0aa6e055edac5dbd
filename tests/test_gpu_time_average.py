"""Velocity time averages (timeAvg) of the GPU path against the oracle.

The oracle's reference is its own trajectory stepped one step at a time (the
velocity after every step), averaged by oracle.time_average.  A binary time step
(2^-26 s) makes t_start + k dt exact, so stepping one step at a time and many
steps per call see identical times on both sides.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import lion_inputs as li

pytestmark = pytest.mark.gpu

DT = 2.0 ** -26
TOL = {"fp64": 1e-10, "mixed": 1e-5, "mixed_kahan": 1e-5}


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


def _sim(w, prec, oracle):
    from paper_1907_10514_amd import Simulation

    batched = w.n_traps > 1
    sim = Simulation(w.mass, w.charge, prec, n_per_trap=np.diff(w.offsets) if batched else None)
    for k, spec in enumerate(w.traps):
        tr = _oracle_trap(oracle, spec)
        sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa, trap=k if batched else -1)
        sim.set_damping(spec.gamma, trap=k if batched else -1)
    sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.0)
    return sim


def _oracle_samples(oracle, w, k, nsteps):
    """Velocities after each of nsteps steps of trap k, one step per call."""
    o, e = int(w.offsets[k]), int(w.offsets[k + 1])
    st = {c: v[o:e].copy() for c, v in w.state().items()}
    tr = _oracle_trap(oracle, w.traps[k])
    out, t = [], 0.0
    for _ in range(nsteps):
        st = oracle.step(st, w.charge[o:e], w.mass[o:e], tr, w.traps[k].gamma, t, DT, 1)
        t = st["t"]
        out.append(np.stack([st["vx"], st["vy"], st["vz"]]))
    return np.array(out)  # [nsteps, 3, n_k]


def _check(oracle, avg, end, ref_samples, origin, window, tol):
    s = ref_samples.reshape(ref_samples.shape[0], -1)
    ends, means = oracle.time_average(s, 1, origin, window)
    assert end == ends[-1], (end, ends)
    ref = means[-1].reshape(3, -1)
    scale = np.max(np.abs(ref_samples))
    err = max(np.max(np.abs(a - r)) for a, r in zip(avg, ref))
    assert err < tol * scale, (err, scale)
    return err / scale


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_time_average_single_trap(torch_gpu, oracle_mod, prec):
    """W = 20 (one rf period at this step) from step 0, stepped in calls of 17
    and 28 steps (windows close at 20 and 40); then restarted at step 45 with
    W = 7 and stepped 20 more (windows close at 52 and 59)."""
    w = li.random_cloud(300, seed=61, sigma=100e-6, light_fraction=0.3)
    ref = _oracle_samples(oracle_mod, w, 0, 65)
    sim = _sim(w, prec, oracle_mod)
    sim.set_time_average(20)
    sim.step(17, DT)
    sim.step(28, DT)
    (vx, vy, vz), end = sim.time_average()
    e1 = _check(oracle_mod, (vx, vy, vz), end, ref[:45], 0, 20, TOL[prec])
    sim.set_time_average(7)
    sim.step(20, DT)
    (vx, vy, vz), end = sim.time_average()
    assert end == 59
    e2 = _check(oracle_mod, (vx, vy, vz), end, ref, 45, 7, TOL[prec])
    print(f"{prec}: relative error of the averages {e1:.2e}, {e2:.2e}")
    sim.close()


@pytest.mark.parametrize("n_max", [200, 32, 16])
@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_time_average_batch(torch_gpu, oracle_mod, prec, n_max):
    """Window means of batched traps against the oracle: traps of up to 200
    ions (the batched kernel) and of up to 32 and 16 (the wave kernel)."""
    w = li.batch512(n_traps=10, n_min=2, n_max=n_max, seed=29, nsteps=0)
    sim = _sim(w, prec, oracle_mod)
    sim.set_time_average(10)
    sim.step(35, DT)
    (vx, vy, vz), end = sim.time_average()
    assert end == 30
    for k in range(w.n_traps):
        o, e = int(w.offsets[k]), int(w.offsets[k + 1])
        ref = _oracle_samples(oracle_mod, w, k, 35)
        _check(oracle_mod, (vx[o:e], vy[o:e], vz[o:e]), end, ref, 0, 10, TOL[prec])
    sim.close()


def test_time_average_of_damped_free_ions_closed_form(torch_gpu, oracle_mod):
    """Free ions under damping: window means follow the geometric sum exactly."""
    from paper_1907_10514_amd import Simulation

    n, gamma, W = 64, 1e6, 20
    rng = np.random.default_rng(8)
    v0 = rng.normal(0, 1.0, (3, n))
    z = np.zeros(n)
    for npt in (None, [32, 32]):
        sim = Simulation(np.full(n, li.REF_MASS), z, "fp64", n_per_trap=npt)
        sim.set_damping(gamma)
        sim.set_state(z, z, z, v0[0], v0[1], v0[2], 0.0)
        sim.set_time_average(W)
        sim.step(50, li.DT)
        avg, end = sim.time_average()
        assert end == 40
        r = math.exp(-gamma * li.DT)
        a = end - W + 1
        geo = r ** a * (1 - r ** W) / (1 - r) / W
        for c in range(3):
            assert np.allclose(avg[c], v0[c] * geo, rtol=1e-12, atol=0)
        sim.close()


def test_time_average_states(torch_gpu, oracle_mod):
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    w = li.random_cloud(50, seed=3)
    sim = _sim(w, "fp64", oracle_mod)
    with pytest.raises(LionError) as ei:
        sim.time_average()  # off
    assert ei.value.code == L.LION_ERR_STATE
    with pytest.raises(LionError) as ei:
        sim.set_time_average(-1)
    assert ei.value.code == L.LION_ERR_ARG
    sim.set_time_average(10)
    sim.step(9, DT)
    with pytest.raises(LionError) as ei:
        sim.time_average()  # no window closed yet
    assert ei.value.code == L.LION_ERR_STATE
    sim.step(1, DT)
    _, end = sim.time_average()
    assert end == 10
    sim.close()
