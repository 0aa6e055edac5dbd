"""Accuracy figures of the GPU path on the 16384-ion workloads.

* Force errors along a run: the mixed-species 16384-ion cloud is advanced with
  the FP64 GPU path and, at steps 0, 1000 and 2000, every precision's forces
  are compared with the oracle on 1024 sampled targets: M1 (max error over the
  contribution scale), M2 (Frobenius norm ratio) and M3 (50th/99th/100th
  percentiles of the per-ion relative error).
* Secular drift of the FP32 pair path: the centre of mass of a one-species
  16384-ion cloud obeys the one-ion equation of motion exactly (the pair forces
  cancel), so any error of the pair sum that does not cancel shows up as a
  departure from the one-ion trajectory.  Reported: the FFT peak of the radial
  COM motion over 10^4 steps (with its bin width) and the largest departure from
  the one-ion oracle run, turned into a bound on the relative frequency error.
"""
from __future__ import annotations

import numpy as np
import pytest

import lion_inputs as li

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


def _sim(w, prec, oracle):
    from paper_1907_10514_amd import Simulation

    sim = Simulation(w.mass, w.charge, prec)
    tr = _oracle_trap(oracle, w.traps[0])
    sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)
    sim.set_damping(w.traps[0].gamma)
    sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.0)
    return sim


def test_force_errors_along_headline_run(torch_gpu, oracle_mod):
    w = li.mixed16384()
    tr = _oracle_trap(oracle_mod, w.traps[0])
    dt = w.traps[0].dt
    run = _sim(w, "fp64", oracle_mod)
    sims = {p: _sim(w, p, oracle_mod) for p in TOL}
    idx = np.sort(np.random.default_rng(17).choice(w.n, 1024, replace=False))
    rows = []
    for step in (0, 1000, 2000):
        if step:
            run.step(1000, dt)
        st, t = run.get_state()
        rx, ry, rz, sc = oracle_mod.accel_at(st["x"], st["y"], st["z"], w.charge, w.mass, tr, t,
                                             idx)
        ref = np.stack([rx, ry, rz])
        for p, sim in sims.items():
            sim.set_state(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], t)
            a = np.stack([c[idx] for c in sim.compute_accel()])
            d = np.linalg.norm(a - ref, axis=0)
            m1 = float(np.max(d / sc))
            m2 = float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
            rel = d / np.linalg.norm(ref, axis=0)
            m3 = np.percentile(rel, [50, 99, 100])
            rows.append((step, p, m1, m2, m3))
            print(f"step {step:5d} {p:12s} M1 {m1:.2e}  M2 {m2:.2e}  "
                  f"M3 p50 {m3[0]:.2e} p99 {m3[1]:.2e} max {m3[2]:.2e}")
    for step, p, m1, _, _ in rows:
        assert m1 <= TOL[p], (step, p, m1)
    for s in [run, *sims.values()]:
        s.close()


def _fft_peak(samples, dt_sample):
    s = samples - np.mean(samples)
    spec = np.abs(np.fft.rfft(s * np.hanning(s.size)))
    f = np.fft.rfftfreq(s.size, dt_sample)
    k = int(np.argmax(spec[1:]) + 1)
    return f[k], f[1] - f[0]


def test_secular_drift_of_fp32_pair_path(torch_gpu, oracle_mod):
    """One species (16384 Ca-40, sigma 200 um, 10 mK, q = 0.25, undamped so the
    line is not broadened), 10^4 steps, COM sampled every 5 steps."""
    w = li.single_trap("single16384", 16384, 200e-6, 10e-3, 2, 0.25, -0.001, 0.0, 10000)
    spec = w.traps[0]
    tr = _oracle_trap(oracle_mod, spec)
    every, samples = 5, 2000
    com0 = {k: np.array([np.mean(getattr(w, k))]) for k in ("x", "y", "z", "vx", "vy", "vz")}
    one = dict(com0)
    ref = np.empty((samples, 3))
    t = 0.0
    for s in range(samples):
        one = oracle_mod.step(one, [li.E_CHARGE], [li.REF_MASS], tr, 0.0, t, spec.dt, every)
        t = one["t"]
        ref[s] = one["x"][0], one["y"][0], one["z"][0]
    amp = np.max(np.abs(ref), axis=0)
    f_ref, bin_w = _fft_peak(ref[:, 0], every * spec.dt)
    omega_x = 2 * np.pi * f_ref
    t_total = samples * every * spec.dt
    for prec in ("fp64", "mixed", "mixed_kahan"):
        sim = _sim(w, prec, oracle_mod)
        com = np.empty((samples, 3))
        for s in range(samples):
            sim.step(every, spec.dt)
            st, _ = sim.get_state()
            com[s] = np.mean(st["x"]), np.mean(st["y"]), np.mean(st["z"])
        sim.close()
        f_p, _ = _fft_peak(com[:, 0], every * spec.dt)
        dev = np.max(np.abs(com - ref), axis=0) / amp
        # a relative frequency error e makes the phase slip by e * omega * t
        bound = float(dev[0] / (omega_x * t_total))
        print(f"{prec:12s} radial COM peak {f_p / 1e3:.3f} kHz (one ion {f_ref / 1e3:.3f} kHz, "
              f"bin {bin_w / 1e3:.3f} kHz); max |COM - one ion| / amplitude "
              f"x {dev[0]:.2e} y {dev[1]:.2e} z {dev[2]:.2e}; |df/f| <= {bound:.1e}")
        assert f_p == f_ref, prec
        if prec == "fp64":
            assert np.all(dev < 1e-6), dev
