#!/usr/bin/env python3
"""Writes crystal1024_observables.json: the oracle's label-free observables of
the 1024-ion cooling run (the paper's "Coulomb crystal of a single species"
example at scale, with the viscous cooling of section "Verifications /
Cooling mechanisms"): kinetic temperature every 1000 steps and the final
energy per ion, for the run from the seeded start state and for TWINS runs
perturbed the way an FP64 force path perturbs it.

A twin starts from the state moved by one ulp (random signs) and, after every
oracle step, gets the velocity kick dt M1 A_i xi_i: A_i the sum of the
magnitudes of every contribution to ion i's acceleration (refreshed every
1000 steps), xi_i a seeded unit vector fixed for the twin, M1 = M1_FP64, the
largest relative force error the FP64 GPU path shows against the oracle.  A
start shift alone is not that model: the cloud is damped, so a start shift
decays, while a force path's rounding enters at every step.  The twins
measure how much the observables of the chaotic cooling move under such
perturbations; the GPU test allows its own run to lie within a multiple of
that spread.  Calls only the oracle and the seeded input generator.
Usage: python tests/golden/make_crystal1024_observables.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lion_inputs as li  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "crystal1024_observables.json")
EVERY = 1000
TWINS = 16
M1_FP64 = 4.2e-16  # largest FP64 force error (M1) of the GPU path in its accuracy tests


def kinetic_temperature(st, mass):
    """(2/3) <E_kin> / k_B over the ions (K), velocities as sampled."""
    v2 = st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2
    return float(np.sum(0.5 * mass * v2) / (1.5 * mass.size * li.K_B))


def run(w, tr, state):
    spec = w.traps[0]
    temps = [kinetic_temperature(state, w.mass)]
    st, t = dict(state), 0.0
    for _ in range(w.nsteps // EVERY):
        st = oracle.step(st, w.charge, w.mass, tr, spec.gamma, t, spec.dt, EVERY)
        t = st["t"]
        temps.append(kinetic_temperature(st, w.mass))
    kin, coul, dc = oracle.energy(st, w.charge, w.mass, tr)
    return dict(temperature_K=temps, energy_per_ion_J=dict(kinetic=kin / w.n, coulomb=coul / w.n,
                                                            dc_trap=dc / w.n), t_end=t)


def nudged(state, seed):
    rng = np.random.default_rng(seed)
    out = {}
    for k, v in state.items():
        out[k] = np.nextafter(v, np.where(rng.random(v.shape) < 0.5, -np.inf, np.inf))
    return out


def run_kicked(w, tr, seed):
    """The run of a twin: one-ulp start shift, then after every step the
    velocity kick dt M1_FP64 A_i xi_i (xi_i fixed for the twin)."""
    spec = w.traps[0]
    st = nudged(w.state(), seed)
    xi = np.random.default_rng(1000 + seed).normal(size=(3, w.n))
    xi /= np.linalg.norm(xi, axis=0)
    temps = [kinetic_temperature(st, w.mass)]
    t = 0.0
    for _ in range(w.nsteps // EVERY):
        sc = oracle.accel_scale(st["x"], st["y"], st["z"], w.charge, w.mass, tr, t)
        dv = spec.dt * M1_FP64 * sc * xi
        for _ in range(EVERY):
            st = oracle.step(st, w.charge, w.mass, tr, spec.gamma, t, spec.dt, 1)
            t = st["t"]
            st["vx"] = st["vx"] + dv[0]
            st["vy"] = st["vy"] + dv[1]
            st["vz"] = st["vz"] + dv[2]
        temps.append(kinetic_temperature(st, w.mass))
    kin, coul, dc = oracle.energy(st, w.charge, w.mass, tr)
    return dict(temperature_K=temps, energy_per_ion_J=dict(kinetic=kin / w.n, coulomb=coul / w.n,
                                                            dc_trap=dc / w.n), t_end=t)


def main():
    oracle.build(force=False)
    w = li.crystal1024()
    spec = w.traps[0]
    V0, U0 = oracle.voltages_for(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                 spec.r0, spec.z0, spec.kappa)
    tr = oracle.Trap(V0=V0, Omega=spec.omega, U0=U0, R0=spec.r0, Z0=spec.z0, kappa=spec.kappa)
    t0 = time.time()
    base = run(w, tr, w.state())
    print(f"oracle run: {time.time() - t0:.1f} s", flush=True)
    twins = []
    for s in range(1, TWINS + 1):
        twins.append(run_kicked(w, tr, s))
        print(f"twin {s} done", flush=True)
    data = dict(
        about="Oracle observables of the crystal1024 cooling run (1024 Ca-40, q=0.2, "
              "a=-0.001, sigma 100 um, 10 mK, gamma 2e5/s, dt = T_rf/20, 50000 steps, "
              "FP64); kinetic temperature (2/3)<E_kin>/k_B at steps 0, 1000, ..., 50000 "
              "(every 50 rf periods, the same rf phase); energies per ion at the end. "
              "twins: the same run from the start state moved by one ulp (random signs) "
              "with the velocity kick dt M1 A_i xi_i after every step (M1 = %.1e, A_i the "
              "sum of the magnitudes of ion i's acceleration terms, xi_i a fixed seeded unit "
              "vector; seeds 1..%d). Written by make_crystal1024_observables.py."
              % (M1_FP64, TWINS),
        every=EVERY, nsteps=w.nsteps, base=base, twins=twins)
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1)
    print(OUT)


if __name__ == "__main__":
    main()
