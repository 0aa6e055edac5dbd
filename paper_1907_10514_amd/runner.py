"""Set up a Simulation from a workload description (ions, traps in Mathieu
coefficients, damping, dt) using only the library's own calls."""
from __future__ import annotations

import numpy as np

from .lion import Simulation, lion_mathieu_to_voltages


def trap_voltages(spec):
    """(V0, U0) of one trap spec (q_x, a_x for its reference ion) via the
    library's eq. (Mathieuaq) helper."""
    return lion_mathieu_to_voltages(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge,
                                    spec.omega, spec.r0, spec.z0, spec.kappa)


def simulation_for(w, precision=None, batched=None, stream=None) -> Simulation:
    """Simulation of workload ``w`` with traps, damping and state applied."""
    prec = precision or ("fp64" if w.precision == "fp64" else "mixed")
    batched = w.n_traps > 1 if batched is None else batched
    npt = np.diff(w.offsets) if batched else None
    sim = Simulation(w.mass, w.charge, prec, n_per_trap=npt, stream=stream)
    for k, spec in enumerate(w.traps):
        V0, U0 = trap_voltages(spec)
        sim.set_trap(V0, spec.omega, U0, spec.r0, spec.z0, spec.kappa, trap=k if batched else -1)
        sim.set_damping(spec.gamma, trap=k if batched else -1)
    sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.0)
    return sim


def step_dts(w):
    return np.array([spec.dt for spec in w.traps])
