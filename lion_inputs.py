"""Seeded synthetic ion clouds and trap settings.

This module only draws inputs: positions, velocities, masses, charges and the
trap parameters of each workload, all from seeded numpy PCG64 generators.  It
holds none of the method's arithmetic (no fields, forces or steps), so both the
oracle and the GPU library can be fed from it.

Workloads follow the paper's examples ("Examples": ion clouds created at random
in a trap, a mixed-species cloud for sympathetic cooling) with the sizes used
for measurement:

* ``crystal8``       8 Ca-40 ions, q=0.3, a=-0.001, sigma 20 um, 10 mK, gamma 1e5/s
* ``crystal1024``    1024 Ca-40 ions, q=0.2, sigma 100 um, 10 mK, gamma 2e5/s
* ``mixed16384``     16384 ions, 80 % Ca-40 and 20 % mass-17 singly charged ions placed
                     at random, q=0.25 (for Ca-40), sigma 200 um, 10 mK per species
* ``batch512``       512 independent traps of N ~ U{2..512}, q ~ U[0.1, 0.6],
                     a ~ U[-0.01, 0] (Mathieu-stable draws only), otherwise as crystal8
* ``clusters65536``  64 rigid clusters of 512 Ca-40 ions (uniform in 5 um balls about
                     Gaussian centres, sigma 400 um) + 32768 free Ca-40 ions, q=0.3

Trap settings are given as Mathieu coefficients (q_x, a_x) for the reference ion
(40 u, +e); each side converts them to voltages with its own implementation of
eq. (Mathieuaq).  Positions are Gaussian per Cartesian axis about the trap
centre, velocities Maxwell-Boltzmann per axis with sigma_v = sqrt(k_B T / M).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

E_CHARGE = 1.602176634e-19  # C
AMU = 1.66053906660e-27  # kg
K_B = 1.380649e-23  # J/K

# Shared trap geometry of every workload.
RF_HZ = 3.85e6
OMEGA = 2.0 * math.pi * RF_HZ
R0 = 0.5e-3
Z0 = 1.0e-3
KAPPA = 0.25
T_RF = 1.0 / RF_HZ
DT = T_RF / 20.0
REF_MASS = 40.0 * AMU
REF_CHARGE = E_CHARGE


@dataclass
class TrapSpec:
    """One trap: Mathieu (q_x, a_x) for the reference ion, geometry, damping, dt."""
    q_x: float
    a_x: float
    omega: float = OMEGA
    r0: float = R0
    z0: float = Z0
    kappa: float = KAPPA
    gamma: float = 0.0
    dt: float = DT
    ref_mass: float = REF_MASS
    ref_charge: float = REF_CHARGE


@dataclass
class Workload:
    name: str
    mass: np.ndarray
    charge: np.ndarray
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    traps: list  # list[TrapSpec], one per trap
    offsets: np.ndarray  # trap k owns ions [offsets[k], offsets[k+1])
    nsteps: int
    precision: str
    notes: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.size)

    @property
    def n_traps(self) -> int:
        return len(self.traps)

    def state(self) -> dict:
        return {k: getattr(self, k).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}

    def ordered_pairs(self) -> int:
        n = np.diff(self.offsets)
        return int(np.sum(n * (n - 1)))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_cloud(rng: np.random.Generator, n: int, sigma: float):
    pos = rng.normal(0.0, sigma, size=(3, n))
    return pos[0].copy(), pos[1].copy(), pos[2].copy()


def thermal_velocities(rng: np.random.Generator, mass: np.ndarray, temperature: float):
    s = np.sqrt(K_B * temperature / mass)
    v = rng.normal(0.0, 1.0, size=(3, mass.size)) * s
    return v[0].copy(), v[1].copy(), v[2].copy()


def single_trap(name: str, n: int, sigma: float, temperature: float, seed: int, q_x: float,
                a_x: float, gamma: float, nsteps: int, precision: str = "fp64",
                light_fraction: float = 0.0, light_mass_u: float = 17.0) -> Workload:
    """One cloud in one trap.  With light_fraction > 0, exactly round(f n) ions
    (chosen by a seeded permutation) get mass light_mass_u and charge +e."""
    rng = _rng(seed)
    mass = np.full(n, REF_MASS)
    charge = np.full(n, REF_CHARGE)
    n_light = int(round(light_fraction * n))
    if n_light:
        idx = rng.permutation(n)[:n_light]
        mass[idx] = light_mass_u * AMU
    x, y, z = gaussian_cloud(rng, n, sigma)
    vx, vy, vz = thermal_velocities(rng, mass, temperature)
    trap = TrapSpec(q_x=q_x, a_x=a_x, gamma=gamma)
    return Workload(name, mass, charge, x, y, z, vx, vy, vz, [trap],
                    np.array([0, n], dtype=np.int64), nsteps, precision,
                    notes=dict(sigma=sigma, temperature=temperature, seed=seed,
                               n_light=n_light))


def crystal8() -> Workload:
    return single_trap("crystal8", 8, 20e-6, 10e-3, 0, 0.3, -0.001, 1e5, 20000)


def crystal1024() -> Workload:
    return single_trap("crystal1024", 1024, 100e-6, 10e-3, 1, 0.2, -0.001, 2e5, 50000)


def mixed16384(n: int = 16384, seed: int = 2) -> Workload:
    return single_trap("mixed16384", n, 200e-6, 10e-3, seed, 0.25, -0.001, 1e5, 10000,
                       precision="mixed", light_fraction=0.2)


def stable_draw(q: float, a: float) -> bool:
    """Input filter for swept traps: keep draws inside the first Mathieu stability
    region with margin (a + q^2/2 >= 4e-4, i.e. a secular frequency of at least
    ~1 % of Omega) and with axial confinement (a_x <= -1e-4)."""
    return a <= -1e-4 and a + 0.5 * q * q >= 4e-4


def batch512(n_traps: int = 512, n_min: int = 2, n_max: int = 512, seed: int = 3,
             nsteps: int = 20000) -> Workload:
    """Independent traps of uneven size and swept (q, a), concatenated in trap order."""
    rng = _rng(seed)
    sizes = rng.integers(n_min, n_max + 1, size=n_traps)
    traps, rejected = [], []
    for _ in range(n_traps):
        while True:
            q = rng.uniform(0.1, 0.6)
            a = rng.uniform(-0.01, 0.0)
            if stable_draw(q, a):
                break
            rejected.append((q, a))
        traps.append(TrapSpec(q_x=q, a_x=a, gamma=1e5))
    offsets = np.zeros(n_traps + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    n = int(offsets[-1])
    mass = np.full(n, REF_MASS)
    charge = np.full(n, REF_CHARGE)
    x, y, z = gaussian_cloud(rng, n, 20e-6)
    vx, vy, vz = thermal_velocities(rng, mass, 10e-3)
    return Workload("batch512", mass, charge, x, y, z, vx, vy, vz, traps, offsets, nsteps,
                    "mixed", notes=dict(seed=seed, rejected=rejected, sizes=sizes))


def clusters65536(n_clusters: int = 64, per_cluster: int = 512, n_free: int = 32768,
                  seed: int = 4, cluster_radius: float = 5e-6, sigma: float = 400e-6) -> Workload:
    """Rigid clusters of Ca-40 ions, each uniform in a ball of radius 5 um about a
    Gaussian (sigma 400 um) centre, plus free Ca-40 ions (sigma 400 um); q = 0.3,
    a = -0.001, 10 mK.  Cluster ions come first, each cluster's ions consecutive;
    notes["body"] holds the body id of every ion (-1 = free)."""
    rng = _rng(seed)
    centres = rng.normal(0.0, sigma, size=(n_clusters, 3))
    d = rng.normal(size=(n_clusters, per_cluster, 3))
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    r = cluster_radius * rng.uniform(0.0, 1.0, size=(n_clusters, per_cluster, 1)) ** (1.0 / 3.0)
    pos_c = (centres[:, None, :] + d * r).reshape(-1, 3)
    pos_f = rng.normal(0.0, sigma, size=(n_free, 3))
    pos = np.concatenate([pos_c, pos_f])
    n = pos.shape[0]
    mass = np.full(n, REF_MASS)
    charge = np.full(n, REF_CHARGE)
    vx, vy, vz = thermal_velocities(rng, mass, 10e-3)
    body = np.concatenate([np.repeat(np.arange(n_clusters, dtype=np.int32), per_cluster),
                           np.full(n_free, -1, dtype=np.int32)])
    trap = TrapSpec(q_x=0.3, a_x=-0.001, gamma=1e5)
    return Workload("clusters65536", mass, charge, pos[:, 0].copy(), pos[:, 1].copy(),
                    pos[:, 2].copy(), vx, vy, vz, [trap], np.array([0, n], dtype=np.int64), 5000,
                    "mixed", notes=dict(seed=seed, body=body, n_clusters=n_clusters,
                                        per_cluster=per_cluster))


def random_cloud(n: int, seed: int, sigma: float = 50e-6, temperature: float = 10e-3,
                 light_fraction: float = 0.0, charge_e=None) -> Workload:
    """Small test cloud in the crystal8 trap; optional per-ion charges in units of e."""
    w = single_trap(f"cloud{n}", n, sigma, temperature, seed, 0.3, -0.001, 1e5, 0,
                    light_fraction=light_fraction)
    if charge_e is not None:
        w.charge = np.asarray(charge_e, dtype=np.float64) * E_CHARGE
    return w


WORKLOADS = {
    "crystal8": crystal8,
    "crystal1024": crystal1024,
    "mixed16384": mixed16384,
    "batch512": batch512,
    "clusters65536": clusters65536,
}
