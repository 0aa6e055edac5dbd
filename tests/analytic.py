"""Independent closed forms and brute-force references used to pin the oracle.

Nothing here calls the oracle or the GPU library: each helper restates a fact
from the paper or from textbook mechanics in separate code, so that a mistake
in the oracle (a dropped term, a wrong sign, a swapped index) shows up as a
disagreement.
"""
from __future__ import annotations

import math
from decimal import Decimal, getcontext

import numpy as np

EPS0 = 8.8541878128e-12
E = 1.602176634e-19
AMU = 1.66053906660e-27


# ------------------------------------------------------------ 40-digit brute force

def _dsqrt(v: Decimal) -> Decimal:
    return v.sqrt()


def decimal_accel(x, y, z, charge, mass, V0, Omega, U0, R0, Z0, kappa, t, body=None):
    """Acceleration of every ion at 40 significant digits: pair Coulomb field of
    eq. (fullPotential) plus eq. (field) with the axially confining dc sign.
    cos(Omega t) is taken from FP64 (it is an FP64 input on both sides).
    Returns (ax, ay, az, scale) as float arrays; scale is the sum of the
    magnitudes of all contributions."""
    getcontext().prec = 40
    D = Decimal
    n = len(x)
    X = [D(float(v)) for v in x]
    Y = [D(float(v)) for v in y]
    Zs = [D(float(v)) for v in z]
    Q = [D(float(v)) for v in charge]
    M = [D(float(v)) for v in mass]
    pi = D("3.141592653589793238462643383279502884197")
    ke = D(1) / (D(4) * pi * D(EPS0))
    arf = D(float(V0)) / (D(float(R0)) ** 2)
    adc = D(float(kappa)) * D(float(U0)) / (D(float(Z0)) ** 2)
    c = D(math.cos(float(Omega) * float(t)))
    ax, ay, az, sc = [], [], [], []
    for i in range(n):
        ex = ey = ez = D(0)
        mag = D(0)
        for j in range(n):
            if j == i:
                continue
            if body is not None and body[i] >= 0 and body[j] == body[i]:
                continue
            dx, dy, dz = X[i] - X[j], Y[i] - Y[j], Zs[i] - Zs[j]
            r2 = dx * dx + dy * dy + dz * dz
            r = _dsqrt(r2)
            ex += ke * Q[j] * dx / (r2 * r)
            ey += ke * Q[j] * dy / (r2 * r)
            ez += ke * Q[j] * dz / (r2 * r)
            mag += ke * abs(Q[j]) / r2
        erf = (arf * c, -arf * c)
        ex += erf[0] * X[i] + adc * X[i]
        ey += erf[1] * Y[i] + adc * Y[i]
        ez += -2 * adc * Zs[i]
        mag += abs(arf * c) * _dsqrt(X[i] ** 2 + Y[i] ** 2)
        mag += abs(adc) * _dsqrt(X[i] ** 2 + Y[i] ** 2 + 4 * Zs[i] ** 2)
        k = Q[i] / M[i]
        ax.append(float(k * ex))
        ay.append(float(k * ey))
        az.append(float(k * ez))
        sc.append(float(abs(k) * mag))
    return np.array(ax), np.array(ay), np.array(az), np.array(sc)


def decimal_steps(state, charge, mass, U0, Z0, kappa, gamma, dt, nsteps):
    """Damped velocity Verlet (velocity scaled by exp(-gamma dt/2) before the
    first half kick and after the second) at 40 digits, rf off."""
    getcontext().prec = 40
    D = Decimal
    n = len(state["x"])
    P = {k: [D(float(v)) for v in state[k]] for k in ("x", "y", "z", "vx", "vy", "vz")}
    dtD = D(float(dt))
    f = (-(D(float(gamma)) * dtD) / 2).exp()

    # accelerations recomputed at 40 digits from the 40-digit positions
    def acc40():
        getcontext().prec = 40
        pi = D("3.141592653589793238462643383279502884197")
        ke = D(1) / (D(4) * pi * D(EPS0))
        adc = D(float(kappa)) * D(float(U0)) / (D(float(Z0)) ** 2)
        out = [[], [], []]
        for i in range(n):
            e = [D(0), D(0), D(0)]
            for j in range(n):
                if j == i:
                    continue
                d = [P["x"][i] - P["x"][j], P["y"][i] - P["y"][j], P["z"][i] - P["z"][j]]
                r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
                r3 = r2 * r2.sqrt()
                for c in range(3):
                    e[c] += ke * D(float(charge[j])) * d[c] / r3
            e[0] += adc * P["x"][i]
            e[1] += adc * P["y"][i]
            e[2] += -2 * adc * P["z"][i]
            k = D(float(charge[i])) / D(float(mass[i]))
            for c in range(3):
                out[c].append(k * e[c])
        return out

    a = acc40()
    for _ in range(nsteps):
        for i in range(n):
            for c, (p, v) in enumerate((("x", "vx"), ("y", "vy"), ("z", "vz"))):
                P[v][i] = f * P[v][i] + dtD / 2 * a[c][i]
                P[p][i] = P[p][i] + dtD * P[v][i]
        a = acc40()
        for i in range(n):
            for c, v in enumerate(("vx", "vy", "vz")):
                P[v][i] = f * (P[v][i] + dtD / 2 * a[c][i])
    return {k: np.array([float(v) for v in P[k]]) for k in P}


# ---------------------------------------------------- linear single-ion dynamics

def verlet_transfer(k_now: float, k_next: float, f: float, dt: float) -> np.ndarray:
    """2x2 map of one damped velocity-Verlet step for x'' = k(t) x on (x, v):
    v <- f v + (dt/2) k_now x; x <- x + dt v; v <- f (v + (dt/2) k_next x)."""
    h = 0.5 * dt
    A = np.array([[1.0, 0.0], [h * k_now, f]])           # v <- f v + h k x
    B = np.array([[1.0, dt], [0.0, 1.0]])                 # x <- x + dt v
    C = np.array([[1.0, 0.0], [f * h * k_next, f]])       # v <- f (v + h k' x)
    return C @ B @ A


def linear_trajectory(x0, v0, k_of_t, f, dt, nsteps, t0=0.0):
    """Iterate ``verlet_transfer`` from (x0, v0); returns arrays x[k], v[k], k=0..nsteps."""
    xs, vs = [x0], [v0]
    s = np.array([x0, v0], dtype=np.float64)
    for k in range(nsteps):
        s = verlet_transfer(k_of_t(t0 + k * dt), k_of_t(t0 + (k + 1) * dt), f, dt) @ s
        xs.append(s[0])
        vs.append(s[1])
    return np.array(xs), np.array(vs)


def floquet_beta(k_of_t, T, steps_per_period):
    """Characteristic exponent beta (secular frequency = beta Omega / 2) of the
    undamped discrete map over one rf period, from the trace of its monodromy."""
    dt = T / steps_per_period
    Mtot = np.eye(2)
    for k in range(steps_per_period):
        Mtot = verlet_transfer(k_of_t(k * dt), k_of_t((k + 1) * dt), 1.0, dt) @ Mtot
    tr = np.trace(Mtot)
    return math.acos(tr / 2.0) / math.pi  # beta in (0, 1)


# --------------------------------------------------------- axial chain equilibrium

def chain_equilibrium(n: int) -> np.ndarray:
    """Dimensionless equilibrium positions u_i = z_i / l of an n-ion chain in a
    harmonic well, l^3 = Q^2/(4 pi eps0 M omega_z^2): roots of
    u_i - sum_{j<i} (u_i-u_j)^-2 + sum_{j>i} (u_i-u_j)^-2 = 0 by Newton's method."""
    if n == 1:
        return np.zeros(1)
    u = np.linspace(-1.0, 1.0, n) * (n ** 0.6)
    for _ in range(200):
        d = u[:, None] - u[None, :]
        np.fill_diagonal(d, np.inf)
        F = u - np.sum(np.sign(d) / d ** 2, axis=1)
        off = 2.0 / np.abs(d) ** 3
        J = -off
        np.fill_diagonal(J, 1.0 + np.sum(off, axis=1))
        du = np.linalg.solve(J, F)
        u = u - du
        if np.max(np.abs(du)) < 1e-15:
            break
    return np.sort(u)
