"""Trajectory bars for the FP32 pair paths on chaotic clouds.

A K-step run of a hot cloud cannot be compared with the oracle's to a fixed
fraction of the displacement: the dynamics amplify any difference in the
forces.  The bar is derived from what the path's forces actually inject.

If a path's acceleration differs from the oracle's by at most M1 A_i per ion
(A_i the sum of the magnitudes of every contribution to a_i, M1 the measured
relative force error of that path on that state), each velocity-Verlet step
adds at most dt M1 A_i to ion i's velocity error.  The envelope is how far
the oracle's own run moves when exactly that is injected: after every oracle
step, ion i's velocity gets dt M1 A_i xi_i, with xi_i a fixed, seeded unit
vector (the same direction every step: a coherent error, the worst case of an
error that varies slowly along the run).  A run passes if it stays within 10x
that envelope.

Ions of a rigid body receive the kick through their body: the summed member
impulse changes the body's COM velocity and its angular momentum about the
COM.

The kicked run also starts from the state with every component moved by one
ulp (random signs): for FP64 paths, whose force error is at the rounding
level, that start shift is the larger part.

The oracle runs one step per call here; the unkicked reference is the test's
own full-length oracle run.  The two differ only in the rounding of the time
t_k (one ulp), far below the kicks.
"""
from __future__ import annotations

import numpy as np

FACTOR = 10.0  # bar = FACTOR x envelope


def m1(a, b, scale) -> float:
    """max_i |a_i - b_i| / scale_i over ions (three components each)."""
    return float(np.max(np.sqrt((np.asarray(a[0]) - b[0]) ** 2 + (np.asarray(a[1]) - b[1]) ** 2
                                + (np.asarray(a[2]) - b[2]) ** 2) / scale))


def kick(scale, m1_value: float, dt: float, seed: int = 0) -> np.ndarray:
    """(3, n) velocity kicks dt M1 A_i xi_i, xi_i seeded unit vectors."""
    scale = np.asarray(scale, dtype=np.float64)
    xi = np.random.default_rng(seed).normal(size=(3, scale.size))
    xi /= np.linalg.norm(xi, axis=0)
    return dt * m1_value * scale * xi


def nudge(state: dict, seed: int = 1) -> dict:
    """The state with every position and velocity component moved by one ulp,
    up or down at random (seeded): the rounding size of an FP64 state.  It is
    part of every envelope, and the larger part for FP64 paths, whose force
    error is at the rounding level; the random signs also perturb the offsets
    and spins of rigid bodies set up from the state, which a common shift
    would leave alone."""
    rng = np.random.default_rng(seed)
    s = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v)
         for k, v in state.items()}
    for k in X + V:
        a = np.asarray(s[k], dtype=np.float64)
        s[k] = np.nextafter(a, np.where(rng.random(a.shape) < 0.5, -np.inf, np.inf))
    return s


def kicked_run(step_one, state: dict, nsteps: int, dv: np.ndarray, apply=None) -> dict:
    """nsteps calls of step_one(state, k) -> state (one step from step index
    k), each followed by the velocity kicks dv: added to the ion velocities,
    or handed to apply(state, dv) when given (rigid bodies)."""
    s = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v)
         for k, v in state.items()}
    for k in range(nsteps):
        s = step_one(s, k)
        if apply is not None:
            apply(s, dv)
        else:
            s["vx"] = s["vx"] + dv[0]
            s["vy"] = s["vy"] + dv[1]
            s["vz"] = s["vz"] + dv[2]
    return s


def kick_rigid(rigid: dict, state: dict, mass, dv: np.ndarray) -> None:
    """Apply the member velocity kicks dv of rigid bodies to their bodies (in
    place): dV = sum m_i dv_i / M, dL = sum (r_i - R) x m_i dv_i."""
    rb = rigid["rb"]
    m = np.asarray(mass, dtype=np.float64)
    pos = np.stack([state["x"], state["y"], state["z"]], 1)
    imp = (m[:, None] * dv.T)
    for b in range(int(rigid["nb"])):
        idx = np.nonzero(rb == b)[0]
        rigid["V"][b] += imp[idx].sum(0) / rigid["M"][b]
        rigid["L"][b] += np.cross(pos[idx] - rigid["R"][b], imp[idx]).sum(0)


def divergence(a: dict, b: dict, keys=("x", "y", "z")) -> float:
    return max(float(np.max(np.abs(np.asarray(a[k]) - np.asarray(b[k])))) for k in keys)


# Relative force error at which the segment bars were shown to catch the
# planted mistakes of the CPU controls (tests/test_trajectory_bar_cpu.py); the
# GPU tests require their measured M1 to be at most this.
M1_REF = 1e-7
# Steps of one re-anchored segment.
SEGMENT = 10
# Lower bound on M1 for the FP64 paths: their rounding differences outside the
# force sum (transcendental functions of the trap phase and of the bath draws,
# the O(N) update) are a few FP64 ulps and are not part of the measured M1.
M1_FLOOR = 1e-15

X = ("x", "y", "z")
V = ("vx", "vy", "vz")


def per_ion(a: dict, b: dict, keys=X) -> np.ndarray:
    """|a_i - b_i| per ion over the given three components."""
    return np.sqrt(sum((np.asarray(a[k]) - np.asarray(b[k])) ** 2 for k in keys))


def ratio(got: dict, ref: dict, kicked: dict, keys=X) -> float:
    """max_i |got_i - ref_i| / (FACTOR max(|kicked_i - ref_i|, ulp_i)): at most
    1 within the per-ion bars.  ulp_i, the spacing of doubles at ion i's largest
    component, keeps a bar above zero where the kicks of an FP64 path are lost
    in the rounding of the state."""
    env = per_ion(kicked, ref, keys)
    ulp = np.spacing(np.max(np.abs(np.stack([np.asarray(ref[k]) for k in keys])), axis=0))
    return float(np.max(per_ion(got, ref, keys) / (FACTOR * np.maximum(env, ulp))))


def _copy_rigid(rg: dict) -> dict:
    return {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in rg.items()}


def rigid_anchor(oracle_mod, setup0: dict, quat0, rs: dict) -> dict:
    """The oracle's body state equal to a GPU body state: the GPU's COM, COM
    velocity and angular momentum, and its orientation carried into the
    oracle's body frame.  setup0 is the oracle's set-up from the start state,
    quat0 the GPU's orientations right after its own set-up from that state and
    rs the GPU's rigid state now.  Each side may pick any principal frame of the
    same inertia tensor; the rotation since the start is common, so with A(q)
    the orientation matrices A_oracle = A_gpu A_gpu(0)^T A_oracle(0).
    (Setting the bodies up again from the GPU's member positions and velocities
    would lose digits: a spin is a small difference of large member
    velocities.)"""
    rg = _copy_rigid(setup0)
    for b in range(int(setup0["nb"])):
        qm = oracle_mod.quaternion_matrix
        A = qm(rs["quaternion"][b]) @ qm(quat0[b]).T @ qm(setup0["q"][b])
        rg["q"][b] = oracle_mod._matrix_to_quaternion(A)  # Shepperd's method
        rg["R"][b] = rs["com"][b]
        rg["V"][b] = rs["com_velocity"][b]
        rg["L"][b] = rs["angular_momentum"][b]
    return rg


def nudge_rigid(rg: dict, seed: int = 2) -> dict:
    """Body state with every component of R, V, L and q moved by one ulp (random
    signs), the rigid counterpart of nudge."""
    rng = np.random.default_rng(seed)
    out = _copy_rigid(rg)
    for k in ("R", "V", "L", "q"):
        a = np.asarray(out[k], dtype=np.float64)
        out[k] = np.nextafter(a, np.where(rng.random(a.shape) < 0.5, -np.inf, np.inf))
    return out


def rigid_segment(oracle_mod, s0, rg0, q, m, body, tr, gamma, t0, dt):
    """(reference run, apply-kick function, one-step function, kicked start
    state) of a rigid segment from ions s0 and bodies rg0 at time t0.  The
    kicked run starts one ulp off (nudge, nudge_rigid); free ions are kicked
    directly, bodies through their summed member impulses."""
    ref, _ = oracle_mod.step_rigid(s0, q, m, body, tr, gamma, t0, dt, SEGMENT,
                                   rigid=_copy_rigid(rg0))
    free = np.asarray(body) < 0

    def apply(s, dv):
        for c, k in enumerate(V):
            s[k] = np.where(free, s[k] + dv[c], s[k])
        kick_rigid(s["rigid"], s, m, dv)

    def one(s, k):
        out, r = oracle_mod.step_rigid(s, q, m, body, tr, gamma, t0 + k * dt, dt, 1,
                                       rigid=s["rigid"])
        out["rigid"] = r
        return out

    init = nudge(s0)
    init["rigid"] = nudge_rigid(rg0)
    return ref, apply, one, init


def ulp_envelope(run, state: dict):
    """FP64 paths over whole runs: how far the oracle's own run moves when every
    start position is moved by one ulp.  Returns (max |dx|, max |dv|)."""
    a = run(state)
    s2 = {k: np.array(v, copy=True) for k, v in state.items()}
    for k in X:
        s2[k] = np.nextafter(s2[k], np.inf)
    b = run(s2)
    return divergence(a, b, X), divergence(a, b, V)
