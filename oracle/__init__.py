"""Oracle for the trapped-ion Coulomb + linear-Paul-trap + velocity-Verlet path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the GPU library (``paper_1907_10514_amd``) and never imports it.

The heavy lifting is ``lion_oracle.c`` (plain FP64 C, compensated sums, no
fast-math), loaded here through ctypes.  The few closed forms that the paper
states directly are written out in numpy below:

* eq. (Mathieuaq): Mathieu coefficients of the linear Paul trap,
* eq. (pseudopot): pseudopotential secular frequency,
* the axial frequency implied by the dc term of eq. (field).

Every function cites the passage it follows; see ``lion_oracle.c`` for the
statement of the field, the acceleration and the step.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lion_oracle.c")
_LIB = os.path.join(_HERE, "liblion_oracle.so")

# CODATA 2018 / SI 2019, written out independently of the GPU library.
E_CHARGE = 1.602176634e-19  # C
EPS0 = 8.8541878128e-12  # F/m
AMU = 1.66053906660e-27  # kg
K_B = 1.380649e-23  # J/K
COULOMB_K = 1.0 / (4.0 * math.pi * EPS0)


def build(force: bool = True) -> str:
    """Compile ``lion_oracle.c`` into ``liblion_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
               "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Beam(ctypes.Structure):
    _fields_ = [("kx", ctypes.c_double), ("ky", ctypes.c_double), ("kz", ctypes.c_double),
                ("gamma", ctypes.c_double), ("species", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Bath(ctypes.Structure):
    _fields_ = [("temperature", ctypes.c_double), ("tau", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("species", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Trap(ctypes.Structure):
    _fields_ = [("V0", ctypes.c_double), ("Omega", ctypes.c_double), ("U0", ctypes.c_double),
                ("R0", ctypes.c_double), ("Z0", ctypes.c_double), ("kappa", ctypes.c_double),
                ("pseudo", ctypes.c_int32), ("pad", ctypes.c_int32)]


@dataclass(frozen=True)
class Trap:
    """Linear Paul trap of eq. (field): rf amplitude V0 (V) at angular frequency
    Omega (rad/s), end-cap voltage U0 (V), lengths R0, Z0 (m), geometry factor kappa.
    pseudo=True replaces the rf by its pseudopotential (eq. (pseudopot)): a static
    radial field -(Q/M) (V0/R0^2)^2 / (2 Omega^2) (x, y, 0) on each ion."""
    V0: float = 0.0
    Omega: float = 1.0
    U0: float = 0.0
    R0: float = 1.0
    Z0: float = 1.0
    kappa: float = 0.0
    pseudo: bool = False

    def _c(self) -> _Trap:
        return _Trap(self.V0, self.Omega, self.U0, self.R0, self.Z0, self.kappa,
                     1 if self.pseudo else 0, 0)


_lib = None


def bind(path: str):
    """Load a compiled oracle library from ``path`` and declare its prototypes."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lp = ctypes.POINTER(ctypes.c_int64)
    tp = ctypes.POINTER(_Trap)
    lib.oracle_coulomb_constant.restype = ctypes.c_double
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    lib.oracle_coulomb_field.argtypes = [i64, dp, dp, dp, dp, dp, dp, dp]
    lib.oracle_coulomb_field.restype = i64
    lib.oracle_accel.argtypes = [i64, dp, dp, dp, dp, dp, tp, ctypes.c_double, dp, dp, dp]
    lib.oracle_accel.restype = i64
    lib.oracle_accel_scale.argtypes = [i64, dp, dp, dp, dp, dp, tp, ctypes.c_double, dp]
    lib.oracle_accel_scale.restype = None
    lib.oracle_accel_at.argtypes = [i64, dp, dp, dp, dp, dp, tp, ctypes.c_double, i64, lp, dp,
                                    dp, dp, dp]
    lib.oracle_accel_at.restype = None
    lib.oracle_accel_bodies.argtypes = [i64, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int32),
                                        tp, ctypes.c_double, dp, dp, dp, dp]
    lib.oracle_accel_bodies.restype = i64
    lib.oracle_accel_bodies_at.argtypes = [i64, dp, dp, dp, dp, dp,
                                           ctypes.POINTER(ctypes.c_int32), tp, ctypes.c_double,
                                           i64, lp, dp, dp, dp, dp]
    lib.oracle_accel_bodies_at.restype = None
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_normals3.argtypes = [ctypes.c_uint64, i64, i64, ctypes.c_int32, ctypes.c_int32, dp]
    lib.oracle_normals3.restype = None
    lib.oracle_step_cooled.argtypes = [i64, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                       ctypes.POINTER(ctypes.c_int32), tp, ctypes.c_double,
                                       ctypes.c_int, ctypes.POINTER(_Beam), ctypes.c_int,
                                       ctypes.POINTER(_Bath), i64, i64, ctypes.c_double,
                                       ctypes.c_double, i64, dp]
    lib.oracle_step_cooled.restype = i64
    lib.oracle_hessian.argtypes = [i64, dp, dp, dp, dp, dp, tp, dp]
    lib.oracle_hessian.restype = None
    lib.oracle_minimize.argtypes = [i64, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, tp,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, i64, dp]
    lib.oracle_minimize.restype = i64
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_step_rigid.argtypes = [i64, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, ip, ip, dp,
                                      ctypes.c_int32, dp, dp, dp, dp, dp, dp, tp, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, i64, dp]
    lib.oracle_step_rigid.restype = i64
    lib.oracle_time_average.argtypes = [i64, i64, dp, i64, i64, i64, i64, dp,
                                        ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_time_average.restype = i64
    lib.oracle_step.argtypes = [i64, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, tp,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, i64, dp]
    lib.oracle_step.restype = i64
    lib.oracle_energy.argtypes = [i64, dp, dp, dp, dp, dp, dp, dp, dp, tp, dp, dp, dp]
    lib.oracle_energy.restype = None
    lib.oracle_step_batch.argtypes = [ctypes.c_int32, lp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                      dp, dp, tp, dp, dp, dp, i64, dp]
    lib.oracle_step_batch.restype = i64
    lib.oracle_accel_batch.argtypes = [ctypes.c_int32, lp, dp, dp, dp, dp, dp, tp, dp, dp,
                                       dp, dp]
    lib.oracle_accel_batch.restype = i64
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = bind(_LIB)
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count for the oracle's later loops (timing on one core)."""
    _load().oracle_set_num_threads(int(n))


def coulomb_constant() -> float:
    """k_e = 1/(4 pi eps0) as the C oracle evaluates it."""
    return _load().oracle_coulomb_constant()


def coulomb_field(x, y, z, charge):
    """E_c,i = k_e sum_{j!=i} Q_j (r_i-r_j)/|r_i-r_j|^3 (V/m); the field whose
    potential is the pair term of eq. (fullPotential).  Returns (ex, ey, ez, coincident)."""
    x, y, z, q = map(_f64, (x, y, z, charge))
    n = x.size
    ex, ey, ez = np.empty(n), np.empty(n), np.empty(n)
    c = _load().oracle_coulomb_field(n, _d(x), _d(y), _d(z), _d(q), _d(ex), _d(ey), _d(ez))
    return ex, ey, ez, int(c)


def accel(x, y, z, charge, mass, trap: Trap, t: float):
    """a_i = (Q_i/M_i)(E_c,i + E_ext(r_i, t)), eq. (field) with the confining dc
    reading.  Returns (ax, ay, az) in m/s^2."""
    x, y, z, q, m = map(_f64, (x, y, z, charge, mass))
    n = x.size
    ax, ay, az = np.empty(n), np.empty(n), np.empty(n)
    tr = trap._c()
    _load().oracle_accel(n, _d(x), _d(y), _d(z), _d(q), _d(m), ctypes.byref(tr), float(t),
                         _d(ax), _d(ay), _d(az))
    return ax, ay, az


def accel_scale(x, y, z, charge, mass, trap: Trap, t: float) -> np.ndarray:
    """Sum of the magnitudes of all contributions to a_i (m/s^2): the scale
    against which a relative force error is measured."""
    x, y, z, q, m = map(_f64, (x, y, z, charge, mass))
    s = np.empty(x.size)
    tr = trap._c()
    _load().oracle_accel_scale(x.size, _d(x), _d(y), _d(z), _d(q), _d(m), ctypes.byref(tr),
                               float(t), _d(s))
    return s


def accel_at(x, y, z, charge, mass, trap: Trap, t: float, idx):
    """``accel`` and ``accel_scale`` for the targets ``idx`` only (every source
    still counts).  Returns (ax, ay, az, scale) of length len(idx)."""
    x, y, z, q, m = map(_f64, (x, y, z, charge, mass))
    ii = np.ascontiguousarray(idx, dtype=np.int64)
    k = ii.size
    ax, ay, az, sc = np.empty(k), np.empty(k), np.empty(k), np.empty(k)
    tr = trap._c()
    _load().oracle_accel_at(x.size, _d(x), _d(y), _d(z), _d(q), _d(m), ctypes.byref(tr), float(t),
                            k, ii.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _d(ax), _d(ay),
                            _d(az), _d(sc))
    return ax, ay, az, sc


def accel_bodies(x, y, z, charge, mass, body, trap: Trap, t: float):
    """``accel`` with the pairs inside each rigid body left out (body[i] >= 0
    names ion i's body, -1 a free ion).  Returns (ax, ay, az, scale)."""
    x, y, z, q, m = map(_f64, (x, y, z, charge, mass))
    b = np.ascontiguousarray(body, dtype=np.int32)
    n = x.size
    ax, ay, az, sc = np.empty(n), np.empty(n), np.empty(n), np.empty(n)
    tr = trap._c()
    _load().oracle_accel_bodies(n, _d(x), _d(y), _d(z), _d(q), _d(m),
                                b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(tr),
                                float(t), _d(ax), _d(ay), _d(az), _d(sc))
    return ax, ay, az, sc


def accel_bodies_at(x, y, z, charge, mass, body, trap: Trap, t: float, idx):
    """``accel_bodies`` for the targets ``idx`` only (every source counts)."""
    x, y, z, q, m = map(_f64, (x, y, z, charge, mass))
    b = np.ascontiguousarray(body, dtype=np.int32)
    ii = np.ascontiguousarray(idx, dtype=np.int64)
    k = ii.size
    ax, ay, az, sc = np.empty(k), np.empty(k), np.empty(k), np.empty(k)
    tr = trap._c()
    _load().oracle_accel_bodies_at(x.size, _d(x), _d(y), _d(z), _d(q), _d(m),
                                   b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   ctypes.byref(tr), float(t), k,
                                   ii.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _d(ax),
                                   _d(ay), _d(az), _d(sc))
    return ax, ay, az, sc


def step(state: dict, charge, mass, trap: Trap, gamma: float, t_start: float, dt: float,
         nsteps: int) -> dict:
    """Advance ``state`` (dict of x, y, z, vx, vy, vz arrays) by ``nsteps``
    damped velocity-Verlet steps from t_start.  Returns a new dict that also
    holds the final accelerations and time ``t``."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    q, m = _f64(charge), _f64(mass)
    ax, ay, az = accel(s["x"], s["y"], s["z"], q, m, trap, t_start)
    t_end = ctypes.c_double(0.0)
    tr = trap._c()
    _load().oracle_step(s["x"].size, _d(s["x"]), _d(s["y"]), _d(s["z"]), _d(s["vx"]), _d(s["vy"]),
                        _d(s["vz"]), _d(ax), _d(ay), _d(az), _d(q), _d(m), ctypes.byref(tr),
                        float(gamma), float(t_start), float(dt), int(nsteps), ctypes.byref(t_end))
    s.update(ax=ax, ay=ay, az=az, t=t_end.value)
    return s


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) of a 4-word counter and 2-word key."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (ctypes.c_uint32 * 4)()
    _load().oracle_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def normals3(seed, ion, step, bath, half):
    """The three standard normals a bath draws for one ion in one half-step."""
    z = np.empty(3)
    _load().oracle_normals3(int(seed), int(ion), int(step), int(bath), int(half), _d(z))
    return z


def step_cooled(state: dict, charge, mass, species, trap: Trap, gamma: float, beams=(),
                baths=(), step_base: int = 0, t_start: float = 0.0, dt: float = 1e-8,
                nsteps: int = 1, ion_base: int = 0) -> dict:
    """``step`` with cooling beams (dicts k=(kx,ky,kz) unit vector, gamma, species)
    and Langevin baths (dicts temperature, tau, seed, species); see lion_oracle.c.
    ion_base numbers this trap's first ion in the run (bath draws are keyed by it)."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    q, m = _f64(charge), _f64(mass)
    sp = np.ascontiguousarray(species, dtype=np.int32)
    ax, ay, az = accel(s["x"], s["y"], s["z"], q, m, trap, t_start)
    bm = (_Beam * max(1, len(beams)))(*[_Beam(b["k"][0], b["k"][1], b["k"][2], b["gamma"],
                                               b.get("species", -1), 0) for b in beams])
    bt = (_Bath * max(1, len(baths)))(*[_Bath(b["temperature"], b["tau"], b["seed"],
                                               b.get("species", -1), 0) for b in baths])
    t_end = ctypes.c_double(0.0)
    tr = trap._c()
    _load().oracle_step_cooled(s["x"].size, _d(s["x"]), _d(s["y"]), _d(s["z"]), _d(s["vx"]),
                               _d(s["vy"]), _d(s["vz"]), _d(ax), _d(ay), _d(az), _d(q), _d(m),
                               sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               ctypes.byref(tr), float(gamma), len(beams), bm, len(baths), bt,
                               int(ion_base), int(step_base), float(t_start), float(dt),
                               int(nsteps),
                               ctypes.byref(t_end))
    s.update(ax=ax, ay=ay, az=az, t=t_end.value)
    return s


def _matrix_to_quaternion(A):
    """Unit quaternion (w, x, y, z) of the rotation matrix A (Shepperd's choice of
    the largest diagonal term for a well-conditioned square root)."""
    tr = A[0, 0] + A[1, 1] + A[2, 2]
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (A[2, 1] - A[1, 2]) / s, (A[0, 2] - A[2, 0]) / s, (A[1, 0] - A[0, 1]) / s]
    elif A[0, 0] > A[1, 1] and A[0, 0] > A[2, 2]:
        s = math.sqrt(1.0 + A[0, 0] - A[1, 1] - A[2, 2]) * 2
        q = [(A[2, 1] - A[1, 2]) / s, 0.25 * s, (A[0, 1] + A[1, 0]) / s, (A[0, 2] + A[2, 0]) / s]
    elif A[1, 1] > A[2, 2]:
        s = math.sqrt(1.0 + A[1, 1] - A[0, 0] - A[2, 2]) * 2
        q = [(A[0, 2] - A[2, 0]) / s, (A[0, 1] + A[1, 0]) / s, 0.25 * s, (A[1, 2] + A[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + A[2, 2] - A[0, 0] - A[1, 1]) * 2
        q = [(A[1, 0] - A[0, 1]) / s, (A[0, 2] + A[2, 0]) / s, (A[1, 2] + A[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    return q / np.linalg.norm(q)


def quaternion_matrix(q):
    """Rotation matrix of the unit quaternion (w, x, y, z): body frame to space."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


RIGID_MOMENT_FLOOR = 1e-10  # principal moments below this fraction of the largest count as 0


def rigid_setup(state: dict, mass, body) -> dict:
    """Body state of the rigid groups (ions with equal body id >= 0), from the
    ions' positions and velocities: mass, centre of mass, COM velocity, angular
    momentum about the COM, principal axes of the inertia tensor (numpy eigh)
    as the body frame (right-handed), inverse principal moments (0 below
    RIGID_MOMENT_FLOOR of the largest), body-frame offsets of the members, and
    member velocities replaced by the rigid motion V + omega x d."""
    m = _f64(mass)
    body = np.ascontiguousarray(body, dtype=np.int32)
    pos = np.stack([_f64(state["x"]), _f64(state["y"]), _f64(state["z"])], 1)
    vel = np.stack([_f64(state["vx"]), _f64(state["vy"]), _f64(state["vz"])], 1)
    ids = np.unique(body[body >= 0])
    n, nb = body.size, ids.size
    rb = np.full(n, -1, dtype=np.int32)
    M, R, V, L = np.zeros(max(nb, 1)), np.zeros((max(nb, 1), 3)), np.zeros((max(nb, 1), 3)), \
        np.zeros((max(nb, 1), 3))
    Q, inv_i = np.zeros((max(nb, 1), 4)), np.zeros((max(nb, 1), 3))
    dbody = np.zeros((n, 3))
    vel_out = vel.copy()
    for k, b in enumerate(ids):
        idx = np.nonzero(body == b)[0]
        rb[idx] = k
        mk = m[idx]
        M[k] = mk.sum()
        R[k] = (mk[:, None] * pos[idx]).sum(0) / M[k]
        V[k] = (mk[:, None] * vel[idx]).sum(0) / M[k]
        d = pos[idx] - R[k]
        inertia = np.zeros((3, 3))
        for mi, di in zip(mk, d):
            inertia += mi * (np.dot(di, di) * np.eye(3) - np.outer(di, di))
        evals, E = np.linalg.eigh(inertia)
        if np.linalg.det(E) < 0:
            E[:, 2] = -E[:, 2]
        top = max(evals.max(), 0.0)
        inv_i[k] = [1.0 / e if top > 0 and e > RIGID_MOMENT_FLOOR * top else 0.0 for e in evals]
        Q[k] = _matrix_to_quaternion(E)
        A = quaternion_matrix(Q[k])
        dbody[idx] = d @ A
        L[k] = (mk[:, None] * np.cross(d, vel[idx] - V[k])).sum(0)
        w = A @ (inv_i[k] * (A.T @ L[k]))
        vel_out[idx] = V[k] + np.cross(w, d)
    return dict(rb=rb, body=body, nb=nb, M=M, R=R, V=V, L=L, q=Q, inv_i=inv_i, dbody=dbody,
                vx=vel_out[:, 0].copy(), vy=vel_out[:, 1].copy(), vz=vel_out[:, 2].copy())


def step_rigid(state: dict, charge, mass, body, trap: Trap, gamma: float, t_start: float,
               dt: float, nsteps: int, rigid: dict | None = None) -> tuple[dict, dict]:
    """``step`` with rigid bodies (see lion_oracle.c).  With rigid=None the body
    state is set up from ``state`` by rigid_setup (member velocities become the
    rigid motion); pass the returned body state to continue a run.  Returns
    (ion state with accelerations and t, body state)."""
    q_, m = _f64(charge), _f64(mass)
    if rigid is None:
        rigid = rigid_setup(state, m, body)
        s = {k: _f64(state[k]).copy() for k in ("x", "y", "z")}
        s.update(vx=rigid["vx"].copy(), vy=rigid["vy"].copy(), vz=rigid["vz"].copy())
    else:
        s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    rg = {k: (np.ascontiguousarray(v).copy() if isinstance(v, np.ndarray) else v)
          for k, v in rigid.items()}
    ax, ay, az, _ = accel_bodies(s["x"], s["y"], s["z"], q_, m, rg["body"], trap, t_start)
    ip = ctypes.POINTER(ctypes.c_int32)
    t_end = ctypes.c_double(0.0)
    tr = trap._c()
    _load().oracle_step_rigid(s["x"].size, _d(s["x"]), _d(s["y"]), _d(s["z"]), _d(s["vx"]),
                              _d(s["vy"]), _d(s["vz"]), _d(ax), _d(ay), _d(az), _d(q_), _d(m),
                              rg["body"].ctypes.data_as(ip), rg["rb"].ctypes.data_as(ip),
                              _d(rg["dbody"]), int(rg["nb"]), _d(rg["M"]), _d(rg["inv_i"]),
                              _d(rg["q"]), _d(rg["R"]), _d(rg["V"]), _d(rg["L"]),
                              ctypes.byref(tr), float(gamma), float(t_start), float(dt),
                              int(nsteps), ctypes.byref(t_end))
    s.update(ax=ax, ay=ay, az=az, t=t_end.value)
    return s, rg


def hessian(x, y, z, charge, mass, trap: Trap) -> np.ndarray:
    """Mass-weighted Hessian (3n x 3n) of the static potential (see lion_oracle.c)."""
    x, y, z, q, m = map(_f64, (x, y, z, charge, mass))
    n = x.size
    D = np.empty((3 * n, 3 * n))
    tr = trap._c()
    _load().oracle_hessian(n, _d(x), _d(y), _d(z), _d(q), _d(m), ctypes.byref(tr), _d(D))
    return D


def normal_modes(x, y, z, charge, mass, trap: Trap):
    """Squared angular frequencies (ascending) and modes (columns, index 3i+axis)
    of the mass-weighted Hessian, by numpy's symmetric eigen-solver."""
    w2, v = np.linalg.eigh(hessian(x, y, z, charge, mass, trap))
    return w2, v


def minimize(state: dict, charge, mass, trap: Trap, dt: float, dmax: float, ftol: float,
             max_iter: int, t: float = 0.0) -> dict:
    """Energy minimisation (see lion_oracle.c): damped dynamics keeping only the
    velocity component along the force, a per-ion step cap dmax (m), until
    max_i |F_i| <= ftol (N) or max_iter iterations.  Returns the state with the
    final accelerations, 'iterations' and 'fmax'."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    q, m = _f64(charge), _f64(mass)
    n = s["x"].size
    ax, ay, az = np.empty(n), np.empty(n), np.empty(n)
    fmax = ctypes.c_double(0.0)
    tr = trap._c()
    it = _load().oracle_minimize(n, _d(s["x"]), _d(s["y"]), _d(s["z"]), _d(s["vx"]), _d(s["vy"]),
                                 _d(s["vz"]), _d(ax), _d(ay), _d(az), _d(q), _d(m),
                                 ctypes.byref(tr), float(t), float(dt), float(dmax), float(ftol),
                                 int(max_iter), ctypes.byref(fmax))
    s.update(ax=ax, ay=ay, az=az, iterations=int(it), fmax=fmax.value)
    return s


def time_average(samples, first_step: int, origin: int, window: int):
    """timeAvg: means of the windows of ``window`` steps closing at origin + m W
    that lie wholly among ``samples`` (rows taken at the end of run-wide steps
    first_step, first_step + 1, ...).  Returns (end_steps, means[n_windows, n])."""
    a = np.ascontiguousarray(samples, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    ns, n = a.shape
    maxw = max(1, ns // max(1, int(window)) + 1)
    means = np.empty((maxw, n))
    ends = np.empty(maxw, dtype=np.int64)
    k = _load().oracle_time_average(n, ns, _d(a), int(first_step), int(origin), int(window), maxw,
                                    _d(means), ends.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return ends[:k].copy(), means[:k].copy()


def energy(state: dict, charge, mass, trap: Trap):
    """(kinetic, Coulomb, dc-trap) energies in J; Coulomb is the pair term of
    eq. (fullPotential) counted once per pair."""
    x, y, z, vx, vy, vz = (_f64(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz"))
    q, m = _f64(charge), _f64(mass)
    k, c, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    tr = trap._c()
    _load().oracle_energy(x.size, _d(x), _d(y), _d(z), _d(vx), _d(vy), _d(vz), _d(q), _d(m),
                          ctypes.byref(tr), ctypes.byref(k), ctypes.byref(c), ctypes.byref(d))
    return k.value, c.value, d.value


def accel_batch(offsets, x, y, z, charge, mass, traps, t):
    """Per-trap accel for independent traps concatenated in trap order."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    x, y, z, q, m = map(_f64, (x, y, z, charge, mass))
    tarr = (_Trap * len(traps))(*[tr._c() for tr in traps])
    tt = _f64(t)
    n = x.size
    ax, ay, az = np.empty(n), np.empty(n), np.empty(n)
    _load().oracle_accel_batch(len(traps), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               _d(x), _d(y), _d(z), _d(q), _d(m), tarr, _d(tt), _d(ax), _d(ay),
                               _d(az))
    return ax, ay, az


def step_batch(offsets, state: dict, charge, mass, traps, gamma, t_start, dt, nsteps: int):
    """``step`` applied to each trap of a batch with its own parameters."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    q, m = _f64(charge), _f64(mass)
    ts, g, h = _f64(t_start), _f64(gamma), _f64(dt)
    ax, ay, az = accel_batch(off, s["x"], s["y"], s["z"], q, m, traps, ts)
    tarr = (_Trap * len(traps))(*[tr._c() for tr in traps])
    t_end = np.empty(len(traps))
    _load().oracle_step_batch(len(traps), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              _d(s["x"]), _d(s["y"]), _d(s["z"]), _d(s["vx"]), _d(s["vy"]),
                              _d(s["vz"]), _d(ax), _d(ay), _d(az), _d(q), _d(m), tarr, _d(g),
                              _d(ts), _d(h), int(nsteps), _d(t_end))
    s.update(ax=ax, ay=ay, az=az, t=t_end)
    return s


# ---------------------------------------------------------------- closed forms

def mathieu_coefficients(V0, U0, M, Q, Omega, R0, Z0, kappa):
    """eq. (Mathieuaq): (q_x, a_x) with q_y = -q_x, a_y = a_x, a_z = -2 a_x, q_z = 0."""
    a_x = -4.0 * Q * kappa * U0 / (M * Z0 ** 2 * Omega ** 2)
    q_x = 2.0 * Q * V0 / (M * R0 ** 2 * Omega ** 2)
    return q_x, a_x


def voltages_for(q_x, a_x, M, Q, Omega, R0, Z0, kappa):
    """Inverse of eq. (Mathieuaq): the (V0, U0) that give (q_x, a_x) to an ion of
    mass M and charge Q."""
    V0 = q_x * M * R0 ** 2 * Omega ** 2 / (2.0 * Q)
    U0 = -a_x * M * Z0 ** 2 * Omega ** 2 / (4.0 * Q * kappa)
    return V0, U0


def pseudopotential_frequency(q, a, Omega):
    """eq. (pseudopot): omega ~ (Omega/2) sqrt(a + q^2/2), rad/s."""
    return 0.5 * Omega * math.sqrt(a + 0.5 * q * q)


def axial_frequency(U0, M, Q, Z0, kappa):
    """omega_z of the dc term of eq. (field): z'' = -(2 Q kappa U0/(M Z0^2)) z."""
    return math.sqrt(2.0 * Q * kappa * U0 / (M * Z0 ** 2))
