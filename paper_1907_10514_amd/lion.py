"""ctypes binding of ``liblion.so`` (the C ABI declared in ``include/lion.h``).

Functions keep the C names and only marshal arguments: numpy arrays become
double pointers, torch supplies the device workspace and the HIP stream.  Every
step of the simulation runs in the library's HIP kernels; if the library is
missing this module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblion.so")

LION_FP64 = 0
LION_MIXED_F64ACC = 1
LION_MIXED_KAHAN = 2
PRECISIONS = {"fp64": LION_FP64, "mixed": LION_MIXED_F64ACC, "mixed_f64acc": LION_MIXED_F64ACC,
              "mixed_kahan": LION_MIXED_KAHAN}

LION_OK = 0
LION_ERR_ARG = -1
LION_ERR_STATE = -2
LION_ERR_HIP = -3
LION_ERR_WORKSPACE = -4
LION_ERR_NONFINITE = -5
LION_ERR_UNSUPPORTED = -6


class LionError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lion error {code}: {msg}")
        self.code = code


class KernelConfig(ctypes.Structure):
    _fields_ = [("i_per_lane", ctypes.c_int32), ("j_split", ctypes.c_int32),
                ("chunk_steps", ctypes.c_int32), ("flush_len", ctypes.c_int32),
                ("batch_block", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("lds_sources", ctypes.c_int32), ("symmetric", ctypes.c_int32),
                ("sym_variant", ctypes.c_int32), ("update_waves", ctypes.c_int32),
                ("small_trap", ctypes.c_int32), ("batch_tpt", ctypes.c_int32),
                ("step_launches", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load the library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1907_10514_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, dp, i32, i64, sz = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                            ctypes.c_int64, ctypes.c_size_t)
    d = ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.lion_workspace_bytes.argtypes = [i64, i32, ctypes.c_int]
    lib.lion_workspace_bytes.restype = sz
    lib.lion_create.argtypes = [pp, i64, dp, dp, ctypes.c_int, vp, sz, vp]
    lib.lion_create_batch.argtypes = [pp, i32, ctypes.POINTER(ctypes.c_int64), dp, dp,
                                      ctypes.c_int, vp, sz, vp]
    lib.lion_set_state.argtypes = [vp, dp, dp, dp, dp, dp, dp, d]
    lib.lion_set_trap.argtypes = [vp, i32, d, d, d, d, d, d]
    lib.lion_set_damping.argtypes = [vp, i32, d]
    lib.lion_set_bodies.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.lion_set_species.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.lion_set_pseudo_trap.argtypes = [vp, i32, d, d, d, d, d, d]
    lib.lion_minimize.argtypes = [vp, d, d, d, i64, ctypes.POINTER(ctypes.c_int64), dp]
    lib.lion_normal_modes_workspace_bytes.argtypes = [vp]
    lib.lion_normal_modes_workspace_bytes.restype = sz
    lib.lion_normal_modes.argtypes = [vp, vp, sz, dp, dp]
    lib.lion_set_rigid_bodies.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.lion_get_rigid_state.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), dp, dp, dp, dp]
    lib.lion_set_beam.argtypes = [vp, i32, i32, d, d, d, d]
    lib.lion_set_bath.argtypes = [vp, i32, i32, d, d, ctypes.c_uint64]
    lib.lion_set_step_index.argtypes = [vp, i64]
    lib.lion_get_step_index.argtypes = [vp]
    lib.lion_get_step_index.restype = i64
    lib.lion_set_time_average.argtypes = [vp, i32]
    lib.lion_get_time_average.argtypes = [vp, dp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.lion_step.argtypes = [vp, i64, d]
    lib.lion_step_batch.argtypes = [vp, i64, dp]
    lib.lion_prepare_step.argtypes = [vp, i64]
    lib.lion_get_state.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp]
    lib.lion_compute_accel.argtypes = [vp, dp, dp, dp]
    lib.lion_get_energy.argtypes = [vp, dp, dp, dp]
    lib.lion_check_finite.argtypes = [vp]
    lib.lion_count_lost.argtypes = [vp, d, ctypes.POINTER(ctypes.c_int64)]
    lib.lion_last_error.argtypes = [vp]
    lib.lion_last_error.restype = ctypes.c_char_p
    lib.lion_destroy.argtypes = [vp]
    lib.lion_destroy.restype = None
    lib.lion_set_kernel_config.argtypes = [vp, ctypes.POINTER(KernelConfig)]
    lib.lion_get_kernel_config.argtypes = [vp, ctypes.POINTER(KernelConfig)]
    lib.lion_time_pair_kernel.argtypes = [vp, i32, dp]
    lib.lion_time_batch_kernel.argtypes = [vp, i32, i32, d, dp]
    lib.lion_mathieu_to_voltages.argtypes = [d, d, d, d, d, d, d, d, dp, dp]
    lib.lion_accel_noalloc.argtypes = [i64, vp, vp, vp, vp, vp, d, d, d, d, d, d, d,
                                       ctypes.c_int, vp, vp, vp, vp]
    lib.lion_constants.argtypes = [dp, dp, dp]
    lib.lion_constants.restype = None
    for name in ("lion_create", "lion_create_batch", "lion_set_state", "lion_set_trap",
                 "lion_set_damping", "lion_set_bodies", "lion_set_rigid_bodies",
                 "lion_get_rigid_state", "lion_set_pseudo_trap", "lion_minimize",
                 "lion_normal_modes",
                 "lion_set_species", "lion_set_beam",
                 "lion_set_bath", "lion_set_step_index", "lion_set_time_average",
                 "lion_get_time_average", "lion_step", "lion_step_batch", "lion_prepare_step",
                 "lion_get_state",
                 "lion_compute_accel", "lion_get_energy", "lion_check_finite", "lion_count_lost",
                 "lion_set_kernel_config", "lion_get_kernel_config", "lion_mathieu_to_voltages",
                 "lion_time_pair_kernel", "lion_time_batch_kernel", "lion_accel_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, handle=None):
    if rc != LION_OK:
        msg = load().lion_last_error(handle)
        raise LionError(rc, msg.decode() if msg else "")


# ------------------------------------------------------------------ raw calls

def lion_workspace_bytes(n_total: int, n_traps: int, precision: int) -> int:
    return int(load().lion_workspace_bytes(int(n_total), int(n_traps), int(precision)))


def lion_create(n, masses, charges, precision, workspace_ptr, ws_bytes, stream_ptr):
    h = ctypes.c_void_p()
    m, q = _f64(masses), _f64(charges)
    _check(load().lion_create(ctypes.byref(h), int(n), _dp(m), _dp(q), int(precision),
                              ctypes.c_void_p(workspace_ptr), int(ws_bytes),
                              ctypes.c_void_p(stream_ptr)))
    return h


def lion_create_batch(n_per_trap, masses, charges, precision, workspace_ptr, ws_bytes,
                      stream_ptr):
    h = ctypes.c_void_p()
    npt = np.ascontiguousarray(n_per_trap, dtype=np.int64)
    m, q = _f64(masses), _f64(charges)
    _check(load().lion_create_batch(ctypes.byref(h), int(npt.size),
                                    npt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(m),
                                    _dp(q), int(precision), ctypes.c_void_p(workspace_ptr),
                                    int(ws_bytes), ctypes.c_void_p(stream_ptr)))
    return h


def lion_set_state(h, x, y, z, vx, vy, vz, t=0.0):
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz)]
    _check(load().lion_set_state(h, *[_dp(a) for a in arrs], float(t)), h)


def lion_set_trap(h, trap, V_rf, Omega, U_dc, r0, z0, kappa):
    _check(load().lion_set_trap(h, int(trap), float(V_rf), float(Omega), float(U_dc), float(r0),
                                float(z0), float(kappa)), h)


def lion_set_damping(h, trap, gamma):
    _check(load().lion_set_damping(h, int(trap), float(gamma)), h)


def lion_set_bodies(h, body_id):
    if body_id is None:
        _check(load().lion_set_bodies(h, None), h)
        return
    b = np.ascontiguousarray(body_id, dtype=np.int32)
    _check(load().lion_set_bodies(h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), h)


def lion_set_rigid_bodies(h, body):
    if body is None:
        _check(load().lion_set_rigid_bodies(h, None), h)
        return
    b = np.ascontiguousarray(body, dtype=np.int32)
    _check(load().lion_set_rigid_bodies(h, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), h)


def lion_get_rigid_state(h, max_bodies):
    nb = ctypes.c_int32(0)
    m = max(1, int(max_bodies))
    com, vel, ang, quat = np.empty(3 * m), np.empty(3 * m), np.empty(3 * m), np.empty(4 * m)
    _check(load().lion_get_rigid_state(h, ctypes.byref(nb), _dp(com), _dp(vel), _dp(ang),
                                       _dp(quat)), h)
    k = nb.value
    return dict(com=com[:3 * k].reshape(k, 3), com_velocity=vel[:3 * k].reshape(k, 3),
                angular_momentum=ang[:3 * k].reshape(k, 3), quaternion=quat[:4 * k].reshape(k, 4))


def lion_set_pseudo_trap(h, trap, V_rf, Omega, U_dc, r0, z0, kappa):
    _check(load().lion_set_pseudo_trap(h, int(trap), float(V_rf), float(Omega), float(U_dc),
                                       float(r0), float(z0), float(kappa)), h)


def lion_minimize(h, dt, dmax, ftol, max_iter):
    it = ctypes.c_int64(0)
    fm = ctypes.c_double(0.0)
    _check(load().lion_minimize(h, float(dt), float(dmax), float(ftol), int(max_iter),
                                ctypes.byref(it), ctypes.byref(fm)), h)
    return int(it.value), float(fm.value)


def lion_normal_modes_workspace_bytes(h):
    nb = int(load().lion_normal_modes_workspace_bytes(h))
    if nb == 0:
        raise LionError(LION_ERR_HIP, lion_last_error(h))
    return nb


def lion_normal_modes(h, n, ws_ptr, ws_bytes, vectors=False):
    m = 3 * int(n)
    w2 = np.empty(m)
    modes = np.empty((m, m), order="F") if vectors else None
    _check(load().lion_normal_modes(h, ctypes.c_void_p(ws_ptr), int(ws_bytes), _dp(w2),
                                    _dp(modes) if vectors else None), h)
    return w2, modes


def lion_set_species(h, species):
    if species is None:
        _check(load().lion_set_species(h, None), h)
        return
    sp = np.ascontiguousarray(species, dtype=np.int32)
    _check(load().lion_set_species(h, sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), h)


def lion_set_beam(h, beam, species, kx, ky, kz, gamma):
    _check(load().lion_set_beam(h, int(beam), int(species), float(kx), float(ky), float(kz),
                                float(gamma)), h)


def lion_set_bath(h, bath, species, temperature, damping_time, seed):
    _check(load().lion_set_bath(h, int(bath), int(species), float(temperature),
                                float(damping_time), int(seed) & 0xffffffffffffffff), h)


def lion_set_step_index(h, steps_done):
    _check(load().lion_set_step_index(h, int(steps_done)), h)


def lion_get_step_index(h) -> int:
    return int(load().lion_get_step_index(h))


def lion_set_time_average(h, window_steps):
    _check(load().lion_set_time_average(h, int(window_steps)), h)


def lion_get_time_average(h, n):
    out = [np.empty(int(n)) for _ in range(3)]
    end = ctypes.c_int64(-1)
    _check(load().lion_get_time_average(h, *[_dp(a) for a in out], ctypes.byref(end)), h)
    return out, int(end.value)


def lion_step(h, nsteps, dt):
    _check(load().lion_step(h, int(nsteps), float(dt)), h)


def lion_step_batch(h, nsteps, dts):
    d = _f64(dts)
    _check(load().lion_step_batch(h, int(nsteps), _dp(d)), h)


def lion_prepare_step(h, nsteps):
    _check(load().lion_prepare_step(h, int(nsteps)), h)


def lion_get_state(h, n):
    out = [np.empty(n) for _ in range(6)]
    t = ctypes.c_double()
    _check(load().lion_get_state(h, *[_dp(a) for a in out], ctypes.byref(t)), h)
    return dict(zip(("x", "y", "z", "vx", "vy", "vz"), out)), t.value


def lion_compute_accel(h, n):
    out = [np.empty(n) for _ in range(3)]
    _check(load().lion_compute_accel(h, *[_dp(a) for a in out]), h)
    return tuple(out)


def lion_get_energy(h):
    k, c, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load().lion_get_energy(h, ctypes.byref(k), ctypes.byref(c), ctypes.byref(d)), h)
    return k.value, c.value, d.value


def lion_check_finite(h) -> int:
    return int(load().lion_check_finite(h))


def lion_count_lost(h, r_lost_m: float) -> int:
    c = ctypes.c_int64()
    _check(load().lion_count_lost(h, float(r_lost_m), ctypes.byref(c)), h)
    return int(c.value)


def lion_last_error(h) -> str:
    m = load().lion_last_error(h)
    return m.decode() if m else ""


def lion_destroy(h):
    load().lion_destroy(h)


def lion_set_kernel_config(h, **kw):
    c = KernelConfig(**{k: int(v) for k, v in kw.items()})
    _check(load().lion_set_kernel_config(h, ctypes.byref(c)), h)


def lion_get_kernel_config(h) -> dict:
    c = KernelConfig()
    _check(load().lion_get_kernel_config(h, ctypes.byref(c)), h)
    return c.as_dict()


def lion_time_pair_kernel(h, reps) -> float:
    ms = ctypes.c_double()
    _check(load().lion_time_pair_kernel(h, int(reps), ctypes.byref(ms)), h)
    return ms.value


def lion_time_batch_kernel(h, reps, nsteps, dt) -> float:
    ms = ctypes.c_double()
    _check(load().lion_time_batch_kernel(h, int(reps), int(nsteps), float(dt), ctypes.byref(ms)),
           h)
    return ms.value


def lion_accel_noalloc(n, x_ptr, y_ptr, z_ptr, charge_ptr, mass_ptr, V_rf, Omega, U_dc, r0, z0,
                       kappa, t, precision, ax_ptr, ay_ptr, az_ptr, stream_ptr):
    """Allocation-free force evaluation; every array argument is a device
    address (int) of n doubles."""
    vp = ctypes.c_void_p
    _check(load().lion_accel_noalloc(int(n), vp(x_ptr), vp(y_ptr), vp(z_ptr), vp(charge_ptr),
                                     vp(mass_ptr), float(V_rf), float(Omega), float(U_dc),
                                     float(r0), float(z0), float(kappa), float(t),
                                     int(precision), vp(ax_ptr), vp(ay_ptr), vp(az_ptr),
                                     vp(stream_ptr)))


def lion_mathieu_to_voltages(q_x, a_x, M, Q, Omega, r0, z0, kappa):
    V0, U0 = ctypes.c_double(), ctypes.c_double()
    _check(load().lion_mathieu_to_voltages(float(q_x), float(a_x), float(M), float(Q),
                                           float(Omega), float(r0), float(z0), float(kappa),
                                           ctypes.byref(V0), ctypes.byref(U0)))
    return V0.value, U0.value


def lion_constants():
    e, eps0, amu = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    load().lion_constants(ctypes.byref(e), ctypes.byref(eps0), ctypes.byref(amu))
    return e.value, eps0.value, amu.value


# ------------------------------------------------------------ object wrapper

class Simulation:
    """One trap (or a batch of traps) on one GPU.  torch provides the device
    workspace (a uint8 tensor kept alive by this object) and the stream."""

    def __init__(self, masses, charges, precision="fp64", n_per_trap=None, device=None,
                 stream=None, autotuned=True):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the engine runs only on the GPU")
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        m, q = _f64(masses), _f64(charges)
        self.n = int(m.size)
        self.batched = n_per_trap is not None
        self.n_per_trap = (np.ascontiguousarray(n_per_trap, dtype=np.int64) if self.batched
                           else np.array([self.n], dtype=np.int64))
        self.n_traps = int(self.n_per_trap.size)
        ws = lion_workspace_bytes(self.n, self.n_traps, self.precision)
        if ws == 0:
            raise LionError(LION_ERR_ARG, "invalid sizes for workspace")
        with torch.cuda.device(self.device):
            self._ws = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
            self.stream = stream or torch.cuda.current_stream(self.device)
            base = self._ws.data_ptr()
            ptr = (base + 255) // 256 * 256
            sptr = self.stream.cuda_stream
            if self.batched:
                self.h = lion_create_batch(self.n_per_trap, m, q, self.precision, ptr, ws, sptr)
            else:
                self.h = lion_create(self.n, m, q, self.precision, ptr, ws, sptr)
        self.ws_bytes = ws
        self.tuned = None
        if autotuned:
            from . import tune

            arch = getattr(torch.cuda.get_device_properties(self.device), "gcnArchName", "")
            n_traps = len(self.n_per_trap) if self.batched else 1
            cfg = tune.lookup(arch, self.n, self.precision, self.batched, n_traps)
            if cfg:
                try:
                    self.set_config(**cfg)
                    self.tuned = cfg
                except LionError:
                    self.tuned = None

    def close(self):
        if getattr(self, "h", None):
            lion_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, x, y, z, vx, vy, vz, t=0.0):
        lion_set_state(self.h, x, y, z, vx, vy, vz, t)

    def set_trap(self, V_rf, Omega, U_dc, r0, z0, kappa, trap=-1):
        lion_set_trap(self.h, trap, V_rf, Omega, U_dc, r0, z0, kappa)

    def set_bodies(self, body_id):
        lion_set_bodies(self.h, body_id)

    def set_pseudo_trap(self, V_rf, Omega, U_dc, r0, z0, kappa, trap=-1):
        """Pseudopotential trap: the rf replaced by its static radial field."""
        lion_set_pseudo_trap(self.h, trap, V_rf, Omega, U_dc, r0, z0, kappa)

    def minimize(self, dt, dmax, ftol, max_iter=100000):
        """Damped minimisation; returns (iterations, largest |F| in N)."""
        return lion_minimize(self.h, dt, dmax, ftol, max_iter)

    def normal_modes(self, vectors=False):
        """(omega^2 ascending [3n], modes [3n, 3n] column k = mode k, or None) at
        the current positions; device scratch is a temporary torch tensor."""
        import torch

        nb = lion_normal_modes_workspace_bytes(self.h)
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        ptr = (ws.data_ptr() + 255) // 256 * 256
        try:
            return lion_normal_modes(self.h, self.n, ptr, nb, vectors)
        finally:
            torch.cuda.current_stream(self.device).synchronize()
            del ws

    def set_rigid_bodies(self, body):
        """Integrate ions with equal body id >= 0 as rigid bodies (None: off)."""
        lion_set_rigid_bodies(self.h, body)

    def rigid_state(self):
        """dict of com, com_velocity, angular_momentum [nb, 3] and quaternion [nb, 4]."""
        return lion_get_rigid_state(self.h, self.n)

    def set_species(self, species):
        lion_set_species(self.h, species)

    def set_beam(self, beam, k, gamma, species=-1):
        lion_set_beam(self.h, beam, species, k[0], k[1], k[2], gamma)

    def set_bath(self, bath, temperature, damping_time, seed, species=-1):
        lion_set_bath(self.h, bath, species, temperature, damping_time, seed)

    def set_step_index(self, steps_done):
        lion_set_step_index(self.h, steps_done)

    def step_index(self) -> int:
        return lion_get_step_index(self.h)

    def set_time_average(self, window_steps):
        """Average the velocities over windows of window_steps steps (0: off)."""
        lion_set_time_average(self.h, window_steps)

    def time_average(self):
        """((vx, vy, vz) averages of the last completed window, its end step)."""
        return lion_get_time_average(self.h, self.n)

    def set_damping(self, gamma, trap=-1):
        lion_set_damping(self.h, trap, gamma)

    def step(self, nsteps, dt):
        if np.ndim(dt):
            lion_step_batch(self.h, nsteps, dt)
        else:
            lion_step(self.h, nsteps, dt)

    def prepare_step(self, nsteps):
        """Capture the launch graphs of a following step(nsteps, ...) call
        without running it."""
        lion_prepare_step(self.h, nsteps)

    def get_state(self):
        return lion_get_state(self.h, self.n)

    def compute_accel(self):
        return lion_compute_accel(self.h, self.n)

    def energy(self):
        return lion_get_energy(self.h)

    def check_finite(self) -> int:
        return lion_check_finite(self.h)

    def count_lost(self, r_lost_m: float) -> int:
        """Ions farther than r_lost_m from the trap centre (or non-finite)."""
        return lion_count_lost(self.h, r_lost_m)

    def time_pair_kernel(self, reps: int) -> float:
        return lion_time_pair_kernel(self.h, reps)

    def time_batch_kernel(self, reps: int, nsteps: int, dt: float) -> float:
        return lion_time_batch_kernel(self.h, reps, nsteps, dt)

    def config(self) -> dict:
        return lion_get_kernel_config(self.h)

    def set_config(self, **kw):
        lion_set_kernel_config(self.h, **kw)
