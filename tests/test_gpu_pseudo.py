"""Pseudopotential trap and energy minimisation on the GPU against the oracle."""
from __future__ import annotations

import math

import numpy as np
import pytest

import lion_inputs as li
from tests import analytic

pytestmark = pytest.mark.gpu

CA, E = li.REF_MASS, li.E_CHARGE
TOL = {"fp64": 1e-12, "mixed": 1e-6, "mixed_kahan": 1e-6}


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _pseudo(oracle, q_x=0.3, a_x=-0.001):
    V0, U0 = oracle.voltages_for(q_x, a_x, CA, E, li.OMEGA, li.R0, li.Z0, li.KAPPA)
    return oracle.Trap(V0=V0, Omega=li.OMEGA, U0=U0, R0=li.R0, Z0=li.Z0, kappa=li.KAPPA,
                       pseudo=True)


def _sim(mass, charge, prec, tr, st, gamma=0.0, n_per_trap=None, **cfg):
    from paper_1907_10514_amd import Simulation

    if cfg.get("symmetric") == 1:
        cfg.setdefault("step_launches", 2)  # the all-pairs pair kernel and its epilogue
    sim = Simulation(mass, charge, prec, n_per_trap=n_per_trap)
    if cfg:
        sim.set_config(**cfg)
    sim.set_pseudo_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)
    sim.set_damping(gamma)
    sim.set_state(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], 0.0)
    return sim


def _m1(a, r, scale):
    return float(np.max(np.sqrt(sum((a[c] - r[c]) ** 2 for c in range(3))) / scale))


def _length_scale(tr):
    wz2 = 2 * E * tr.kappa * tr.U0 / (CA * tr.Z0 ** 2)
    return (E * E / (4 * math.pi * analytic.EPS0 * CA * wz2)) ** (1 / 3), CA * wz2


@pytest.mark.parametrize("prec,sym", [("fp64", 1), ("mixed", 1), ("mixed_kahan", 1),
                                      ("fp64", 2), ("mixed", 2), ("mixed_kahan", 2)])
@pytest.mark.parametrize("n", [1, 257, 4097])
def test_pseudo_accel_parity(torch_gpu, oracle_mod, n, prec, sym):
    """Two species in the pseudopotential trap: one force evaluation, on the
    all-pairs (sym 1) and the pair-once (sym 2) kernels."""
    w = li.random_cloud(n, seed=400 + n, sigma=60e-6, light_fraction=0.3)
    tr = _pseudo(oracle_mod)
    sim = _sim(w.mass, w.charge, prec, tr, w.state(), symmetric=sym)
    a = sim.compute_accel()
    r = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    err = _m1(a, r, sc)
    print(f"pseudo n={n} {prec} M1={err:.2e}")
    assert err <= TOL[prec]
    sim.close()


@pytest.mark.parametrize("n_max", [300, 32, 16])
def test_pseudo_batch_accel_parity(torch_gpu, oracle_mod, n_max):
    """Batched pseudopotential traps: the batched kernel (traps of up to 300
    ions) and the wave kernel (up to 32 ions on 256 threads, up to 16 on one
    wave)."""
    w = li.batch512(n_traps=10, n_min=2, n_max=n_max, seed=41, nsteps=0)
    trs = [_pseudo(oracle_mod, s.q_x, s.a_x) for s in w.traps]
    from paper_1907_10514_amd import Simulation

    for prec in TOL:
        sim = Simulation(w.mass, w.charge, prec, n_per_trap=np.diff(w.offsets))
        for k, tr in enumerate(trs):
            sim.set_pseudo_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa, trap=k)
        sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, 0.0)
        a = sim.compute_accel()
        r = oracle_mod.accel_batch(w.offsets, w.x, w.y, w.z, w.charge, w.mass, trs,
                                   np.zeros(w.n_traps))
        for k, tr in enumerate(trs):
            o, e = w.offsets[k], w.offsets[k + 1]
            sc = oracle_mod.accel_scale(w.x[o:e], w.y[o:e], w.z[o:e], w.charge[o:e],
                                        w.mass[o:e], tr, 0.0)
            assert _m1([c[o:e] for c in a], [c[o:e] for c in r], sc) <= TOL[prec], (prec, k)
        sim.close()


def test_pseudo_single_ions_follow_oracle(torch_gpu, oracle_mod):
    """One Ca-40 and one 17 u ion far apart (Coulomb coupling negligible is not
    assumed: the oracle includes it) over 3000 steps."""
    tr = _pseudo(oracle_mod)
    st = {"x": np.array([3e-6, -40e-6]), "y": np.array([-2e-6, 30e-6]),
          "z": np.array([5e-6, -60e-6]), "vx": np.array([0.4, -0.1]),
          "vy": np.array([0.7, 0.2]), "vz": np.array([-0.3, 0.5])}
    m = np.array([CA, 17 * li.AMU])
    q = np.array([E, E])
    sim = _sim(m, q, "fp64", tr, st)
    sim.step(3000, li.DT)
    got, _ = sim.get_state()
    ref = oracle_mod.step(st, q, m, tr, 0.0, 0.0, li.DT, 3000)
    for k in ("x", "y", "z"):
        assert np.max(np.abs(got[k] - ref[k])) < 1e-11 * 60e-6, k
    sim.close()


def test_pseudo_energy_matches_oracle(torch_gpu, oracle_mod):
    w = li.random_cloud(500, seed=9, sigma=40e-6, light_fraction=0.3)
    tr = _pseudo(oracle_mod)
    sim = _sim(w.mass, w.charge, "fp64", tr, w.state())
    k, c, d = sim.energy()
    ko, co, do = oracle_mod.energy(w.state(), w.charge, w.mass, tr)
    assert k == pytest.approx(ko, rel=1e-13, abs=0)
    assert c == pytest.approx(co, rel=1e-12, abs=0)
    assert d == pytest.approx(do, rel=1e-12, abs=0)
    sim.close()


def _chain_start(n, seed):
    rng = np.random.default_rng(seed)
    st = {k: np.zeros(n) for k in ("vx", "vy", "vz")}
    st["z"] = np.linspace(-1.0, 1.0, n) * 12e-6 * max(n - 1, 1) ** 0.7 + rng.normal(0, 1e-6, n)
    st["x"] = rng.normal(0, 1e-6, n)
    st["y"] = rng.normal(0, 1e-6, n)
    return st


@pytest.mark.parametrize("prec,ftol,tol", [("fp64", 1e-10, 1e-8), ("mixed", 1e-5, 1e-4),
                                           ("mixed_kahan", 1e-5, 1e-4)])
@pytest.mark.parametrize("n,sym", [(2, 1), (5, 1), (10, 1), (10, 2)])
def test_minimised_chain(torch_gpu, oracle_mod, n, sym, prec, ftol, tol):
    """Minimising from a scattered start gives the linear chain: sorted axial
    positions equal the Newton roots of the axial force balance (and the
    oracle's minimiser), on the all-pairs and the pair-once kernels.  The FP32
    pair path cannot resolve forces below ~1e-7 of the force scale, so it
    stops at a looser force tolerance."""
    tr = _pseudo(oracle_mod)
    l, k = _length_scale(tr)
    fu = k * l
    st = _chain_start(n, seed=n)
    m, q = np.full(n, CA), np.full(n, E)
    sim = _sim(m, q, prec, tr, st, symmetric=sym)
    it, fmax = sim.minimize(dt=2e-8, dmax=1e-6, ftol=ftol * fu, max_iter=200000)
    got, _ = sim.get_state()
    assert fmax <= ftol * fu
    u = np.sort(got["z"]) / l
    ref = oracle_mod.minimize(st, q, m, tr, dt=2e-8, dmax=1e-6, ftol=ftol * fu, max_iter=200000)
    print(f"chain n={n} {prec}: {it} iterations (oracle {ref['iterations']}), "
          f"max |u - newton| {np.max(np.abs(u - analytic.chain_equilibrium(n))):.2e}")
    assert np.max(np.abs(u - analytic.chain_equilibrium(n))) < tol
    assert np.max(np.abs(u - np.sort(ref["z"]) / l)) < tol
    sim.close()


def test_minimised_crystal_is_a_minimum_of_the_oracle_energy(torch_gpu, oracle_mod):
    """A 200-ion two-species cloud minimised on the GPU (FP64): at the result
    the oracle's force is below tolerance, and the oracle's energy rises along
    random small displacements."""
    w = li.random_cloud(200, seed=23, sigma=30e-6, light_fraction=0.3)
    tr = _pseudo(oracle_mod)
    l, k = _length_scale(tr)
    fu = k * l
    st = w.state()
    for c in ("vx", "vy", "vz"):
        st[c] = np.zeros(w.n)
    sim = _sim(w.mass, w.charge, "fp64", tr, st)
    it, fmax = sim.minimize(dt=2e-8, dmax=1e-6, ftol=1e-9 * fu, max_iter=500000)
    got, _ = sim.get_state()
    ax, ay, az = oracle_mod.accel(got["x"], got["y"], got["z"], w.charge, w.mass, tr, 0.0)
    f = w.mass * np.sqrt(ax * ax + ay * ay + az * az)
    print(f"crystal: {it} iterations, GPU fmax {fmax / fu:.2e}, oracle fmax {f.max() / fu:.2e} (force units)")
    assert f.max() <= 2e-9 * fu

    def pot(s):
        return sum(oracle_mod.energy(s, w.charge, w.mass, tr)[1:])

    e0 = pot(got)
    rng = np.random.default_rng(5)
    for _ in range(10):
        d = rng.normal(size=(3, w.n)) * 1e-3 * l
        assert pot(dict(got, x=got["x"] + d[0], y=got["y"] + d[1], z=got["z"] + d[2])) > e0
    sim.close()


def test_minimize_rejections(torch_gpu, oracle_mod):
    from paper_1907_10514_amd import LionError, Simulation
    from paper_1907_10514_amd import lion as L

    tr = _pseudo(oracle_mod)
    st = _chain_start(4, seed=1)
    m, q = np.full(4, CA), np.full(4, E)
    sim = Simulation(m, q, "fp64")
    with pytest.raises(LionError) as ei:
        sim.minimize(1e-8, 1e-6, 0.0)
    assert ei.value.code == L.LION_ERR_STATE
    sim.set_state(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], 0.0)
    sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)  # full rf field
    with pytest.raises(LionError) as ei:
        sim.minimize(1e-8, 1e-6, 0.0)
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    sim.set_pseudo_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)
    for bad in ((0.0, 1e-6, 0.0), (1e-8, -1.0, 0.0), (1e-8, 1e-6, -1.0)):
        with pytest.raises(LionError) as ei:
            sim.minimize(*bad)
        assert ei.value.code == L.LION_ERR_ARG
    it, _ = sim.minimize(1e-8, 1e-6, 0.0, max_iter=7)
    assert it == 7
    sim.set_rigid_bodies([0, 0, -1, -1])
    with pytest.raises(LionError) as ei:
        sim.minimize(1e-8, 1e-6, 0.0)
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    sim.close()
    bat = Simulation(np.full(4, CA), np.full(4, E), "fp64", n_per_trap=[2, 2])
    bat.set_pseudo_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)
    bat.set_state(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], 0.0)
    with pytest.raises(LionError) as ei:
        bat.minimize(1e-8, 1e-6, 0.0)
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    bat.close()


# ------------------------------------------------------------------ normal modes

def _modes_case(oracle_mod, kind):
    tr = _pseudo(oracle_mod)
    l, k = _length_scale(tr)
    fu = k * l
    if kind == "chain6":
        st = _chain_start(6, seed=6)
        m, q = np.full(6, CA), np.full(6, E)
        st = oracle_mod.minimize(st, q, m, tr, dt=2e-8, dmax=1e-6, ftol=1e-11 * fu,
                                 max_iter=400000)
    elif kind == "crystal60":
        w = li.random_cloud(60, seed=61, sigma=20e-6, light_fraction=0.3)
        m, q = w.mass, w.charge
        st = w.state()
        for c in ("vx", "vy", "vz"):
            st[c] = np.zeros(60)
        st = oracle_mod.minimize(st, q, m, tr, dt=2e-8, dmax=1e-6, ftol=1e-10 * fu,
                                 max_iter=800000)
    else:  # an unrelaxed 512-ion two-species cloud (modes of a saddle: some omega^2 < 0)
        w = li.random_cloud(512, seed=62, sigma=40e-6, light_fraction=0.3)
        m, q, st = w.mass, w.charge, w.state()
    return tr, m, q, st


@pytest.mark.parametrize("kind", ["chain6", "crystal60", "cloud512"])
def test_normal_modes_match_oracle(torch_gpu, oracle_mod, kind):
    """Eigenvalues of the GPU's mass-weighted Hessian (HIP kernel + rocSOLVER)
    against the oracle's (plain loops + numpy eigh) at the same positions;
    eigenvectors satisfy D v = omega^2 v with the oracle's D and are
    orthonormal."""
    tr, m, q, st = _modes_case(oracle_mod, kind)
    sim = _sim(m, q, "fp64", tr, st)
    w2, V = sim.normal_modes(vectors=True)
    ref, _ = oracle_mod.normal_modes(st["x"], st["y"], st["z"], q, m, tr)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(w2 - ref))
    print(f"{kind}: max |omega^2 - oracle| / max|omega^2| = {err / scale:.2e}")
    assert err < 1e-12 * scale
    D = oracle_mod.hessian(st["x"], st["y"], st["z"], q, m, tr)
    assert np.max(np.abs(D @ V - V * w2)) < 1e-11 * scale
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[0]))) < 1e-11
    if kind != "cloud512":
        assert np.min(w2) > 0
    sim.close()


def test_normal_modes_single_ion_and_rejections(torch_gpu, oracle_mod):
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    tr = _pseudo(oracle_mod)
    st = {"x": np.array([1e-6]), "y": np.array([2e-6]), "z": np.array([-1e-6]),
          "vx": np.zeros(1), "vy": np.zeros(1), "vz": np.zeros(1)}
    m = 17 * li.AMU
    sim = _sim(np.array([m]), np.array([E]), "fp64", tr, st)
    w2, _ = sim.normal_modes()
    q_x, a_x = oracle_mod.mathieu_coefficients(tr.V0, tr.U0, m, E, tr.Omega, tr.R0, tr.Z0,
                                               tr.kappa)
    wr = oracle_mod.pseudopotential_frequency(q_x, a_x, tr.Omega)
    wz = oracle_mod.pseudopotential_frequency(0.0, -2 * a_x, tr.Omega)
    assert np.allclose(w2, np.sort([wz ** 2, wr ** 2, wr ** 2]), rtol=1e-12, atol=0)
    sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)  # full rf: no static modes
    with pytest.raises(LionError) as ei:
        sim.normal_modes()
    assert ei.value.code == L.LION_ERR_UNSUPPORTED
    sim.set_pseudo_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)
    import torch

    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(LionError) as ei:
        L.lion_normal_modes(sim.h, 1, small.data_ptr(), 256)
    assert ei.value.code == L.LION_ERR_WORKSPACE
    sim.close()


def test_normal_modes_workspace_holds_the_solver_scratch(torch_gpu, oracle_mod):
    """The solver's scratch is part of the caller's workspace: the size asked of
    the handle covers the Hessian, two vectors and the rocSOLVER scratch; one
    byte less than the Hessian part is refused, and the full size works twice
    in a row on one handle (one rocBLAS handle per simulation)."""
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L
    import torch

    tr, m, q, st = _modes_case(oracle_mod, "chain6")
    sim = _sim(m, q, "fp64", tr, st)
    n = len(m)
    up = lambda b: (b + 255) // 256 * 256  # noqa: E731
    fixed = up((3 * n) ** 2 * 8) + 2 * up(3 * n * 8) + up(4)
    nb = L.lion_normal_modes_workspace_bytes(sim.h)
    assert nb > fixed
    buf = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    ptr = (buf.data_ptr() + 255) // 256 * 256
    with pytest.raises(LionError) as ei:
        L.lion_normal_modes(sim.h, n, ptr, fixed - 1)
    assert ei.value.code == L.LION_ERR_WORKSPACE
    ref, _ = oracle_mod.normal_modes(st["x"], st["y"], st["z"], q, m, tr)
    for vectors in (True, False):
        w2, _ = L.lion_normal_modes(sim.h, n, ptr, nb, vectors)
        assert np.max(np.abs(w2 - ref)) < 1e-12 * np.max(np.abs(ref))
    sim.close()
