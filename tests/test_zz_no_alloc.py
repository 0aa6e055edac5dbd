"""The allocation-free force evaluation lion_accel_noalloc, called through the C
ABI with device inputs and outputs, against lion_compute_accel of a
single-trap handle on the same ions and trap (and both against the oracle),
over two calls in a row of which the second is smaller, at the maximum size,
and its refusals (which happen before any device work)."""
from __future__ import annotations

import numpy as np
import pytest

import lion_inputs as li
from tests import trajectory_bar as tb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6, "mixed_kahan": 1e-6}


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _trap(oracle, spec):
    V0, U0 = oracle.voltages_for(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                 spec.r0, spec.z0, spec.kappa)
    return oracle.Trap(V0=V0, Omega=spec.omega, U0=U0, R0=spec.r0, Z0=spec.z0, kappa=spec.kappa)


def _noalloc(torch, w, tr, t, prec):
    from paper_1907_10514_amd import lion as L

    dev = [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
           for a in (w.x, w.y, w.z, w.charge, w.mass)]
    out = [torch.empty(w.n, dtype=torch.float64, device="cuda") for _ in range(3)]
    stream = torch.cuda.current_stream()
    L.lion_accel_noalloc(w.n, *[a.data_ptr() for a in dev], tr.V0, tr.Omega, tr.U0, tr.R0,
                         tr.Z0, tr.kappa, t, L.PRECISIONS[prec], *[a.data_ptr() for a in out],
                         stream.cuda_stream)
    stream.synchronize()
    return tuple(a.cpu().numpy() for a in out)


def _handle(w, tr, t, prec):
    from paper_1907_10514_amd import Simulation

    sim = Simulation(w.mass, w.charge, prec)
    sim.set_trap(tr.V0, tr.Omega, tr.U0, tr.R0, tr.Z0, tr.kappa)
    sim.set_state(w.x, w.y, w.z, w.vx, w.vy, w.vz, t)
    a = sim.compute_accel()
    sim.close()
    return a


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_kahan"])
def test_noalloc_matches_compute_accel_two_calls(torch_gpu, oracle_mod, prec):
    """Two calls in a row, the second with fewer ions (the scratch array keeps
    the first call's contents), at t != 0 with mixed charges."""
    for n, seed in ((20000, 1), (3000, 2)):
        w = li.random_cloud(n, seed=950 + seed, sigma=80e-6, light_fraction=0.2,
                            charge_e=np.random.default_rng(seed).choice([1, 1, 2, -1], n))
        tr = _trap(oracle_mod, w.traps[0])
        t = 3.7e-8 * seed
        got = _noalloc(torch_gpu, w, tr, t, prec)
        ref = _handle(w, tr, t, prec)
        idx = np.random.default_rng(seed).choice(n, 512, replace=False)
        ox, oy, oz, sc = oracle_mod.accel_at(w.x, w.y, w.z, w.charge, w.mass, tr, t, idx)
        e_or = tb.m1([g[idx] for g in got], (ox, oy, oz), sc)
        scale = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, t)
        e_h = tb.m1(got, ref, scale)
        print(f"{prec} n={n}: M1 vs oracle {e_or:.2e}, vs lion_compute_accel {e_h:.2e}")
        assert all(np.all(np.isfinite(g)) for g in got)
        assert e_or <= TOL[prec] and e_h <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_at_maximum_size(torch_gpu, oracle_mod, prec):
    """65536 ions, the most the scratch array holds (two source slices)."""
    w = li.random_cloud(65536, seed=960, sigma=300e-6, light_fraction=0.2)
    tr = _trap(oracle_mod, w.traps[0])
    got = _noalloc(torch_gpu, w, tr, 0.0, prec)
    idx = np.concatenate([[0, w.n - 1], np.random.default_rng(9).choice(w.n, 254, replace=False)])
    ox, oy, oz, sc = oracle_mod.accel_at(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0, idx)
    err = tb.m1([g[idx] for g in got], (ox, oy, oz), sc)
    print(f"{prec} n=65536: sampled M1 vs oracle {err:.2e}")
    assert err <= TOL[prec]


def test_noalloc_refusals(torch_gpu):
    from paper_1907_10514_amd import LionError
    from paper_1907_10514_amd import lion as L

    torch = torch_gpu
    a = torch.zeros(4, dtype=torch.float64, device="cuda")
    p = a.data_ptr()
    good = dict(V_rf=9.0, Omega=li.OMEGA, U_dc=0.24, r0=li.R0, z0=li.Z0, kappa=li.KAPPA, t=0.0)
    for n, kw, prec in ((0, {}, 0), (65537, {}, 0), (4, dict(r0=0.0), 0), (4, {}, 3),
                        (4, dict(t=float("nan")), 1)):
        args = dict(good, **kw)
        with pytest.raises(LionError) as ei:
            L.lion_accel_noalloc(n, p, p, p, p, p, args["V_rf"], args["Omega"], args["U_dc"],
                                 args["r0"], args["z0"], args["kappa"], args["t"], prec, p, p, p,
                                 None)
        assert ei.value.code == L.LION_ERR_ARG
        assert "lion_accel_noalloc" in L.lion_last_error(None)
    with pytest.raises(LionError) as ei:
        L.lion_accel_noalloc(4, 0, p, p, p, p, 9.0, li.OMEGA, 0.24, li.R0, li.Z0, li.KAPPA, 0.0,
                             0, p, p, p, None)
    assert ei.value.code == L.LION_ERR_ARG
