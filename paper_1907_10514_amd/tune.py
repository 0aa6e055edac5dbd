"""Autotuner for the launch shapes of the pair kernels and the batched kernel.

For a given workload size and precision it times every candidate launch shape
(targets per lane I, source slices J, FP32 run length L, LDS or scalar source
feed, pair-once kernel variant, one launch per step or pair kernel + epilogue;
for batches the workgroup size per trap and the
targets per thread) with the library's own kernel timer, rejects candidates
whose forces differ from the FP64 path by more than half the precision's bar on
a validation cloud (for batches, on every trap of the batch), times the fastest again as whole
steps (median of three runs, then the steps per captured graph), and stores the
winner in a JSON cache keyed by (GPU arch, ROCm version, size bucket, precision,
single trap or batch shape).  ``Simulation`` applies a cached shape when one
exists.

Usage:  python -m paper_1907_10514_amd.tune [--n 16384] [--precision mixed]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import time

import numpy as np

from . import lion as L

CACHE_ENV = "LION_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
BAR = {L.LION_FP64: 1e-12, L.LION_MIXED_F64ACC: 1e-6, L.LION_MIXED_KAHAN: 1e-6}
# largest single trap for which the one-launch step is a candidate (its workgroups
# each read every source, so it loses to the pair kernels well before this)
ONE_LAUNCH_MAX = 8192


def cache_path() -> str:
    return os.environ.get(CACHE_ENV, DEFAULT_CACHE)


def size_bucket(n: int) -> int:
    """Power-of-two bucket of the ion count (a shape tuned at 16384 serves 12k..23k)."""
    return int(2 ** round(np.log2(max(int(n), 1))))


def rocm_version() -> str:
    """major.minor of the HIP runtime torch was built with ("" if unknown)."""
    try:
        import torch

        return ".".join((torch.version.hip or "").split(".")[:2])
    except ImportError:
        return ""


def cache_key(arch: str, n: int, precision: int, batched: bool, n_traps: int = 1,
              rocm: str | None = None) -> str:
    """(GPU arch, ROCm version, ion-count bucket, precision, single trap or batch
    of n_traps traps)."""
    rocm = rocm_version() if rocm is None else rocm
    shape = f"batch{int(n_traps)}" if batched else "single"
    return f"{arch.split(':')[0]}|rocm{rocm}|n{size_bucket(n)}|p{int(precision)}|{shape}"


def load_cache(path: str | None = None) -> dict:
    try:
        with open(path or cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(arch: str, n: int, precision: int, batched: bool, n_traps: int = 1) -> dict | None:
    ent = load_cache().get(cache_key(arch, n, precision, batched, n_traps))
    return ent.get("config") if ent else None


def _arch() -> str:
    import torch

    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "unknown")


def _scale(x, y, z, q_e):
    """Sum of |q_j| / r_ij^2 per target (field scale, units of e/m^2) on the host."""
    p = np.stack([x, y, z], 1)
    out = np.empty(x.size)
    for a in range(0, x.size, 256):
        d = p[a:a + 256, None, :] - p[None, :, :]
        r2 = np.sum(d * d, -1)
        r2[r2 == 0] = np.inf
        out[a:a + 256] = np.sum(np.abs(q_e)[None, :] / r2, 1)
    return out


def single_candidates(n: int, precision: int):
    """Pair kernel + epilogue shapes (step_launches=2); the one-launch step,
    which has no pair kernel of its own, is timed with the whole steps."""
    for cfg in _two_launch_candidates(n, precision):
        yield dict(cfg, step_launches=2)


def _two_launch_candidates(n: int, precision: int):
    js = [j for j in (1, 2, 4, 8, 12, 16, 24, 32, 48, 64)]
    if precision == L.LION_FP64:
        for i, j in itertools.product((1, 2, 4), js):
            yield dict(i_per_lane=i, j_split=j, symmetric=1)
        if (n + 255) // 256 <= 512:
            for v in (1, 2, 3, 5, 6, 7):
                yield dict(symmetric=2, sym_variant=v)
    elif precision == L.LION_MIXED_F64ACC:
        for i, j, fl, lds in itertools.product((1, 2, 4), js, (8, 16), (1, 2)):
            yield dict(i_per_lane=i, j_split=j, flush_len=fl, lds_sources=lds, symmetric=1)
        if (n + 255) // 256 <= 512:
            for v in (1, 2, 4, 5, 6, 7, 8, 9):
                yield dict(symmetric=2, sym_variant=v)
    else:
        for i, j, lds in itertools.product((1, 2, 4), js, (1, 2)):
            yield dict(i_per_lane=i, j_split=j, lds_sources=lds, symmetric=1)
        if (n + 255) // 256 <= 512:
            yield dict(symmetric=2)


def _cloud(n, seed=12345, sigma=200e-6):
    rng = np.random.default_rng(seed)
    x, y, z = rng.normal(0, sigma, (3, n))
    return x, y, z


def tune_single(n: int, precision: int, reps: int = 20, verbose: bool = True,
                top_steps: int = 12, step_reps: int = 1000) -> dict:
    """Time every candidate for a single trap of n ions; returns the best entry."""
    e, _, amu = L.lion_constants()
    mass = np.full(n, 40 * amu)
    charge = np.full(n, e)
    x, y, z = _cloud(n)
    zeros = np.zeros(n)
    sim = L.Simulation(mass, charge, precision, stream=None, autotuned=False)
    sim.set_trap(9.0, 2 * np.pi * 3.85e6, 0.24, 0.5e-3, 1e-3, 0.25)
    sim.set_state(x, y, z, zeros, zeros, zeros)
    # validation cloud (smaller) against the FP64 path
    nv = min(n, 2048)
    xv, yv, zv = _cloud(nv, seed=7)
    ref = L.Simulation(np.full(nv, 40 * amu), np.full(nv, e), L.LION_FP64, autotuned=False)
    ref.set_state(xv, yv, zv, np.zeros(nv), np.zeros(nv), np.zeros(nv))
    a_ref = np.array(ref.compute_accel())
    ref.close()
    k_scale = (e / (40 * amu)) * e / (4 * np.pi * 8.8541878128e-12)
    sc = k_scale * _scale(xv, yv, zv, np.ones(nv))
    val = L.Simulation(np.full(nv, 40 * amu), np.full(nv, e), precision, autotuned=False)
    val.set_state(xv, yv, zv, np.zeros(nv), np.zeros(nv), np.zeros(nv))
    results = []
    for cfg in single_candidates(n, precision):
        try:
            sim.set_config(**cfg)
            vcfg = dict(cfg)
            if "j_split" in vcfg:
                vcfg["j_split"] = min(cfg["j_split"], max(1, (nv + 63) // 64))
            val.set_config(**vcfg)
        except L.LionError:
            continue
        a = np.array(val.compute_accel())
        err = float(np.max(np.linalg.norm(a - a_ref, axis=0) / sc))
        ms = sim.time_pair_kernel(reps)
        ent = dict(config=cfg, pair_ms=ms, m1_vs_fp64=err, ok=err <= BAR[precision] * 0.5)
        results.append(ent)
        if verbose:
            print(f"  {cfg} -> {ms * 1e3:8.2f} us  M1 {err:.2e}{'' if ent['ok'] else '  REJECT'}",
                  flush=True)
    # the fastest pair kernels are timed again as whole steps (pair + epilogue +
    # launch gaps): more source slices shorten the pair kernel but lengthen the
    # epilogue's partial-sum reads
    import torch

    ok = sorted([r for r in results if r["ok"]], key=lambda r: r["pair_ms"])[:top_steps]
    dt = 1.0 / 3.85e6 / 20

    def median_step_ms(cfg):
        sim.set_config(**cfg)
        sim.step(200, dt)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            sim.step(step_reps, dt)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0) / step_reps)
        return sorted(times)[1]

    # one launch per step (up to ONE_LAUNCH_MAX ions), accuracy-gated like the rest
    if n <= ONE_LAUNCH_MAX:
        cfg = dict(step_launches=1)
        sim.set_config(**cfg)
        val.set_config(**cfg)
        a = np.array(val.compute_accel())
        err = float(np.max(np.linalg.norm(a - a_ref, axis=0) / sc))
        ent = dict(config=cfg, pair_ms=None, m1_vs_fp64=err, ok=err <= BAR[precision] * 0.5)
        results.append(ent)
        if ent["ok"]:
            ok.append(ent)
        elif verbose:
            print(f"  {cfg} M1 {err:.2e}  REJECT", flush=True)
    for r in ok:
        r["step_ms"] = median_step_ms(r["config"])
        if verbose:
            print(f"  step {r['config']} -> {r['step_ms'] * 1e3:8.2f} us/step", flush=True)
    best = min(ok, key=lambda r: r["step_ms"])
    # steps per captured graph for the winning shape
    for steps in (50, 200):
        cfg = dict(best["config"], chunk_steps=steps)
        ms = median_step_ms(cfg)
        if verbose:
            print(f"  step {cfg} -> {ms * 1e3:8.2f} us/step", flush=True)
        if ms < best["step_ms"]:
            best = dict(best, config=cfg, step_ms=ms)
    sim.close()
    val.close()
    return dict(best=best, n=n, precision=precision, candidates=len(results))


def batch_candidates():
    """Workgroup size per trap x targets per thread for traps of >= 128 ions
    (at most 2 with 1024 threads)."""
    for block in (256, 512, 1024):
        for tpt in (1, 2, 4):
            if block == 1024 and tpt == 4:
                continue
            yield dict(batch_block=block, batch_tpt=tpt)


def _batch_scale(npt, x, y, z):
    """Per-ion Coulomb field scale sum_j |q_j| / r_ij^2 within each trap (units
    e/m^2; all ions carry +e)."""
    out = np.empty(x.size)
    o = 0
    for m in np.asarray(npt, dtype=np.int64):
        sl = slice(o, o + int(m))
        out[sl] = _scale(x[sl], y[sl], z[sl], np.ones(int(m)))
        o += int(m)
    return out


def tune_batch(n_per_trap, precision: int, steps: int = 100, verbose: bool = True) -> dict:
    """Time every batch launch shape on a batch of the given trap sizes, reject
    shapes whose forces differ from the FP64 batched path by more than half the
    precision's bar (M1 against the Coulomb scale of each ion, all traps),
    then time the steps per captured launch (chunk_steps) for the winner."""
    import torch

    e, _, amu = L.lion_constants()
    npt = np.asarray(n_per_trap, dtype=np.int64)
    n = int(npt.sum())
    x, y, z = _cloud(n, sigma=20e-6)
    zeros = np.zeros(n)
    trap = (9.0, 2 * np.pi * 3.85e6, 0.24, 0.5e-3, 1e-3, 0.25)
    dt = 1.0 / 3.85e6 / 20

    def make(prec):
        sim = L.Simulation(np.full(n, 40 * amu), np.full(n, e), prec, n_per_trap=npt,
                           autotuned=False)
        sim.set_trap(*trap)
        sim.set_state(x, y, z, zeros, zeros, zeros)
        return sim

    ref = make(L.LION_FP64)
    a_ref = np.array(ref.compute_accel())
    ref.close()
    k_scale = (e / (40 * amu)) * e / (4 * np.pi * 8.8541878128e-12)
    sc = k_scale * _batch_scale(npt, x, y, z)
    res = []
    sim = make(precision)
    for cfg in batch_candidates():
        sim.set_config(**cfg)
        sim.set_state(x, y, z, zeros, zeros, zeros)
        err = float(np.max(np.linalg.norm(np.array(sim.compute_accel()) - a_ref, axis=0) / sc))
        sim.time_batch_kernel(1, 10, dt)
        ms = min(sim.time_batch_kernel(3, steps, dt) for _ in range(2))
        ent = dict(config=cfg, kernel_ms=ms, m1_vs_fp64=err, ok=err <= BAR[precision] * 0.5)
        res.append(ent)
        if verbose:
            print(f"  {cfg} -> {ms:.3f} ms / {steps} steps  M1 {err:.2e}"
                  f"{'' if ent['ok'] else '  REJECT'}", flush=True)
    best = min([r for r in res if r["ok"]], key=lambda r: r["kernel_ms"])

    def step_ms(cfg):
        sim.set_config(**cfg)
        sim.set_state(x, y, z, zeros, zeros, zeros)
        sim.step(200, dt)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            sim.step(1000, dt)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0) / 1000)
        return sorted(times)[1]

    best["step_ms"] = step_ms(best["config"])
    for steps_per_launch in (50, 200):
        cfg = dict(best["config"], chunk_steps=steps_per_launch)
        ms = step_ms(cfg)
        if verbose:
            print(f"  step {cfg} -> {ms * 1e3:8.2f} us/step", flush=True)
        if ms < best["step_ms"]:
            best = dict(best, config=cfg, step_ms=ms)
    sim.close()
    return dict(best=best, n=n, precision=precision, candidates=len(res))


def store(key: str, entry: dict, path: str | None = None):
    path = path or cache_path()
    data = load_cache(path)
    data[key] = dict(config=entry["best"]["config"], measured=entry["best"],
                     tuned_at=time.strftime("%Y-%m-%d %H:%M:%S"))
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="*", default=[16384])
    ap.add_argument("--precision", nargs="*", default=["fp64", "mixed", "mixed_kahan"])
    ap.add_argument("--batch", action="store_true", help="tune the 512-trap batch instead")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    arch = _arch()
    for pname in args.precision:
        p = L.PRECISIONS[pname]
        if args.batch:
            rng = np.random.Generator(np.random.PCG64(3))
            npt = rng.integers(2, 513, size=512)
            print(f"[tune] batch {pname}", flush=True)
            r = tune_batch(npt, p)
            store(cache_key(arch, int(npt.sum()), p, True, npt.size), r)
            print(f"[tune] best {r['best']}", flush=True)
            continue
        for n in args.n:
            print(f"[tune] n={n} {pname}", flush=True)
            r = tune_single(n, p, reps=args.reps)
            store(cache_key(arch, n, p, False), r)
            print(f"[tune] best {r['best']}", flush=True)


if __name__ == "__main__":
    main()
