#!/usr/bin/env python3
"""Benchmark of the trapped-ion hot path on one MI355X.

One step = drift + all-pairs Coulomb field + trap field + kick/damping for the
whole cloud (every kernel of the path).  Default workload: the 16384-ion
mixed-species cloud (80 % Ca-40, 20 % mass-17, sigma 200 um, 10 mK, q = 0.25),
run with FP32 pair arithmetic + FP64 accumulation (the headline value), with
plain FP64 and with compensated FP32 beside it; plus the 512-trap batch.

Prints ONE JSON line.  `value` = ordered pair interactions per second (N(N-1)
per step) of the whole job, inputs resident in HBM before timing starts.
Before the first timed configuration the GPU runs about 0.5 s of untimed pair
kernels, so that no configuration is timed from idle clocks; each then takes
its --warmup steps and exactly --steps timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Coulomb pair-interactions/s + steps/s at N=16384, FP64 vs FP32-mixed, % vector peak"
FLOP_PER_PAIR = 20  # credited: 3 sub, 3 mul/fma for r^2, rsqrt ~ 4, r^-3 x q 3, 3 fma, flop-counted
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3, "mixed_kahan": 157.3}
DTYPE = {"fp64": "f64", "mixed": "f32", "mixed_kahan": "f32"}
KERNEL_SRC = os.path.join(ROOT, "paper_1907_10514_amd", "csrc", "lion_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def profile_value(path: str, kernel_key: str, launch: dict, field: str):
    """A per-launch figure of a kernel from a committed rocprofv3 counter
    summary, or None if absent, taken on a different kernel source, or taken
    with a different launch shape."""
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("kernel_source_sha256") != kernel_source_sha():
        return None
    if any(launch.get(k) != v for k, v in ent.get("launch", {}).items()):
        return None
    return ent.get(field)


def traffic_for(kernel_key: str, launch: dict):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return profile_value(TRAFFIC_FILE, kernel_key, launch, "bytes_per_launch")


def sync(torch):
    torch.cuda.synchronize()


def warm_gpu(torch, w, seconds=0.5):
    """Untimed pair-kernel launches of workload w for about `seconds`, so that
    the first configuration timed does not start at idle clocks."""
    from paper_1907_10514_amd import runner

    sim = runner.simulation_for(w, precision="mixed")
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sim.time_pair_kernel(100)
    sim.close()
    sync(torch)


def time_single(torch, w, precision, steps, warmup, reps):
    from paper_1907_10514_amd import runner

    sim = runner.simulation_for(w, precision=precision)
    dt = w.traps[0].dt
    sim.step(warmup, dt)
    # the launch graphs of the timed call are captured and instantiated here,
    # outside the timed region (no step runs)
    sim.prepare_step(steps)
    sync(torch)
    t0 = time.perf_counter()
    sim.step(steps, dt)
    sync(torch)
    el = time.perf_counter() - t0
    finite = sim.check_finite() == 0
    chunk = chunk_times(torch, sim, dt)
    kernel_ms = sim.time_pair_kernel(reps)
    cfg = sim.config()
    sim.close()
    n = w.n
    pairs = n * (n - 1)
    return dict(pairs_per_s=pairs * steps / el, steps_per_s=steps / el,
                ms_per_step=1e3 * el / steps, chunk_ms_per_step=chunk, pair_kernel_ms=kernel_ms,
                pair_kernel_tflops=FLOP_PER_PAIR * pairs / (kernel_ms * 1e-3) / 1e12,
                pct_vector_peak=100.0 * FLOP_PER_PAIR * pairs * steps / el / 1e12
                / PEAK_TFLOPS[precision],
                finite=finite, launch=cfg)


def chunk_times(torch, sim, dt, launches=10, steps=100):
    """ms per step of single 100-step calls (one graph launch each), timed with
    events on the simulation's stream: median and min over the launches."""
    import statistics

    sim.prepare_step(steps)
    ms = []
    for _ in range(launches):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(steps, dt)
        e1.record(sim.stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1) / steps)
    return dict(median=statistics.median(ms), min=min(ms), launches=launches,
                steps_per_launch=steps)


def _parse_clocks(text):
    try:
        data = json.loads(text)
    except ValueError:
        return None
    card = next(iter(data.values()), {}) if isinstance(data, dict) else {}
    return {k: v for k, v in card.items() if "clk" in k.lower() or "clock" in k.lower()} or None


def gpu_clocks(torch=None, w=None, precision="mixed", max_s=20.0):
    """Shader and memory clocks as rocm-smi reports them.  With a workload the
    reading is taken while that workload steps on the GPU (rocm-smi runs as a
    child process meanwhile); without one, at idle.  None if the tool is
    unavailable."""
    import subprocess

    try:
        proc = subprocess.Popen(["rocm-smi", "--showclocks", "--json"], stdout=subprocess.PIPE,
                                stderr=subprocess.DEVNULL, text=True)
    except OSError:
        return None
    if torch is not None and w is not None:
        from paper_1907_10514_amd import runner

        sim = runner.simulation_for(w, precision=precision)
        t0 = time.perf_counter()
        while proc.poll() is None and time.perf_counter() - t0 < max_s:
            sim.step(500, w.traps[0].dt)
            sync(torch)
        sim.close()
    try:
        out, _ = proc.communicate(timeout=30)
    except subprocess.SubprocessError:
        proc.kill()
        proc.communicate()
        return None
    return _parse_clocks(out)


def time_batch(torch, precision, steps, warmup, seq_steps):
    import numpy as np

    import lion_inputs as li
    from paper_1907_10514_amd import runner

    w = li.batch512(nsteps=steps)
    pairs = w.ordered_pairs()
    sim = runner.simulation_for(w, precision=precision)
    # the workload runs one launch per 100 steps (the tuned shape otherwise)
    sim.set_config(**dict(sim.tuned or {}, chunk_steps=100))
    dts = runner.step_dts(w)
    sim.step(warmup, dts)
    sim.prepare_step(steps)
    sync(torch)
    t0 = time.perf_counter()
    sim.step(steps, dts)
    sync(torch)
    el = time.perf_counter() - t0
    finite = sim.check_finite() == 0
    kernel_ms = sim.time_batch_kernel(3, 100, float(dts[0]))
    cfg = sim.config()
    sim.close()
    # the same traps one by one through the single-trap path
    seq_el = 0.0
    for k in range(w.n_traps):
        o, e = int(w.offsets[k]), int(w.offsets[k + 1])
        sub = li.Workload(f"trap{k}", w.mass[o:e], w.charge[o:e], w.x[o:e], w.y[o:e], w.z[o:e],
                          w.vx[o:e], w.vy[o:e], w.vz[o:e], [w.traps[k]],
                          np.array([0, e - o], dtype=np.int64), seq_steps, w.precision)
        s1 = runner.simulation_for(sub, precision=precision, batched=False)
        s1.step(seq_steps, w.traps[k].dt)  # warm-up call of the same length
        s1.prepare_step(seq_steps)
        sync(torch)
        t0 = time.perf_counter()
        s1.step(seq_steps, w.traps[k].dt)
        sync(torch)
        seq_el += time.perf_counter() - t0
        s1.close()
    seq_pairs_per_s = pairs * seq_steps / seq_el
    return dict(pairs_per_s=pairs * steps / el, steps_per_s=steps / el,
                ms_per_step=1e3 * el / steps, kernel_ms_per_100_steps=kernel_ms,
                kernel_tflops=FLOP_PER_PAIR * pairs * 100 / (kernel_ms * 1e-3) / 1e12,
                pct_vector_peak=100.0 * FLOP_PER_PAIR * pairs * steps / el / 1e12
                / PEAK_TFLOPS[precision],
                sequential_single_trap_pairs_per_s=seq_pairs_per_s,
                speedup_vs_sequential=(pairs * steps / el) / seq_pairs_per_s,
                finite=finite, launch=cfg, n_traps=w.n_traps, n_ions=w.n,
                ordered_pairs_per_step=pairs)


def time_clusters(torch, precision, steps, warmup, reps):
    """The 65536-ion cloud with 64 rigid clusters integrated as rigid bodies:
    intra-cluster pairs left out of the pair sum (body-id exclusion mask), body
    force/torque reductions and rigid-body steps every step."""
    import numpy as np

    import lion_inputs as li
    from paper_1907_10514_amd import runner

    w = li.clusters65536()
    body = w.notes["body"]
    sizes = np.bincount(body[body >= 0])
    pairs = w.n * (w.n - 1) - int(np.sum(sizes * (sizes - 1)))
    sim = runner.simulation_for(w, precision=precision)
    sim.set_rigid_bodies(body)
    dt = w.traps[0].dt
    sim.step(warmup, dt)
    sim.prepare_step(steps)
    sync(torch)
    t0 = time.perf_counter()
    sim.step(steps, dt)
    sync(torch)
    el = time.perf_counter() - t0
    finite = sim.check_finite() == 0
    kernel_ms = sim.time_pair_kernel(reps)
    cfg = sim.config()
    sim.close()
    return dict(pairs_per_s=pairs * steps / el, steps_per_s=steps / el,
                ms_per_step=1e3 * el / steps, pair_kernel_ms=kernel_ms,
                pair_kernel_tflops=FLOP_PER_PAIR * pairs / (kernel_ms * 1e-3) / 1e12,
                pct_vector_peak=100.0 * FLOP_PER_PAIR * pairs * steps / el / 1e12
                / PEAK_TFLOPS[precision], ordered_pairs_per_step=pairs, n_ions=w.n,
                finite=finite, launch=cfg)


def time_small(torch, w, steps, oracle_steps):
    """The 8-ion and 1024-ion FP64 configurations: GPU steps/s and pairs/s over
    `steps` steps, beside the oracle on `oracle_steps` steps of the same input
    (the whole run for 8 ions; a bounded sample for 1024)."""
    import oracle

    from paper_1907_10514_amd import runner

    spec = w.traps[0]
    sim = runner.simulation_for(w, precision="fp64")
    sim.step(min(steps, 200), spec.dt)
    sim.prepare_step(steps)
    sync(torch)
    t0 = time.perf_counter()
    sim.step(steps, spec.dt)
    sync(torch)
    el = time.perf_counter() - t0
    finite = sim.check_finite() == 0
    sim.close()
    V0, U0 = oracle.voltages_for(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                 spec.r0, spec.z0, spec.kappa)
    tr = oracle.Trap(V0=V0, Omega=spec.omega, U0=U0, R0=spec.r0, Z0=spec.z0, kappa=spec.kappa)
    t0 = time.perf_counter()
    oracle.step(w.state(), w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, oracle_steps)
    oel = time.perf_counter() - t0
    pairs = w.n * (w.n - 1)
    return dict(n_ions=w.n, precision="fp64", steps=steps, steps_per_s=steps / el,
                pairs_per_s=pairs * steps / el, finite=finite,
                oracle=dict(steps=oracle_steps, steps_per_s=oracle_steps / oel,
                            pairs_per_s=pairs * (oracle_steps + 1) / oel,
                            cores=oracle.num_threads()))


def cpu_baseline_clusters(evals):
    """The FP64 oracle's field with the body-id exclusion on the 65536-ion
    cluster workload: `evals` force evaluations on the host cores (the GPU
    figure beside it is the pair kernel's, which computes the same sum)."""
    import numpy as np

    import lion_inputs as li
    import oracle

    w = li.clusters65536()
    body = w.notes["body"]
    sizes = np.bincount(body[body >= 0])
    pairs = w.n * (w.n - 1) - int(np.sum(sizes * (sizes - 1)))
    spec = w.traps[0]
    V0, U0 = oracle.voltages_for(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                 spec.r0, spec.z0, spec.kappa)
    tr = oracle.Trap(V0=V0, Omega=spec.omega, U0=U0, R0=spec.r0, Z0=spec.z0, kappa=spec.kappa)
    t0 = time.perf_counter()
    for _ in range(evals):
        oracle.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, body, tr, 0.0)
    el = time.perf_counter() - t0
    return dict(pairs_per_s=pairs * evals / el, cores=oracle.num_threads(), kind="oracle",
                sample=f"{evals} force evaluations with the exclusion mask in {el:.1f} s")


def cpu_baseline(w, seconds):
    """The FP64 oracle on the host cores, on a bounded number of steps of the
    same workload."""
    import oracle

    oracle.build(force=False)
    spec = w.traps[0]
    V0, U0 = oracle.voltages_for(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                 spec.r0, spec.z0, spec.kappa)
    tr = oracle.Trap(V0=V0, Omega=spec.omega, U0=U0, R0=spec.r0, Z0=spec.z0, kappa=spec.kappa)
    st = w.state()
    # oracle.step evaluates the starting acceleration, then one evaluation per
    # step: calibrate on one step, then time one call of k steps (k + 1 passes)
    t0 = time.perf_counter()
    oracle.step(st, w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, 1)
    per_eval = (time.perf_counter() - t0) / 2
    k = max(3, int(seconds / per_eval) - 1)
    t0 = time.perf_counter()
    oracle.step(st, w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, k)
    el = time.perf_counter() - t0
    steps, evals = k, k + 1
    n = w.n
    cores = oracle.num_threads()
    # the same oracle on one core: one step (two force evaluations)
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.step(st, w.charge, w.mass, tr, spec.gamma, 0.0, spec.dt, 1)
    el1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    return dict(value=n * (n - 1) * evals / el, unit="pair-interactions/s",
                cores=cores, kind="oracle",
                steps_per_s=steps / el,
                single_core_value=n * (n - 1) * 2 / el1,
                sample=f"{steps} steps of the {n}-ion workload in {el:.1f} s (FP64 oracle, "
                       f"OpenMP over targets; {evals} all-pairs force evaluations, each "
                       f"N(N-1) pair interactions); single_core_value: 1 step (2 evaluations) "
                       f"on one thread in {el1:.1f} s")


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def profile_pass(torch, w, precisions, batch=False):
    """Short run for counter collection: each benchmarked pair kernel (tuned
    launch shape) 5 times plus 3 steps (with batch: instead, two launches of the
    batched kernel over the 512-trap batch, 100 in-kernel steps each, then two
    over its largest trap alone, a one-workgroup launch), then a
    device-to-device copy of 256 MiB whose FETCH_SIZE / WRITE_SIZE readings
    calibrate the counters."""
    import numpy as np

    import lion_inputs as li
    from paper_1907_10514_amd import runner

    for p in precisions:
        if batch:
            wb = li.batch512(nsteps=0)
            sim = runner.simulation_for(wb, precision=p)
            sim.time_batch_kernel(2, 100, float(wb.traps[0].dt))
            torch.cuda.synchronize()
            sim.close()
            k = int(np.argmax(np.diff(wb.offsets)))
            o, e = int(wb.offsets[k]), int(wb.offsets[k + 1])
            one = li.Workload(f"trap{k}", wb.mass[o:e], wb.charge[o:e], wb.x[o:e], wb.y[o:e],
                              wb.z[o:e], wb.vx[o:e], wb.vy[o:e], wb.vz[o:e], [wb.traps[k]],
                              np.array([0, e - o], dtype=np.int64), 0, wb.precision)
            sim = runner.simulation_for(one, precision=p, batched=True)
            sim.time_batch_kernel(2, 100, float(wb.traps[k].dt))
        else:
            sim = runner.simulation_for(w, precision=p)
            sim.time_pair_kernel(5)
            sim.step(3, w.traps[0].dt)
        torch.cuda.synchronize()
        log(f"[profile] {p} launch shape {sim.config()}")
        sim.close()
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("[profile] done (copy calibration: 256 MiB read + 256 MiB written per copy)")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--seq-steps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-clusters", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 8-ion and 1024-ion configurations")
    ap.add_argument("--cluster-steps", type=int, default=200)
    ap.add_argument("--precisions", default="fp64,mixed,mixed_kahan")
    ap.add_argument("--profile-pass", action="store_true",
                    help="only launch the benchmarked pair kernels a few times and a 256 MiB "
                         "device copy (for rocprofv3 counter passes), then exit")
    ap.add_argument("--profile-batch", action="store_true",
                    help="with --profile-pass: the batched kernel over the 512-trap batch "
                         "instead of the pair kernels")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "this engine measures the path on one GPU only.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import lion_inputs as li

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    props = torch.cuda.get_device_properties(0)
    w = li.mixed16384()
    if args.profile_pass:
        profile_pass(torch, w, [p for p in args.precisions.split(",") if p], args.profile_batch)
        return
    n = w.n
    precs = [p for p in args.precisions.split(",") if p]
    res = {}
    warm_gpu(torch, w)
    for p in precs:
        log(f"[bench] {p}: N={n}, {args.warmup} warmup + {args.steps} timed steps")
        res[p] = time_single(torch, w, p, args.steps, args.warmup, args.kernel_reps)
        log(f"[bench] {p}: {res[p]['pairs_per_s']:.4e} pairs/s, {res[p]['ms_per_step']:.4f} ms/step, "
            f"pair kernel {res[p]['pair_kernel_ms']:.4f} ms")
    head = "mixed" if "mixed" in res else precs[0]
    r = res[head]
    pairs = n * (n - 1)
    kern_key = f"pair_{head}_n{n}"
    out = {
        "metric": METRIC,
        "value": r["pairs_per_s"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic",
        "config": {"workload": w.name, "n_ions": n, "precision": head,
                   "species": "80% Ca-40 + 20% mass-17 (+e)", "sigma_m": 200e-6,
                   "temperature_K": 10e-3, "q_x": 0.25, "dt_s": w.traps[0].dt,
                   "launch": r["launch"]},
        "steps_per_s": r["steps_per_s"],
        "pct_vector_peak": r["pct_vector_peak"],
        "flop_per_pair_credited": FLOP_PER_PAIR,
        "precisions": res,
    }
    if "fp64" in res and head != "fp64":
        out["speedup_mixed_over_fp64"] = r["pairs_per_s"] / res["fp64"]["pairs_per_s"]
    if "mixed_kahan" in res and "fp64" in res:
        out["speedup_kahan_over_fp64"] = res["mixed_kahan"]["pairs_per_s"] / res["fp64"]["pairs_per_s"]
    out["roofline"] = {
        "kernel": kern_key,
        "bound": "alu",
        "achieved": r["pair_kernel_tflops"],
        "peak": PEAK_TFLOPS[head],
        "unit": "TFLOP/s",
        "frac": r["pair_kernel_tflops"] / PEAK_TFLOPS[head],
        "traffic": traffic_for(kern_key, r["launch"]),
        "algorithmic_flop_per_launch": FLOP_PER_PAIR * pairs,
        "avg_launch_ms": r["pair_kernel_ms"],
    }
    # issued FLOP per launch from the VALU instruction counters (each unordered
    # pair is evaluated once, so fewer are issued than credited)
    issued = profile_value(VALU_FILE, kern_key, r["launch"], "issued_flop_per_launch")
    out["roofline"]["issued_flop_per_launch"] = issued
    out["roofline"]["issued_tflops"] = (issued / (r["pair_kernel_ms"] * 1e-3) / 1e12
                                        if issued else None)
    if not args.no_batch:
        out["batch512"] = {}
        for p in ("mixed", "fp64"):
            if p not in precs:
                continue
            log(f"[bench] batch512 {p}: {args.batch_steps} steps")
            out["batch512"][p] = time_batch(torch, p, args.batch_steps, 100, args.seq_steps)
            log(f"[bench] batch512 {p}: {out['batch512'][p]['pairs_per_s']:.4e} pairs/s, "
                f"x{out['batch512'][p]['speedup_vs_sequential']:.1f} vs one-by-one")
        if "mixed" in out["batch512"] and "fp64" in out["batch512"]:
            out["batch512"]["speedup_mixed_over_fp64"] = (
                out["batch512"]["mixed"]["pairs_per_s"] / out["batch512"]["fp64"]["pairs_per_s"])
        # the batched launch against the plain FP64 path on one 16384-ion trap
        # (pair interactions per second of each)
        if "fp64" in res:
            for p in out["batch512"]:
                if isinstance(out["batch512"][p], dict):
                    out["batch512"][p]["speedup_vs_plain_fp64_n16384"] = (
                        out["batch512"][p]["pairs_per_s"] / res["fp64"]["pairs_per_s"])
    if not args.no_clusters:
        out["clusters65536"] = {}
        for p in ("mixed", "fp64"):
            if p not in precs:
                continue
            log(f"[bench] clusters65536 {p}: {args.cluster_steps} steps")
            out["clusters65536"][p] = time_clusters(torch, p, args.cluster_steps, 20, 10)
            log(f"[bench] clusters65536 {p}: {out['clusters65536'][p]['pairs_per_s']:.4e} pairs/s, "
                f"pair kernel {out['clusters65536'][p]['pair_kernel_ms']:.3f} ms")
    if not args.no_cpu_baseline:
        # the CPU-baseline leg: the only place the oracle runs in this script
        log(f"[bench] cpu baseline: oracle for ~{args.cpu_seconds} s")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        if not args.no_clusters:
            log("[bench] clusters65536: oracle field, 2 evaluations")
            out["clusters65536"]["oracle"] = cpu_baseline_clusters(2)
        if not args.no_small:
            out["small_configs"] = {}
            for wk, steps, osteps in ((li.crystal8(), 20000, 20000), (li.crystal1024(), 50000, 2000)):
                log(f"[bench] {wk.name}: {steps} GPU steps, {osteps} oracle steps")
                out["small_configs"][wk.name] = time_small(torch, wk, steps, osteps)
                r = out["small_configs"][wk.name]
                log(f"[bench] {wk.name}: GPU {r['steps_per_s']:.0f} steps/s, "
                    f"oracle {r['oracle']['steps_per_s']:.1f} steps/s")
    out["device"] = {"name": props.name, "gcn_arch": getattr(props, "gcnArchName", ""),
                     "cu": props.multi_processor_count,
                     "clocks_under_load": gpu_clocks(torch, w, head),
                     "host_cpu": host_cpu(), "host_threads": os.cpu_count()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
