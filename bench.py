"""Benchmark of the DABA iteration on one MI355X.

One step = one DABA iteration (Algorithm 1's loop body) over the whole
synthetic problem.  Default workload: 20,000 cameras, 10,000,000 landmarks,
~60M observations (track lengths 2 + Geometric(1/5)), 64 camera partitions,
Huber loss: the largest configuration of the metric, FP64 against
FP32-mixed at equal final objective.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload cam20k-lm10m]
                  [--no-cpu-baseline] [--no-fp32] [--no-attainable] [--copy-calibration MB]
                  [--surrogate entity|partition]

--surrogate partition measures the device surrogate of eq. Ealpha instead
(include/daba_part.h; its own JSON line, at most 20 timed iterations).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP64_VECTOR_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


SURVEY_BYTES_PER_OBS = 260.0   # whole iteration, reference design with a contribution buffer, S > 1


def kernel_bytes(prob, S: int, T: int, fp32: bool) -> dict:
    """Algorithmic HBM bytes one launch of each observation-pass kernel must
    move (FP64 / FP32-mixed):

    k_tiles, per observation: the pixel (16 / 8), the landmark index (4) and
    the used part of the landmark's pair record, l^k, partition, l^(k-1)
    (52 / 28); per tile: three camera records read (3 x 120), the 76 moment
    and 2 share sums written (624) and the partition bins (16 S).

    k_lms, per observation: the pixel and the camera index at the slot
    (16 / 8 + 4); per landmark: its pair record read (52) and both candidate
    records written (2 x 56, plus 2 x 28 for the FP32 copies) (the two sums
    per block, about 16 bytes per 1,000 observations, are left out).  The
    camera records each observation gathers (2 x 128 / 128 bytes) come from
    cache and are counted apart."""
    K, N = prob["n_obs"], prob["n_landmarks"]
    tiles = ((8 if fp32 else 16) + 4 + (28 if fp32 else 52)) * K + (3 * 120 + 78 * 8 + 16 * S) * T
    lms = ((8 if fp32 else 16) + 4) * K + (52 + 2 * 56 + (2 * 28 if fp32 else 0)) * N
    cache = (128 if fp32 else 256) * K
    return {"k_tiles": float(tiles), "k_lms": float(lms), "k_lms_camera_gathers_from_cache": float(cache)}


_CSRC = os.path.join(ROOT, "paper_2305_07026_amd", "csrc")
# the iteration's kernels and the device headers they include
KERNEL_SOURCES = tuple(os.path.join(_CSRC, f) for f in ("daba_kernels.hip", "daba_internal.h", "daba_rotation.h",
                                                   "daba_eval.h"))


def source_digest(paths=KERNEL_SOURCES) -> str:
    """SHA-256 of the code of the given source files: comments, trailing
    blanks and empty lines removed, so that only a change of code changes
    it."""
    import hashlib
    import re
    h = hashlib.sha256()
    for path in ([paths] if isinstance(paths, str) else paths):
        t = open(path).read()
        t = re.sub(r"/\*.*?\*/", "", t, flags=re.S)
        t = re.sub(r"//[^\n]*", "", t)
        h.update("\n".join(line.rstrip() for line in t.splitlines() if line.strip()).encode())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (calibrated against a device copy), if
    they were taken on the kernel code as it is now; else None."""
    rec = os.path.join(ROOT, "profiles", f"{kernel}_traffic_{workload}_{precision}.json")
    if not os.path.exists(rec):
        return None
    t = json.load(open(rec))
    if source_digest() != t.get("kernel_code_sha256"):
        return None
    return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]


def n_tiles(prob) -> int:
    """Camera tiles of the layout: each camera's observations in pieces of at
    most 1,024."""
    cnt = __import__("numpy").bincount(prob["obs_camera"], minlength=prob["n_cameras"])
    return int(sum(-(-int(c) // 1024) for c in cnt))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def equal_objective(prob, ms64, ms32, iters, S, make):
    """Speedup of FP32-mixed over FP64 in time to F_target =
    F_64 + 1e-4 (F_init - F_64) (the paper's time-to-target metric with
    Delta = 1e-4), F_64 the FP64 objective after `iters` iterations."""
    import numpy as np
    a = make("fp64")
    F0 = a.objective()
    F64 = a.iterate(iters)
    b = make("fp32_mixed")
    F32a = b.iterate(iters)
    # the FP32-mixed iterate against the FP64 one after the same iterations:
    # largest relative difference per column group (R, t, f, k1, k2, l)
    sa, sb = a.get_state(), b.get_state()
    ca, cb, la, lb = sa["cams"], sb["cams"], sa["lms"], sb["lms"]

    def rel(x, y):
        return float(np.max(np.abs(x - y)) / max(np.max(np.abs(x)), 1e-300))
    groups = {"R": slice(0, 9), "t": slice(9, 12), "f": slice(12, 13), "f k1": slice(13, 14), "f k2": slice(14, 15)}
    state_err = {g: rel(ca[:, sl], cb[:, sl]) for g, sl in groups.items()}
    state_err["l"] = rel(la, lb)
    del a
    F32 = np.concatenate([F32a, b.iterate(iters // 2)])
    del b
    target = F64[-1] + 1e-4 * (F0 - F64[-1])
    n64 = int(np.argmax(F64 <= target)) + 1 if np.any(F64 <= target) else None
    n32 = int(np.argmax(F32 <= target)) + 1 if np.any(F32 <= target) else None
    out = dict(F_init=F0, F_fp64_final=float(F64[-1]), F_target=float(target), iters_fp64=n64, iters_fp32=n32,
               fp32_rel_err_at_fp64_final_iter=float(abs(F32[iters - 1] - F64[-1]) / F64[-1]),
               fp32_vs_fp64_state_rel_err_after_iters=state_err)
    if n64 and n32:
        out["time_fp64_ms"] = n64 * ms64
        out["time_fp32_ms"] = n32 * ms32
        out["speedup_fp32_vs_fp64"] = (n64 * ms64) / (n32 * ms32)
    else:
        out["speedup_fp32_vs_fp64"] = None
    return out


def cpu_baseline(prob, S, budget_s=15.0, budget_1t_s=6.0, one_thread=True):
    """The oracle, as it stands, on the same problem and options: whole
    iterations from x^0 until about budget_s of CPU work has been done on
    every host core, then (continuing from there, if one_thread) about
    budget_1t_s on one thread."""
    from oracle import Oracle, num_threads, set_num_threads
    t0 = time.perf_counter()
    o = Oracle(prob, n_partitions=S, loss="huber", delta=1.0, xi=1e-9, eta=0.5)
    setup = time.perf_counter() - t0

    def run(budget):
        n, t0 = 0, time.perf_counter()
        while True:
            o.iterate(1)
            n += 1
            dt = time.perf_counter() - t0
            if dt >= budget or n >= 200:
                return n, dt

    cores = num_threads()
    n, dt = run(budget_s)
    out = dict(value=prob["n_obs"] * n / dt, unit="obs*iter/s", cores=cores, kind="oracle",
               sample=f"{n} oracle iteration(s) of the same {prob['n_obs']}-observation problem from x^0, "
                      f"{dt:.1f} s wall (oracle setup {setup:.1f} s not counted), OpenMP over entities",
               cpu_model=cpu_model())
    if one_thread:
        set_num_threads(1)
        n1, dt1 = run(budget_1t_s)
        set_num_threads(0)
        out["value_1thread"] = prob["n_obs"] * n1 / dt1
        out["sample_1thread"] = f"the next {n1} iteration(s) on 1 thread, {dt1:.1f} s wall"
    del o
    return out


def attainable_bandwidth(mib=1024, reps=10, grids=(512, 768, 1024, 1280)):
    """HBM bandwidth a plain streaming copy reaches on this GPU (read + write
    bytes per second; the best of a few grid sizes), the practical ceiling
    next to the vendor peak.  The copy is the library's measurement hook."""
    import torch
    from paper_2305_07026_amd import binding as B
    n = mib * (1 << 20)
    a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    best = 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for g in grids:
        for _ in range(2):
            B.check(B.lib.daba_stream_copy(b.data_ptr(), a.data_ptr(), n, g, sp), "daba_stream_copy")
        e0.record(stream)
        for _ in range(reps):
            B.check(B.lib.daba_stream_copy(b.data_ptr(), a.data_ptr(), n, g, sp), "daba_stream_copy")
        e1.record(stream)
        torch.cuda.synchronize()
        best = max(best, 2 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def partition_cpu_baseline(prob, S, n_cams=60, n_lms=3000, iters=2):
    """The partition-level oracle (dense solve per partition) on a bounded
    sample: the sub-problem on the first n_cams cameras and the n_lms
    landmarks they see most, same partition count."""
    from oracle.partition import PartOracle
    from synth import subproblem
    sub = subproblem(prob, n_cams, n_lms)
    po = PartOracle(sub, n_partitions=S, loss="huber", delta=1.0, xi=1e-9, eta=0.5)
    t0 = time.perf_counter()
    po.iterate(iters)
    dt = time.perf_counter() - t0
    return {"value": sub["n_obs"] * iters / dt, "unit": "obs*iter/s", "cores": int(os.cpu_count() or 1),
            "kind": "oracle",
            "sample": f"{iters} iterations of the partition-level oracle (numpy, dense LM solve per partition) "
                      f"on the sub-problem of the first {n_cams} cameras and {sub['n_landmarks']} landmarks "
                      f"({sub['n_obs']} observations), {S} partitions; the full workload's dense partition "
                      f"systems do not fit the oracle",
            "numpy_threads_note": "numpy's BLAS uses the host's threads; cores is the host count"}


def bench_partition(args, prob, S):
    """The device surrogate (exact intra-partition pairs, LM per partition) on
    the same workload: per-iteration time, the time per launch group, and the
    Cholesky factorisations against the FP64 vector peak."""
    import numpy as np
    import torch
    import paper_2305_07026_amd as P
    K = prob["n_obs"]
    log("create (device surrogate)")
    t0 = time.perf_counter()
    sol = P.DabaPartSolver(prob, n_partitions=S, loss="huber", delta=1.0, xi=1e-9, eta=0.5, accelerate=True,
                           inner_steps=1)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    warm, steps = min(args.warmup, 5), min(args.steps, 20)
    sol.iterate(warm, trace=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sol.stream)
    sol.iterate(steps, trace=False)
    e1.record(sol.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    groups = sol.iterate_timed(steps)
    # reduced camera systems: one per partition, order 9 M_a (the kernels
    # factor it padded to a multiple of 64; the flops counted are those of
    # the unpadded order)
    cam_part = np.arange(prob["n_cameras"]) // -(-prob["n_cameras"] // S)
    n_a = 9 * np.bincount(cam_part, minlength=S)
    flops = float(2.0 * np.sum(n_a.astype(np.float64) ** 3) / 3.0)  # Cholesky: n^3/3 multiply-adds
    fact_ms = groups["cholesky"] / max(groups["lm_attempts"], 1)
    solve_ms = groups["solve"] / max(groups["lm_attempts"], 1)
    achieved = flops / (fact_ms / 1e3) / 1e12
    out = {
        "metric": "observation-iterations/s, device surrogate (exact intra-partition pairs, LM per partition)",
        "value": K / (ms / 1e3),
        "unit": "obs*iter/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator standing in for the paper's BAL/1DSfM scenes)",
        "config": {"workload": f"{args.workload}: {prob['n_cameras']} cameras, {prob['n_landmarks']} landmarks, "
                               f"{K} observations, {S} camera partitions, Huber delta=1px, device surrogate of "
                               f"eq. Ealpha, DABA, one successful LM step per partition, fp64",
                   "n_cameras": prob["n_cameras"], "n_landmarks": prob["n_landmarks"], "n_obs": K,
                   "n_partitions": S, "surrogate": "partition"},
        "roofline": {"bound": "alu", "kernel": "Cholesky of the reduced camera systems (kp_chol_*)",
                     "achieved": achieved, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_TFLOPS, "traffic": None,
                     "algorithmic_flops_per_factorisation": flops, "avg_factorisation_ms": fact_ms,
                     "order_per_partition": int(n_a.max()),
                     "factorisation_plus_solve_ms_per_attempt": fact_ms + solve_ms},
        "group_ms_per_step": {k: v / steps for k, v in groups.items() if k not in ("lm_attempts", "cholesky_launches")},
        "lm_attempts_per_step": groups["lm_attempts"] / steps,
        "setup_s": setup_s,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (partition oracle, bounded sample)")
        out["cpu_baseline"] = partition_cpu_baseline(prob, S)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="cam20k-lm10m")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a device copy of this many MiB (for HBM counter calibration)")
    ap.add_argument("--no-attainable", action="store_true",
                    help="skip the copy-bandwidth measurement (implied by --copy-calibration)")
    ap.add_argument("--surrogate", default="entity", choices=["entity", "partition"],
                    help="entity: every pair majorized (the default measurement); partition: the device "
                         "surrogate of eq. Ealpha with exact intra-partition pairs (include/daba_part.h)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: every partition runs as a "
              "camera block of one GPU, and the multi-GPU path is a design, not code.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from synth import CONFIGS, make_problem
    import paper_2305_07026_amd as P

    cfg = CONFIGS[args.workload]
    S = cfg["n_partitions"]
    log(f"generating {args.workload}")
    prob = make_problem(args.workload)
    if args.surrogate == "partition":
        print(json.dumps(bench_partition(args, prob, S)), flush=True)
        return
    K = prob["n_obs"]
    T = n_tiles(prob)
    opts = dict(n_partitions=S, loss="huber", delta=1.0, xi=1e-9, eta=0.5, accelerate=True, inner_steps=1)

    def make(prec):
        return P.DabaSolver(prob, precision=prec, **opts)

    def timed(sol, steps):
        """GPU ms per iteration over `steps` graph-replayed iterations, with
        HIP events on the solver's stream."""
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(sol.stream)
        sol.iterate(steps, trace=False)
        e1.record(sol.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def measure(prec):
        log(f"create ({prec})")
        t0 = time.perf_counter()
        sol = make(prec)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        log(f"warmup {args.warmup} ({prec})")
        sol.iterate(args.warmup, trace=False)
        log(f"timed 3 x {args.steps} ({prec})")
        w0 = time.perf_counter()
        reps = [timed(sol, args.steps)]
        wall = time.perf_counter() - w0
        reps += [timed(sol, args.steps) for _ in range(2)]
        # per-kernel durations from HIP events around each launch, over the
        # same number of steps of the same run (instrumented launches, no graph)
        log(f"kernel timing ({prec})")
        kern = sol.iterate_timed(args.steps) / args.steps
        return sol, reps, wall, kern, setup

    prec = args.precision
    fp32 = prec == "fp32_mixed"
    sol, repeats, wall, kern, setup_s = measure(prec)
    ms_per_step = repeats[0]
    value = K / (ms_per_step / 1e3)
    F_final = sol.objective()
    del sol
    torch.cuda.empty_cache()
    kb = kernel_bytes(prob, S, T, fp32)
    names = ["k_tiles", "k_lms", "k_entity", "k_decide (+k_finalize once)"]
    dom = "k_tiles" if kern[0] >= kern[1] else "k_lms"
    dom_ms = kern[0] if dom == "k_tiles" else kern[1]
    achieved = kb[dom] / (dom_ms / 1e3) / 1e9
    attainable = None
    if not (args.no_attainable or args.copy_calibration):
        log("copy bandwidth")
        attainable = attainable_bandwidth()

    out = {
        "metric": "observation-iterations/s and HBM GB/s (FP32-mixed vs FP64) at equal final objective",
        "value": value,
        "unit": "obs*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic (seeded generator standing in for the paper's BAL/1DSfM scenes)",
        "config": {"workload": f"{args.workload}: {prob['n_cameras']} cameras, {prob['n_landmarks']} landmarks, "
                               f"{K} observations, {S} camera partitions, Huber delta=1px, DABA (Nesterov + "
                               f"adaptive restart), 1 inner LM step, {prec}",
                   "n_cameras": prob["n_cameras"], "n_landmarks": prob["n_landmarks"], "n_obs": K,
                   "n_partitions": S, "precision": prec},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, args.workload, prec),
                     "algorithmic_bytes_per_launch": kb[dom], "avg_launch_ms": dom_ms,
                     "attainable_copy_GBs": attainable,
                     "frac_of_attainable": achieved / attainable if attainable else None},
        "kernels": {n: {"ms": float(kern[i]),
                        "algorithmic_bytes": kb.get(n),
                        "GBs": kb[n] / (kern[i] / 1e3) / 1e9 if n in kb else None,
                        "traffic": measured_traffic(n, args.workload, prec) if n in kb else None}
                    for i, n in enumerate(names)},
        "k_lms_camera_gathers_from_cache_bytes": kb["k_lms_camera_gathers_from_cache"],
        "iteration_at_survey_bytes": {
            "bytes_per_obs": SURVEY_BYTES_PER_OBS,
            "GBs": SURVEY_BYTES_PER_OBS * K / (ms_per_step / 1e3) / 1e9,
            "frac": SURVEY_BYTES_PER_OBS * K / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        "ms_per_step_repeats": repeats,
        "ms_per_step_median": sorted(repeats)[1],
        "wall_s_timed_region": wall,
        "setup_s": setup_s,
        "F_after": F_final,
    }
    if not args.no_fp32 and not fp32:
        s32, reps32, _, k32, _ = measure("fp32_mixed")
        ms32 = reps32[0]
        del s32
        torch.cuda.empty_cache()
        kb32 = kernel_bytes(prob, S, T, True)
        log("equal objective")
        eq = equal_objective(prob, ms_per_step, ms32, cfg["iterations"] or 200, S, make)
        out["fp32_mixed"] = {"value": K / (ms32 / 1e3), "ms_per_step": ms32, "ms_per_step_repeats": reps32,
                             "kernels": {n: {"ms": float(k32[i]),
                                             "algorithmic_bytes": kb32.get(n),
                                             "GBs": kb32[n] / (k32[i] / 1e3) / 1e9 if n in kb32 else None,
                                             "traffic": (measured_traffic(n, args.workload, "fp32_mixed")
                                                         if n in kb32 else None)}
                                         for i, n in enumerate(names)},
                             "equal_objective": eq}
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * n * 8
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(prob, S, one_thread=K <= 20_000_000)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
