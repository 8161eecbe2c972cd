"""Benchmark: FP64 GEMM C <- A*B + C at n=8192 on one MI355X (gfx950).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

A step is one C <- alpha*A*B + beta*C with m=n=k=8192, alpha=beta=1, FP64,
entries uniform in [-1, 1) (the square size sweep's largest size), operands
resident in HBM.  W untimed steps, then K timed steps bracketed by device
synchronisation.  ``value`` is 2*n^3 / (time per step) in TFLOP/s.

Also reported on the same line (measured in the same run, outside the timed
region of the headline):
  roofline      achieved TFLOP/s of the GEMM kernel from HIP events around
                each launch on its stream, against the 78.6 TFLOP/s FP64
                matrix peak; ``traffic`` from committed rocprofv3 counters
                when they were taken on the current kernel source, else null.
  error         relative Frobenius error of sampled outputs vs the oracle.
  split         the split-precision path (INT8 and BF16 slices) at n=4096
                with exponent-spread entries: FP64-equivalent TFLOP/s and
                relative error of sampled outputs vs the oracle.
  cpu_baseline  the CPU oracle (compensated FP64 triple loop, OpenMP) timed
                on this host's cores on a bounded sample of output rows.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK = 78.6  # TFLOP/s, MI355X FP64 matrix (= vector) peak
INT8_PEAK = 5000.0  # TOP/s dense
BF16_PEAK = 2500.0  # TFLOP/s dense
METRIC = "GEMM TFLOP/s & %peak: FP64 vs split-prec at 1e-12 rel err; p99 latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dgemm_f64_n8192.json")
KERNEL_SOURCES = ["paper_1602_08477_amd/csrc/gemm_tile.h",
                  "paper_1602_08477_amd/csrc/gemm_native.hip",
                  "paper_1602_08477_amd/csrc/common.h"]


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters(launch_bytes_alg: float):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs, scaled by the copy-kernel calibration; None if the counters were
    taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def sample_idx(seed, count, hi):
    import synth
    v = synth.log_uniform_int(seed, 9, count, 1, hi - 1)
    return np.unique(np.concatenate([[0, hi - 1], v]))


def sampled_error(dA, dB, C0, dC, alpha, beta, seed):
    import torch
    import oracle
    m, k = dA.shape
    n = dB.shape[1]
    rows = sample_idx(seed, 24, m)
    cols = sample_idx(seed + 1, 24, n)
    rt, ct = torch.from_numpy(rows).to(dA.device), torch.from_numpy(cols).to(dA.device)
    ref = oracle.dgemm(alpha, dA[rt].cpu().numpy(), dB[:, ct].cpu().numpy(), beta,
                       None if beta == 0 else C0[rt][:, ct].cpu().numpy())
    return oracle.rel_fro_err(dC[rt][:, ct].cpu().numpy(), ref)


def time_launches(fn, steps, warmup, stream):
    """Per-launch durations (ms) from HIP events recorded on ``stream``."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        fn()
        e.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return [s.elapsed_time(e) for s, e in ev], wall


def bench_native(n, steps, warmup):
    import torch
    import paper_1602_08477_amd as mg
    import synth
    seed = synth.config_seed(2)
    dA = synth.matrix(seed, synth.STREAM_A, n, n, device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, n, n, device="cuda")
    dC = synth.matrix(seed, synth.STREAM_C, n, n, device="cuda")
    C0 = dC.clone()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    # headline: W untimed + K timed steps bracketed by synchronisation
    for _ in range(warmup):
        mg.gemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mg.gemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps

    # kernel duration from events on the launch stream
    per_launch, _ = time_launches(lambda: mg.gemm(dA, dB, dC, 1.0, 1.0), steps, 1, stream)
    kern_ms = float(np.mean(per_launch))

    # parity of one fresh step
    dC.copy_(C0)
    mg.gemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    err = sampled_error(dA, dB, C0, dC, 1.0, 1.0, seed)
    del dA, dB, dC, C0
    torch.cuda.empty_cache()
    return ms_per_step, kern_ms, err


def bench_split(n, steps, warmup):
    import torch
    import paper_1602_08477_amd as mg
    import synth
    seed = synth.config_seed(3)
    dA = synth.matrix(seed, synth.STREAM_A, n, n, kind="spread", device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, n, n, kind="spread", device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    flop = 2.0 * n ** 3
    for name, algo in (("native_f64", mg.NATIVE), ("i8", mg.SPLIT_I8), ("bf16", mg.SPLIT_BF16)):
        dC = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        if algo == mg.NATIVE:
            fn = lambda: mg.gemm(dA, dB, dC, 1.0, 0.0)  # noqa: E731
        else:
            s = mg.split_default_slices(algo)
            ws = mg.split_workspace(algo, s, n, n, n)
            fn = lambda: mg.gemm_split(dA, dB, dC, 1.0, 0.0, algo=algo, slices=s,  # noqa: E731
                                       workspace=ws)
        per, _ = time_launches(fn, steps, warmup, stream)
        ms = float(np.median(per))
        err = sampled_error(dA, dB, None, dC, 1.0, 0.0, seed)
        rec = {"ms": round(ms, 4), "tflops_fp64_equiv": round(flop / ms / 1e9, 2),
               "rel_fro_err_sampled": float(f"{err:.3e}")}
        if algo != mg.NATIVE:
            pairs = s * (s + 1) // 2
            peak = INT8_PEAK if algo == mg.SPLIT_I8 else BF16_PEAK
            rec.update({"slices": s, "pairs": pairs,
                        "lowprec_util": round(pairs * flop / ms / 1e9 / peak, 4)})
            del ws
        out[name] = rec
        del dC
    out["split_faster_than_native"] = out["i8"]["ms"] < out["native_f64"]["ms"]
    del dA, dB
    torch.cuda.empty_cache()
    return out


def cpu_baseline(n, target_s=12.0):
    """The oracle on this host: output rows of the n=8192 workload, doubling
    the row count until one run takes at least ``target_s`` / 4 seconds, then
    timing a run of about ``target_s``."""
    import oracle
    import synth
    seed = synth.config_seed(2)
    B = synth.matrix(seed, synth.STREAM_B, n, n)
    rows = 1
    while True:
        A = synth.uniform_pm1(seed, synth.STREAM_A, rows * n).reshape(rows, n)
        C = synth.uniform_pm1(seed, synth.STREAM_C, rows * n).reshape(rows, n)
        t0 = time.perf_counter()
        oracle.dgemm(1.0, A, B, 1.0, C)
        dt = time.perf_counter() - t0
        if dt >= target_s / 4 or rows >= n:
            break
        rows = min(n, rows * 2 if dt < target_s / 16 else rows * 4)
    tflops = 2.0 * rows * n * n / dt / 1e12
    return {"value": float(f"{tflops:.6g}"), "unit": "TFLOP/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{rows} of {n} output rows of the n={n} FP64 GEMM ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--quick", action="store_true", help="headline only (for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the GEMM path "
              "here is single-GPU; see DESIGN.md for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1602_08477_amd as mg
    mg.lib()
    if not torch.cuda.is_available():
        eprint("no GPU visible")
        sys.exit(3)
    n = args.n
    eprint(f"bench: native FP64 n={n} steps={args.steps} warmup={args.warmup}")
    ms_step, kern_ms, err = bench_native(n, args.steps, args.warmup)
    flop = 2.0 * n ** 3
    value = flop / ms_step / 1e9
    achieved = flop / kern_ms / 1e9
    alg_bytes = 4.0 * n * n * 8  # A, B read, C read and written once
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 GEMM C=A*B+C, m=n=k={n}, row-major, U[-1,1), alpha=beta=1",
                   "m": n, "n": n, "k": n, "alpha": 1.0, "beta": 1.0,
                   "tile_cfg": mg.tile_cfg_info(mg.pick_tile_cfg(n, n, n))},
        "pct_peak": round(100.0 * value / FP64_PEAK, 2),
        "rel_fro_err_sampled": float(f"{err:.3e}"),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK, 4),
                     "traffic": traffic_from_counters(alg_bytes),
                     "alg_flop_per_launch": flop, "alg_bytes_per_launch": alg_bytes,
                     "kernel_ms": round(kern_ms, 4)},
    }
    if not args.quick:
        eprint("bench: split precision n=4096")
        rec["split"] = bench_split(4096, max(5, args.steps), 2)
        if not args.no_cpu_baseline:
            eprint("bench: cpu baseline (oracle)")
            rec["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
