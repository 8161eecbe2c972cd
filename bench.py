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
                  "paper_1602_08477_amd/csrc/gemm_dma.h",
                  "paper_1602_08477_amd/csrc/gemm_launch.h",
                  "paper_1602_08477_amd/csrc/gemm_native.hip",
                  "paper_1602_08477_amd/csrc/common.h"]


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


DAXPY_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_daxpy_n2p27.json")
DAXPY_SOURCES = ["paper_1602_08477_amd/csrc/axpy.hip", "paper_1602_08477_amd/csrc/common.h"]


def kernel_source_hash(sources=None) -> str:
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters(launch_bytes_alg: float, path=None, sources=None):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs, scaled by the copy-kernel calibration; None if the counters were
    taken on different kernel sources."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash(sources):
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


def time_interleaved(fns, steps, warmup, stream):
    """Per-launch durations (ms) of several launchers timed in rotation (one
    launch of each per round), so that clock drift affects all alike."""
    import torch
    for _ in range(warmup):
        for fn in fns:
            fn()
    torch.cuda.synchronize()
    out = [[] for _ in fns]
    for _ in range(steps):
        for i, fn in enumerate(fns):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record(stream)
            fn()
            e.record(stream)
            out[i].append((s, e))
    torch.cuda.synchronize()
    return [[s.elapsed_time(e) for s, e in evs] for evs in out]


def back_to_back_ms(fn, reps, stream, rounds=3):
    """Mean per-launch time (ms) of `reps` launches issued back to back
    between one pair of HIP events; the median over `rounds` such runs."""
    import torch
    fn()
    torch.cuda.synchronize()
    res = []
    for _ in range(rounds):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(reps):
            fn()
        e.record(stream)
        torch.cuda.synchronize()
        res.append(s.elapsed_time(e) / reps)
    return float(np.median(res))


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
    spread = {f"kernel_ms_p{q}": round(float(np.percentile(per_launch, q)), 4)
              for q in (10, 50, 90)}

    # parity of one fresh step
    dC.copy_(C0)
    mg.gemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    err = sampled_error(dA, dB, C0, dC, 1.0, 1.0, seed)
    del dA, dB, dC, C0
    torch.cuda.empty_cache()
    return ms_per_step, kern_ms, err, spread


def bench_sizes(steps, warmup):
    """The square size sweep (n = 512 with alpha = 1.5, beta = 0.5; n = 1024 ...
    4096, (8192, 1024, 4096) and the 8-GPU row-panel shard (1024, 8192, 8192)
    with alpha = beta = 1), default work division:
    median kernel time from HIP events, warm operands; for n <= 2048 also a
    cold time with the L2 and MALL flushed by a 512 MiB write before each
    launch.  For context only, the platform BLAS (in-place torch addmm_, one
    GEMM launch per call) is timed on the same operands, its launches
    alternating with this library's; both are also timed with their
    launches back to back (steady state, as the headline is timed)."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    stream = torch.cuda.current_stream()
    flush = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
    out = []
    cases = [((512, 512, 512), 1.5, 0.5, 1)] + [((n, n, n), 1.0, 1.0, 2)
                                                for n in (1024, 2048, 4096)]
    cases.append(((8192, 1024, 4096), 1.0, 1.0, 2))
    # one GPU's shard of the n = 8192 product split over 8 GPUs by row panels
    cases.append(((1024, 8192, 8192), 1.0, 1.0, 2))
    for (m, n, k), alpha, beta, cfg_id in cases:
        seed = synth.config_seed(cfg_id)
        dA = synth.matrix(seed, synth.STREAM_A, m, k, device="cuda")
        dB = synth.matrix(seed, synth.STREAM_B, k, n, device="cuda")
        dC = synth.matrix(seed, synth.STREAM_C, m, n, device="cuda")
        fn = lambda: mg.gemm(dA, dB, dC, alpha, beta)  # noqa: E731
        reps = max(steps, 20)
        # context: the platform BLAS on the same operands, timed in rotation
        # with this library's launch so both see the same clocks; in place on
        # its own copy of C (C <- beta*C + alpha*A@B, one GEMM launch, no
        # copy of C inside the timed launch)
        ref = dC.clone()
        per, per_v = time_interleaved(
            [fn, lambda: ref.addmm_(dA, dB, beta=beta, alpha=alpha)], reps,
            max(warmup, 5), stream)
        ms = float(np.median(per))
        ms_v = float(np.median(per_v))
        flop = 2.0 * m * n * k
        rec = {"m": m, "n": n, "k": k, "alpha": alpha, "beta": beta,
               "tile_cfg": mg.pick_tile_cfg(m, n, k), "ms": round(ms, 5),
               "tflops": round(flop / ms / 1e9, 3),
               "pct_peak": round(100 * flop / ms / 1e9 / FP64_PEAK, 2),
               "context_torch_addmm_tflops": round(flop / ms_v / 1e9, 3)}
        # steady state, as the headline is timed: launches back to back (no
        # other kernel in between), one pair of events around a run of them
        b2b = back_to_back_ms(fn, reps, stream)
        b2b_v = back_to_back_ms(lambda: ref.addmm_(dA, dB, beta=beta, alpha=alpha), reps,
                                stream)
        rec["ms_back_to_back"] = round(b2b, 5)
        rec["pct_peak_back_to_back"] = round(100 * flop / b2b / 1e9 / FP64_PEAK, 2)
        rec["context_torch_addmm_tflops_back_to_back"] = round(flop / b2b_v / 1e9, 3)
        if max(m, n, k) <= 2048:
            cold = []
            for _ in range(reps):
                flush.fill_(1.0)
                s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s.record(stream)
                fn()
                e.record(stream)
                torch.cuda.synchronize()
                cold.append(s.elapsed_time(e))
            rec["ms_cold"] = round(float(np.median(cold)), 5)
        out.append(rec)
        del dA, dB, dC, ref
    del flush
    torch.cuda.empty_cache()
    return out


def bench_trans(n, steps, warmup):
    """Operand layouts at the headline shape (m = n = k, alpha = beta = 1):
    C <- op(A) op(B) + C for op = identity / transpose on each side (mg_gemm_ex
    with the stored transposed copies), launches timed in rotation with HIP
    events; each layout's output checked on sampled entries."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    seed = synth.config_seed(2)
    dA = synth.matrix(seed, synth.STREAM_A, n, n, device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, n, n, device="cuda")
    C0 = synth.matrix(seed, synth.STREAM_C, n, n, device="cuda")
    sA, sB = dA.t().contiguous(), dB.t().contiguous()
    dC = C0.clone()
    stream = torch.cuda.current_stream()
    layouts = [(0, 0), (1, 0), (0, 1), (1, 1)]
    fns = [lambda ta=ta, tb=tb: mg.gemm_ex(sA if ta else dA, sB if tb else dB, dC, 1.0, 1.0,
                                          transa=bool(ta), transb=bool(tb))
           for ta, tb in layouts]
    per = time_interleaved(fns, steps, warmup, stream)
    flop = 2.0 * n ** 3
    out = {}
    for (ta, tb), fn, p in zip(layouts, fns, per):
        dC.copy_(C0)
        fn()
        torch.cuda.synchronize()
        ms = float(np.mean(p))
        out["NT"[ta] + "NT"[tb]] = {
            "ms": round(ms, 4), "tflops": round(flop / ms / 1e9, 3),
            "pct_peak": round(100 * flop / ms / 1e9 / FP64_PEAK, 2),
            "rel_fro_err_sampled": float(f"{sampled_error(dA, dB, C0, dC, 1.0, 1.0, seed):.3e}")}
    del dA, dB, C0, sA, sB, dC
    torch.cuda.empty_cache()
    return {"m": n, "n": n, "k": n, "tile_cfg": mg.pick_tile_cfg(n, n, n), "layouts": out}


def bench_daxpy(n, steps, warmup, cpu=True, small_n=True):
    """DAXPY y <- 1.5 x + y (Section 4.1) on U[-1,1) vectors of n doubles:
    kernel time from HIP events on the launch stream, 24 bytes per element
    (x and y read, y written) against the 8 TB/s HBM peak; a plain 1 GiB
    device copy timed the same way for the bandwidth this part reaches; the
    library's per-call cost at tiny n (host wall time per call over 2000
    back-to-back calls vs the kernel's event time); every element of one
    launch checked against the oracle; the oracle's own rate on the host."""
    import torch
    import paper_1602_08477_amd as mg
    import oracle
    import synth
    seed = synth.config_seed(3)
    stream = torch.cuda.current_stream()
    dx = synth.uniform_pm1(seed, 0, n, device="cuda")
    dy = synth.uniform_pm1(seed, 1, n, device="cuda")
    x_h, y_h = dx.cpu().numpy(), dy.cpu().numpy()
    per, _ = time_launches(lambda: mg.daxpy(1.5, dx, dy), max(steps, 20), warmup, stream)
    ms = float(np.mean(per))
    alg_bytes = 24.0 * n
    gbs = alg_bytes / ms / 1e6
    # parity of one launch on fresh inputs
    dy.copy_(torch.from_numpy(y_h))
    mg.daxpy(1.5, dx, dy)
    torch.cuda.synchronize()
    exact = bool(np.array_equal(dy.cpu().numpy(), oracle.daxpy(1.5, x_h, y_h)))
    # a plain device-to-device copy of 1 GiB (reads and writes 2 GiB)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    per_c, _ = time_launches(lambda: dst.copy_(src), 20, 2, stream)
    copy_gbs = 2.0 * src.numel() * 8 / float(np.mean(per_c)) / 1e6
    del src, dst
    # per-call cost at small n: host wall time per call vs kernel time
    small = []
    for m in ((1, 1024, 65536, 1 << 20) if small_n else ()):
        sx, sy = dx[:m], dy[:m]
        fn = lambda: mg.daxpy(1.5, sx, sy)  # noqa: E731
        k_ms = float(np.median(time_launches(fn, 50, 5, stream)[0]))
        torch.cuda.synchronize()
        reps = 2000
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        wall_us = (time.perf_counter() - t0) * 1e6 / reps
        small.append({"n": m, "kernel_us": round(k_ms * 1e3, 2),
                      "wall_us_per_call": round(wall_us, 2)})
    rec = {"n": n, "alpha": 1.5, "ms": round(ms, 4), "gb_per_s": round(gbs, 1),
           "bit_exact_vs_oracle": exact,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                        "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                        "traffic": traffic_from_counters(alg_bytes, DAXPY_TRAFFIC_FILE,
                                                         DAXPY_SOURCES)
                        if n == 1 << 27 else None,
                        "alg_bytes_per_launch": alg_bytes, "kernel_ms": round(ms, 4)},
           "context_device_copy_gb_per_s": round(copy_gbs, 1),
           "small_n": small}
    if cpu:
        oracle.daxpy(1.5, x_h[:1 << 20], y_h[:1 << 20])  # first touch of the pages, threads up
        t0 = time.perf_counter()
        oracle.daxpy(1.5, x_h, y_h)
        t = time.perf_counter() - t0
        rec["cpu_oracle"] = {"gb_per_s": round(alg_bytes / t / 1e9, 2), "cores": oracle.threads(),
                             "seconds": round(t, 3)}
    del dx, dy
    torch.cuda.empty_cache()
    return rec


def bench_overhead():
    """Library overhead and the naive mapping (paper Section 4.2, Figs. 5-6
    on MI355X): runs the mg_overhead driver (C++, linked against libmg.so),
    which times the same tiled kernel reached through mg_gemm and launched
    directly with hipLaunchKernelGGL (device time per launch, host time per
    enqueue), and the naive one-output-per-lane work division."""
    import subprocess
    from paper_1602_08477_amd import build as b
    exe = b.driver_path(os.path.join(b.HERE, "drivers", "overhead.hip"))
    if not os.path.exists(exe):
        raise RuntimeError(f"{exe} is missing: build with __graft_entry__.build()")
    r = subprocess.run([exe, "200"], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        raise RuntimeError(f"mg_overhead failed ({r.returncode}): {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


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
    # smaller sizes (the serving mix's range): split INT8 against native FP64
    sweep = []
    for sn in (128, 256, 512, 1024, 2048):
        sA = synth.matrix(seed, synth.STREAM_A, sn, sn, kind="spread", device="cuda")
        sB = synth.matrix(seed, synth.STREAM_B, sn, sn, kind="spread", device="cuda")
        sC = torch.zeros(sn, sn, dtype=torch.float64, device="cuda")
        ss = mg.split_default_slices(mg.SPLIT_I8)
        ws = mg.split_workspace(mg.SPLIT_I8, ss, sn, sn, sn)
        per_n, per_s = time_interleaved(
            [lambda: mg.gemm(sA, sB, sC, 1.0, 0.0),
             lambda: mg.gemm_split(sA, sB, sC, 1.0, 0.0, algo=mg.SPLIT_I8, slices=ss,
                                   workspace=ws)], steps, warmup, stream)
        ms_n, ms_s = float(np.median(per_n)), float(np.median(per_s))
        sweep.append({"n": sn, "native_ms": round(ms_n, 4), "i8_ms": round(ms_s, 4),
                      "native_tflops": round(2.0 * sn ** 3 / ms_n / 1e9, 2),
                      "i8_tflops_fp64_equiv": round(2.0 * sn ** 3 / ms_s / 1e9, 2)})
        del sA, sB, sC, ws
    out["sizes"] = sweep
    torch.cuda.empty_cache()
    return out


def profile_batched():
    """For counter runs: the 2000-problem batch (autotuned table) launched 3
    times in FP64, then 3 times in FP32; these are the last 3 dispatches of
    each grouped kernel."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    seed = synth.config_seed(4)
    shapes = synth.batch_shapes(seed, 2000)
    out = {}
    for name, dt, code in (("f64", torch.float64, mg.F64), ("f32", torch.float32, mg.F32)):
        offs = {"A": [0], "B": [0], "C": [0]}
        for m_, n_, k_ in shapes:
            for key, sz in (("A", m_ * k_), ("B", k_ * n_), ("C", m_ * n_)):
                offs[key].append(offs[key][-1] + -(-int(sz) // 32) * 32)
        flats = {key: synth.flat_uniform(seed, i, offs[key][-1], device="cuda").to(dt)
                 for i, key in enumerate(("A", "B", "C"))}
        probs = []
        for i, (m_, n_, k_) in enumerate(shapes):
            m_, n_, k_ = int(m_), int(n_), int(k_)
            probs.append(mg.problem(
                flats["A"][offs["A"][i]: offs["A"][i] + m_ * k_].view(m_, k_),
                flats["B"][offs["B"][i]: offs["B"][i] + k_ * n_].view(k_, n_),
                flats["C"][offs["C"][i]: offs["C"][i] + m_ * n_].view(m_, n_), 1.0, 1.0))
        table = mg.autotune(code, reps=1)
        plan = mg.Plan(code, probs, table)
        torch.cuda.synchronize()
        for _ in range(3):
            plan.launch(graph=False)
        torch.cuda.synchronize()
        out[name] = plan.stats()
        plan.close()
        del flats, probs
        torch.cuda.empty_cache()
    return out


def profile_batched_split():
    """For counter runs: the 2000-problem FP64 batch through the batched
    split path, 3 times with MG_SPLIT_I8, then 3 times with MG_SPLIT_BF16."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    seed = synth.config_seed(4)
    shapes = synth.batch_shapes(seed, 2000)
    offs = {"A": [0], "B": [0], "C": [0]}
    for m_, n_, k_ in shapes:
        for key, sz in (("A", m_ * k_), ("B", k_ * n_), ("C", m_ * n_)):
            offs[key].append(offs[key][-1] + -(-int(sz) // 32) * 32)
    flats = {key: synth.flat_uniform(seed, i, offs[key][-1], device="cuda")
             for i, key in enumerate(("A", "B", "C"))}
    probs = []
    for i, (m_, n_, k_) in enumerate(shapes):
        m_, n_, k_ = int(m_), int(n_), int(k_)
        probs.append(mg.problem(
            flats["A"][offs["A"][i]: offs["A"][i] + m_ * k_].view(m_, k_),
            flats["B"][offs["B"][i]: offs["B"][i] + k_ * n_].view(k_, n_),
            flats["C"][offs["C"][i]: offs["C"][i] + m_ * n_].view(m_, n_), 1.0, 1.0))
    for algo in (mg.SPLIT_I8, mg.SPLIT_BF16):
        for _ in range(3):
            mg.gemm_batched(probs, dtype=mg.F64, algo=algo)
        torch.cuda.synchronize()
    return {"problems": len(probs)}


def profile_split(n=4096):
    """For counter runs: native FP64, then split INT8 three times, then split
    BF16 once, at n = 4096 on the exponent-spread workload (alpha=1, beta=0)."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    seed = synth.config_seed(3)
    dA = synth.matrix(seed, synth.STREAM_A, n, n, kind="spread", device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, n, n, kind="spread", device="cuda")
    dC = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    mg.gemm(dA, dB, dC, 1.0, 0.0)
    for algo, reps in ((mg.SPLIT_I8, 3), (mg.SPLIT_BF16, 1)):
        s = mg.split_default_slices(algo)
        ws = mg.split_workspace(algo, s, n, n, n)
        for _ in range(reps):
            mg.gemm_split(dA, dB, dC, 1.0, 0.0, algo=algo, slices=s, workspace=ws)
        torch.cuda.synchronize()
        del ws
    return {"n": n}


def batched_roofline_ms(shapes, esz, peak_tflops):
    """Sum over problems of max(FLOP / peak, compulsory bytes / 8 TB/s), ms."""
    m, n, k = (shapes[:, i].astype(np.float64) for i in range(3))
    flop = 2 * m * n * k
    byts = esz * (m * k + k * n + 2 * m * n)
    return float(np.sum(np.maximum(flop / (peak_tflops * 1e12), byts / 8e12)) * 1e3), \
        float(flop.sum()), float(byts.sum())


def batched_oracle_error(shapes, offs, flats, C_init):
    """Largest relative Frobenius error over all problems of a batch against
    the oracle (run on the operands as stored, FP32 widened exactly)."""
    import oracle
    h = {key: t.double().cpu().numpy() for key, t in flats.items()}
    c0 = C_init.double().cpu().numpy()
    worst = 0.0
    for i, (m_, n_, k_) in enumerate(shapes):
        m_, n_, k_ = int(m_), int(n_), int(k_)
        A = h["A"][offs["A"][i]: offs["A"][i] + m_ * k_].reshape(m_, k_)
        B = h["B"][offs["B"][i]: offs["B"][i] + k_ * n_].reshape(k_, n_)
        C = c0[offs["C"][i]: offs["C"][i] + m_ * n_].reshape(m_, n_)
        got = h["C"][offs["C"][i]: offs["C"][i] + m_ * n_].reshape(m_, n_)
        worst = max(worst, oracle.rel_fro_err(got, oracle.dgemm(1.0, A, B, 1.0, C)))
    return worst


def bench_batched(steps):
    """2000 problems, m, n, k log-uniform in [16, 512], FP64 and FP32: one
    persistent launch per batch, graph-replayed, tile classes autotuned."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    seed = synth.config_seed(4)
    shapes = synth.batch_shapes(seed, 2000)
    out = {}
    for name, dt, code, peak in (("f64", torch.float64, mg.F64, FP64_PEAK),
                                 ("f32", torch.float32, mg.F32, 157.3)):
        esz = 8 if dt == torch.float64 else 4
        offs = {"A": [0], "B": [0], "C": [0]}
        for m_, n_, k_ in shapes:
            for key, sz in (("A", m_ * k_), ("B", k_ * n_), ("C", m_ * n_)):
                offs[key].append(offs[key][-1] + -(-int(sz) // 32) * 32)
        flats = {key: synth.flat_uniform(seed, i, offs[key][-1], device="cuda").to(dt)
                 for i, key in enumerate(("A", "B", "C"))}
        probs = []
        for i, (m_, n_, k_) in enumerate(shapes):
            m_, n_, k_ = int(m_), int(n_), int(k_)
            A = flats["A"][offs["A"][i]: offs["A"][i] + m_ * k_].view(m_, k_)
            B = flats["B"][offs["B"][i]: offs["B"][i] + k_ * n_].view(k_, n_)
            C = flats["C"][offs["C"][i]: offs["C"][i] + m_ * n_].view(m_, n_)
            probs.append(mg.problem(A, B, C, 1.0, 1.0))
        C_init = flats["C"].clone()
        t0 = time.perf_counter()
        table = mg.autotune(code, reps=2)
        tune_s = time.perf_counter() - t0
        plan = mg.Plan(code, probs, table)
        plan_h = mg.Plan(code, probs)  # heuristic table, for comparison
        stream = torch.cuda.current_stream()
        per_g, per_d, per_h = time_interleaved(
            [lambda: plan.launch(graph=True), lambda: plan.launch(graph=False),
             lambda: plan_h.launch(graph=True)], steps, 5, stream)
        ms = float(np.median(per_g))
        roof_ms, flop, byts = batched_roofline_ms(shapes, esz, peak)
        st = plan.stats()
        out[name] = {"problems": 2000, "ms": round(ms, 4), "tflops": round(flop / ms / 1e9, 2),
                     "roofline_ms": round(roof_ms, 4), "roofline_frac": round(roof_ms / ms, 4),
                     "ms_direct_launch": round(float(np.median(per_d)), 4),
                     "ms_heuristic_table": round(float(np.median(per_h)), 4),
                     "tiles": st["tiles"], "workgroups": st["workgroups"],
                     "tiles_per_class": st["tiles_per_class"], "autotune_s": round(tune_s, 2),
                     "gflop": round(flop / 1e9, 3), "gbytes": round(byts / 1e9, 3)}
        # every problem of one fresh launch against the oracle
        flats["C"].copy_(C_init)
        plan.launch(graph=True)
        torch.cuda.synchronize()
        out[name]["rel_fro_err_max_all_problems"] = float(
            f"{batched_oracle_error(shapes, offs, flats, C_init):.3e}")
        if dt == torch.float64:
            # the same problems through the batched split-precision path
            # (mg_gemm_batched with MG_SPLIT_I8 / BF16; each call builds its
            # descriptors and workspace), with every problem's error against
            # the oracle
            parr = mg.problems_array(probs)  # descriptors marshalled once, as for a plan
            for sname, salgo in (("split_i8", mg.SPLIT_I8), ("split_bf16", mg.SPLIT_BF16)):
                flats["C"].copy_(C_init)
                (per_s,) = time_interleaved(
                    [lambda: mg.gemm_batched(parr, dtype=code, algo=salgo)], steps, 3, stream)
                ms_s = float(np.median(per_s))
                flats["C"].copy_(C_init)
                mg.gemm_batched(probs, dtype=code, algo=salgo)
                torch.cuda.synchronize()
                out[name][sname] = {
                    "ms": round(ms_s, 4), "fp64_equivalent_tflops": round(flop / ms_s / 1e9, 2),
                    "rel_fro_err_max_all_problems": float(
                        f"{batched_oracle_error(shapes, offs, flats, C_init):.3e}")}
        del C_init
        if dt == torch.float64:
            # context: the same problems with every row pitch rounded up to an
            # even count (16-byte rows, so all tiles take the 16-byte loads)
            ev = lambda x: -(-int(x) // 2) * 2  # noqa: E731
            offp = {"A": [0], "B": [0], "C": [0]}
            for m_, n_, k_ in shapes:
                for key, sz in (("A", m_ * ev(k_)), ("B", k_ * ev(n_)), ("C", m_ * ev(n_))):
                    offp[key].append(offp[key][-1] + -(-int(sz) // 32) * 32)
            flp = {key: synth.flat_uniform(seed, i, offp[key][-1], device="cuda").to(dt)
                   for i, key in enumerate(("A", "B", "C"))}
            pp = []
            for i, (m_, n_, k_) in enumerate(shapes):
                m_, n_, k_ = int(m_), int(n_), int(k_)
                A = flp["A"][offp["A"][i]: offp["A"][i] + m_ * ev(k_)].view(m_, ev(k_))[:, :k_]
                B = flp["B"][offp["B"][i]: offp["B"][i] + k_ * ev(n_)].view(k_, ev(n_))[:, :n_]
                C = flp["C"][offp["C"][i]: offp["C"][i] + m_ * ev(n_)].view(m_, ev(n_))[:, :n_]
                pp.append(mg.problem(A, B, C, 1.0, 1.0))
            plan_p = mg.Plan(code, pp, table)
            (per_p,) = time_interleaved([lambda: plan_p.launch(graph=True)], steps, 5, stream)
            out[name]["ms_even_row_pitch"] = round(float(np.median(per_p)), 4)
            plan_p.close()
            del flp, pp
        plan.close()
        plan_h.close()
        del flats, probs
        torch.cuda.empty_cache()
    return out


def serve_offsets(ns, arena_elems):
    """C of request i at a 256-byte aligned offset of the arena, handed out in
    arrival order and wrapping to 0 when the rest of the arena is too small.
    Returns (offsets, wrap number per request)."""
    offs = np.empty(len(ns), dtype=np.int64)
    wraps = np.empty(len(ns), dtype=np.int64)
    cur, w = 0, 0
    for i, n in enumerate(ns):
        sz = -(-int(n) * int(n) // 32) * 32
        if cur + sz > arena_elems:
            cur, w = 0, w + 1
        offs[i], wraps[i] = cur, w
        cur += sz
    return offs, wraps


def output_conflicts(ns, offs, wraps, res):
    """Requests whose C region was reused by a later request that the server
    launched before this one had finished (host timestamps: t_launch is taken
    before the batch is enqueued, t_done after its completion event fired).
    Launches follow arrival order, so only the first later request that
    reuses the region needs checking."""
    ends = offs + ns.astype(np.int64) ** 2
    launch = np.array([r.t_launch_ns for r in res])
    done = np.array([r.t_done_ns for r in res])
    bad = 0
    for w in range(int(wraps.max())):
        cur = np.nonzero(wraps == w)[0]
        nxt = np.nonzero(wraps == w + 1)[0]
        if len(nxt) == 0:
            continue
        # first request of the next wrap whose region ends past this one's start
        pos = np.searchsorted(ends[nxt], offs[cur], side="right")
        j = nxt[pos.clip(max=len(nxt) - 1)]
        reuse = (pos < len(nxt)) & (offs[j] < ends[cur])
        bad += int(np.sum(reuse & (launch[j] < done[cur])))
    return bad


def serve_trace(mg, synth, seed, rate, seconds, pools, arena, nmax, budget, table):
    """One open-loop replay: Poisson arrivals at ``rate``, square n
    log-uniform in [32, 2048], 70 % native / 30 % split-INT8; A and B are
    views of resident pools, each request writes its own region of the C
    arena.  Returns latency percentiles, throughput and the number of
    requests whose output region a later, concurrently running request
    reused (expected 0)."""
    count = max(1, int(rate * seconds))
    gaps = synth.poisson_gaps(seed, synth.STREAM_ARRIVALS, count, rate)
    t_arr = np.cumsum(gaps) - gaps[0]
    ns = synth.log_uniform_int(seed, synth.STREAM_SIZES, count, 32, nmax)
    mix = synth.uniform_unit(seed, synth.STREAM_MIX, count)
    algos = np.where(mix < 0.3, mg.SPLIT_I8, mg.NATIVE)
    pool_a, pool_b, pool_elems = pools
    offs = synth.log_uniform_int(seed, 12, count, 1, pool_elems - nmax * nmax - 1) // 32 * 32
    c_offs, wraps = serve_offsets(ns, arena.numel())
    reqs = (mg.Request * count)()
    base_a, base_b, base_c = pool_a.data_ptr(), pool_b.data_ptr(), arena.data_ptr()
    for i in range(count):
        n = int(ns[i])
        o = int(offs[i]) * 8
        reqs[i] = mg.Request(mg.F64, int(algos[i]),
                             mg.Problem(n, n, n, 1.0, 1.0, base_a + o, n, base_b + o, n,
                                        base_c + int(c_offs[i]) * 8, n),
                             int(t_arr[i] * 1e9))
    with mg.Server(n_streams=4, max_slots=256, max_batch=64, hbm_budget_bytes=budget,
                   table=table) as srv:
        res = srv.replay(reqs)
        st = srv.stats()
    ok = np.array([r.status == 0 for r in res])
    lat = np.array([(r.t_done_ns - r.t_arrival_ns) / 1e6 for r in res])[ok]
    t0 = min(r.t_arrival_ns for r in res)
    t1 = max(r.t_done_ns for r in res if r.status == 0)
    flop = float(np.sum(2.0 * ns.astype(np.float64) ** 3 * ok))
    bsz = np.array([r.batch_size for r in res])[ok]
    return {"requests": count, "rate_per_s": rate, "seconds": seconds,
            "hbm_budget_gib": round(budget / 2 ** 30, 3),
            "completed_ok": int(ok.sum()), "rejected_or_failed": int((~ok).sum()),
            "p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "p999_ms": round(float(np.percentile(lat, 99.9)), 4),
            "mean_ms": round(float(lat.mean()), 4),
            "delivered_tflops": round(flop / ((t1 - t0) / 1e9) / 1e12, 3),
            "mean_batch_size": round(float(bsz.mean()), 2), "batches": st["batches"],
            "max_batch": st["max_batch_seen"],
            "max_inflight_gib": round(st["max_inflight_bytes"] / 2 ** 30, 3),
            "max_slots_used": st["max_slots_used"],
            "arena_wraps": int(wraps.max()),
            "output_conflicts": output_conflicts(ns, c_offs, wraps, res)}


def serve_verify(mg, synth, pools, nmax, table, seconds=1.0, rate=2000.0):
    """The workload-5 mix for ``seconds`` with every request's C in its own
    region (no reuse), then 1 % of the requests (at least 200) against the
    oracle: full outputs below n = 512, 16 x 16 sampled outputs above."""
    import torch
    import oracle
    seed = synth.config_seed(5, 9)
    count = int(rate * seconds)
    gaps = synth.poisson_gaps(seed, synth.STREAM_ARRIVALS, count, rate)
    t_arr = np.cumsum(gaps) - gaps[0]
    ns = synth.log_uniform_int(seed, synth.STREAM_SIZES, count, 32, nmax).astype(np.int64)
    algos = np.where(synth.uniform_unit(seed, synth.STREAM_MIX, count) < 0.3, mg.SPLIT_I8,
                     mg.NATIVE)
    pool_a, pool_b, pool_elems = pools
    offs = synth.log_uniform_int(seed, 12, count, 1, pool_elems - nmax * nmax - 1) // 32 * 32
    c_off = np.concatenate([[0], np.cumsum((ns * ns + 31) // 32 * 32)])
    C0 = synth.flat_uniform(seed, 2, int(c_off[-1]), device="cuda")
    C = C0.clone()
    reqs = (mg.Request * count)()
    for i in range(count):
        n, o = int(ns[i]), int(offs[i]) * 8
        reqs[i] = mg.Request(mg.F64, int(algos[i]),
                             mg.Problem(n, n, n, 1.0, 1.0, pool_a.data_ptr() + o, n,
                                        pool_b.data_ptr() + o, n,
                                        C.data_ptr() + int(c_off[i]) * 8, n),
                             int(t_arr[i] * 1e9))
    with mg.Server(n_streams=4, max_slots=256, max_batch=64, hbm_budget_bytes=64 << 30,
                   table=table) as srv:
        res = srv.replay(reqs)
    # a seeded sample of distinct requests: 1 % of them, at least 200
    pick = np.sort(np.argsort(synth.uniform_unit(seed, 13, count))[:max(200, count // 100)])
    worst = {"native": 0.0, "split_i8": 0.0}
    checked = {"native": 0, "split_i8": 0}
    for i in pick:
        n = int(ns[i])
        o = int(offs[i])
        a = pool_a[o: o + n * n].view(n, n)
        b = pool_b[o: o + n * n].view(n, n)
        lo = int(c_off[i])
        c0 = C0[lo: lo + n * n].view(n, n)
        got = C[lo: lo + n * n].view(n, n)
        if n < 512:
            r = c = None
            ref = oracle.dgemm(1.0, a.cpu().numpy(), b.cpu().numpy(), 1.0, c0.cpu().numpy())
            g = got.cpu().numpy()
        else:
            r = np.unique((synth.uniform_unit(seed + int(i), 14, 16) * n).astype(np.int64))
            c = np.unique((synth.uniform_unit(seed + int(i), 15, 16) * n).astype(np.int64))
            rt, ct = torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()
            ref = oracle.dgemm(1.0, a[rt].cpu().numpy(), b[:, ct].cpu().numpy(), 1.0,
                               c0[rt][:, ct].cpu().numpy())
            g = got[rt][:, ct].cpu().numpy()
        key = "native" if algos[i] == mg.NATIVE else "split_i8"
        worst[key] = max(worst[key], oracle.rel_fro_err(g, ref))
        checked[key] += 1
    del C0, C
    torch.cuda.empty_cache()
    return {"requests": count, "completed_ok": int(sum(r.status == 0 for r in res)),
            "checked_vs_oracle": checked,
            "rel_fro_err_max": {k: float(f"{v:.3e}") for k, v in worst.items()}}


def profile_serving(rate=16000.0, seconds=2.0):
    """For kernel traces: one open-loop trace of the serving mix at ``rate``
    under a 64 GiB budget."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    nmax, pool_elems = 2048, 1 << 26
    seed = synth.config_seed(5)
    pools = (synth.flat_uniform(seed, 0, pool_elems, device="cuda"),
             synth.flat_uniform(seed, 1, pool_elems, device="cuda"), pool_elems)
    arena = torch.zeros(1 << 31, dtype=torch.float64, device="cuda")
    table = mg.autotune(mg.F64, reps=2)
    t0 = time.perf_counter()
    out = serve_trace(mg, synth, synth.config_seed(5, 3), rate, seconds, pools, arena, nmax,
                      64 << 30, table)
    out["wall_s"] = round(time.perf_counter() - t0, 3)
    return out


def bench_serving(seconds, rate=2000.0):
    """Open-loop Poisson serving at 2000 requests/s for ``seconds`` under a
    64 GiB HBM budget; then the same mix under a 1 GiB budget (admission
    binds), a saturation sweep of higher arrival rates, and a short trace
    whose results are checked against the oracle."""
    import torch
    import paper_1602_08477_amd as mg
    import synth
    nmax = 2048
    pool_elems = 1 << 26  # 512 MiB of U[-1,1) operands, requests read views of it
    seed = synth.config_seed(5)
    pools = (synth.flat_uniform(seed, 0, pool_elems, device="cuda"),
             synth.flat_uniform(seed, 1, pool_elems, device="cuda"), pool_elems)
    # 32 GiB of outputs: each request writes its own region until the arena
    # wraps; output_conflicts counts any reuse while the earlier one ran
    arena = torch.zeros(1 << 32, dtype=torch.float64, device="cuda")
    table = mg.autotune(mg.F64, reps=2)
    args = (pools, arena, nmax)
    out = serve_trace(mg, synth, seed, rate, seconds, *args, 64 << 30, table)
    short = min(seconds, 10.0)
    out["stress_1gib"] = serve_trace(mg, synth, synth.config_seed(5, 1), rate, short, *args,
                                     1 << 30, table)
    out["saturation"] = [serve_trace(mg, synth, synth.config_seed(5, 2 + i), r,
                                     min(seconds, 3.0), *args, 64 << 30, table)
                         for i, r in enumerate((8000.0, 16000.0, 32000.0, 64000.0))]
    del arena
    torch.cuda.empty_cache()
    out["verify"] = serve_verify(mg, synth, pools, nmax, table)
    del pools
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    """The host CPU's model name (as lscpu reports it, from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    if rows < n and dt < target_s:  # the timed sample: about target_s of work
        rows = min(n, max(rows, int(rows * target_s / dt)))
        A = synth.uniform_pm1(seed, synth.STREAM_A, rows * n).reshape(rows, n)
        C = synth.uniform_pm1(seed, synth.STREAM_C, rows * n).reshape(rows, n)
        t0 = time.perf_counter()
        oracle.dgemm(1.0, A, B, 1.0, C)
        dt = time.perf_counter() - t0
    tflops = 2.0 * rows * n * n / dt / 1e12
    cores = oracle.threads()
    # The whole small workloads, on all cores and on one core.
    small = {}
    for sn in (512, 1024):
        sd = synth.config_seed(1 if sn == 512 else 2)
        A = synth.matrix(sd, synth.STREAM_A, sn, sn)
        Bs = synth.matrix(sd, synth.STREAM_B, sn, sn)
        C = synth.matrix(sd, synth.STREAM_C, sn, sn)
        for tag, th in (("all_cores", cores), ("1_core", 1)):
            oracle.set_threads(th)
            t0 = time.perf_counter()
            oracle.dgemm(1.0, A, Bs, 1.0, C)
            small[f"n{sn}_{tag}_gflops"] = round(2.0 * sn ** 3 / (time.perf_counter() - t0) / 1e9, 3)
    oracle.set_threads(cores)
    return {"value": float(f"{tflops:.6g}"), "unit": "TFLOP/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{rows} of {n} output rows of the n={n} FP64 GEMM ({dt:.1f} s)",
            "small_workloads": small}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--quick", action="store_true", help="headline only (for profiling)")
    ap.add_argument("--leg", choices=["sizes", "trans", "daxpy", "overhead", "split", "batched",
                                      "serving", "profile_batched", "profile_batched_split",
                                      "profile_split", "profile_serving"],
                    default=None,
                    help="run only this secondary leg and print its record (for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="also run one plain device-to-device copy of this many GiB "
                         "(reference kernel for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the GEMM path "
              "here is single-GPU; sharding it over GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1602_08477_amd as mg
    mg.lib()
    if not torch.cuda.is_available():
        eprint("no GPU visible")
        sys.exit(3)
    if args.leg is not None:
        fn = {"split": lambda: bench_split(4096, max(3, args.steps), 1),
              "sizes": lambda: bench_sizes(args.steps, args.warmup),
              "trans": lambda: bench_trans(args.n, args.steps, args.warmup),
              "overhead": bench_overhead,
              "daxpy": lambda: bench_daxpy(1 << 27, args.steps, args.warmup,
                                           cpu=not args.quick, small_n=not args.quick),
              "batched": lambda: bench_batched(max(3, args.steps)),
              "serving": lambda: bench_serving(args.serve_seconds),
              "profile_batched": profile_batched,
              "profile_batched_split": profile_batched_split,
              "profile_split": profile_split,
              "profile_serving": profile_serving}[args.leg]
        print(json.dumps({"leg": args.leg, "record": fn()}), flush=True)
        return
    n = args.n
    eprint(f"bench: native FP64 n={n} steps={args.steps} warmup={args.warmup}")
    ms_step, kern_ms, err, spread = bench_native(n, args.steps, args.warmup)
    if args.copy_gib > 0:
        nb = int(args.copy_gib * 2 ** 30) // 8
        src = torch.ones(nb, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
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
                     "kernel_ms": round(kern_ms, 4), **spread},
    }
    if not args.quick:
        eprint("bench: size sweep")
        rec["sizes"] = bench_sizes(args.steps, args.warmup)
        eprint("bench: operand layouts")
        rec["trans"] = bench_trans(n, args.steps, args.warmup)
        eprint("bench: daxpy n=2^27")
        rec["daxpy"] = bench_daxpy(1 << 27, args.steps, args.warmup)
        eprint("bench: library overhead and naive mapping")
        rec["overhead"] = bench_overhead()
        eprint("bench: split precision n=4096")
        rec["split"] = bench_split(4096, max(5, args.steps), 2)
        eprint("bench: batched 2000 problems")
        rec["batched"] = bench_batched(max(10, args.steps))
        if args.serve_seconds > 0:
            eprint(f"bench: serving {args.serve_seconds:.0f} s")
            rec["serving"] = bench_serving(args.serve_seconds)
        if not args.no_cpu_baseline:
            eprint("bench: cpu baseline (oracle)")
            rec["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
