"""Cases for the LDS-poison check, run once with the release library and once,
in a child process, with the debug build whose kernels fill every LDS stage
with 0xFF bytes (NaN as FP64 / FP32 / BF16, -1 as INT8) before refilling it
(tests/test_lds_poison_gpu.py compares the two bit for bit).

Every staged kernel takes part: each native work division on 16-byte aligned
rows (direct global->LDS rings) and on unaligned rows (register-staged double
buffer), the transposed layouts, FP32, each split work division (INT8 and
BF16, one k segment and several), the persistent grouped kernel (FP64 and
FP32) and the batched split kernels.  Shapes are ragged in every extent so
tile edges and partial k-steps are exercised.

Child usage: python tests/lds_poison_cases.py OUT.npz
"""

from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))


def run(out_path: str) -> int:
    import numpy as np
    import torch

    import paper_1602_08477_amd as mg
    import synth
    from helpers import make_batch, to_dev

    res = {}

    def put(name, t):
        torch.cuda.synchronize()
        res[name] = t.detach().cpu().numpy()

    m, n, k = 150, 97, 203
    A = synth.matrix(11, synth.STREAM_A, m, k)
    B = synth.matrix(11, synth.STREAM_B, k, n)
    C = synth.matrix(11, synth.STREAM_C, m, n)
    dA, dB = to_dev(A), to_dev(B)
    dAu = to_dev(A, ld=k + 1)  # rows not 16-byte aligned: register-staged tiles
    for cfg in range(mg.num_tile_cfgs()):
        for tag, a_ in (("al", dA), ("un", dAu)):
            c = to_dev(C)
            mg.gemm(a_, dB, c, 1.5, 0.5, cfg=cfg)
            put(f"native_f64_{cfg}_{tag}", c)
    A32, B32, C32 = (torch.from_numpy(x).float().cuda() for x in (A, B, C))
    for cfg in (None, 0, 5, 14):
        c = C32.clone()
        mg.gemm(A32, B32, c, 1.5, 0.5, cfg=cfg)
        put(f"native_f32_{cfg}", c)
    At, Bt = dA.t().contiguous(), dB.t().contiguous()
    for ta in (False, True):
        for tb in (False, True):
            for cfg in (None, 0, 20):
                c = to_dev(C)
                mg.gemm_ex(At if ta else dA, Bt if tb else dB, c, 1.5, 0.5, transa=ta,
                           transb=tb, cfg=cfg)
                put(f"trans_{int(ta)}{int(tb)}_{cfg}", c)

    sA = synth.matrix(12, synth.STREAM_A, 200, 300, kind="spread")
    sB = synth.matrix(12, synth.STREAM_B, 300, 150, kind="spread")
    sC = synth.matrix(12, synth.STREAM_C, 200, 150)
    dsA, dsB = to_dev(sA), to_dev(sB)
    for algo in (mg.SPLIT_I8, mg.SPLIT_BF16):
        for cfg in range(mg.split_num_cfgs()):
            c = to_dev(sC)
            mg.gemm_split(dsA, dsB, c, 1.0, 1.0, algo=algo, cfg=cfg)
            put(f"split_{algo}_{cfg}", c)
        # several exact-INT32 k segments
        kl = 20000 if algo == mg.SPLIT_I8 else 6000
        lA = synth.matrix(13, synth.STREAM_A, 40, kl, kind="spread")
        lB = synth.matrix(13, synth.STREAM_B, kl, 48, kind="spread")
        c = torch.zeros(40, 48, dtype=torch.float64, device="cuda")
        mg.gemm(to_dev(lA), to_dev(lB), c, 1.0, 0.0, algo=algo)
        put(f"split_{algo}_longk", c)

    for dt, code in ((torch.float64, mg.F64), (torch.float32, mg.F32)):
        shapes = [tuple(int(x) for x in s) for s in synth.batch_shapes(14, 60, 1, 300)]
        views, flats, probs = make_batch(14, shapes, dtype=dt)
        mg.gemm_batched(probs, dtype=code)
        put(f"grouped_{code}", flats["C"])
        del views, flats, probs
    shapes = [tuple(int(x) for x in s) for s in synth.batch_shapes(15, 30, 1, 400)]
    for algo in (mg.SPLIT_I8, mg.SPLIT_BF16):
        views, flats, probs = make_batch(15, shapes)
        mg.gemm_batched(probs, dtype=mg.F64, algo=algo)
        put(f"batched_split_{algo}", flats["C"])
        del views, flats, probs
    res["build_flags"] = np.array([mg.build_flags()], dtype=np.int32)
    np.savez(out_path, **res)
    return len(res)


if __name__ == "__main__":
    print(f"lds poison cases: {run(sys.argv[1])} outputs written", flush=True)
