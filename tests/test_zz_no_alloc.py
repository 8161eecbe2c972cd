"""The batched entry point that allocates nothing (needs a GPU).

mg_gemm_batched_noalloc keeps its work list in the library's static device
buffer: it must give the same bits as mg_gemm_batched (same tile classes, same
kernel) and match the oracle, on two calls in a row with the second batch
smaller than the first (the buffer keeps the first call's list), and reject a
batch whose list does not fit before enqueueing anything.
"""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from helpers import elementwise_bound, log, make_batch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")


def _check_oracle(views, C0, alpha, beta, f32):
    for (A, B, C), c0 in zip(views, C0):
        An, Bn, Cn = (x.double().cpu().numpy() for x in (A, B, c0))
        got = C.double().cpu().numpy()
        ref = oracle.dgemm(alpha, An, Bn, beta, Cn)
        assert oracle.rel_fro_err(got, ref) <= (1e-5 if f32 else 1e-13)
        bound = elementwise_bound(alpha, An, Bn, beta, Cn, An.shape[1],
                                  u=2.0 ** -24 if f32 else 2.0 ** -53)
        assert (np.abs(got - ref) <= bound).all()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_matches_batched_twice(dt):
    dtype = torch.float64 if dt == "f64" else torch.float32
    code = mg.F64 if dt == "f64" else mg.F32
    first = [tuple(int(x) for x in s) for s in synth.batch_shapes(87, 300, 1, 512)]
    second = [tuple(int(x) for x in s) for s in synth.batch_shapes(88, 40, 1, 200)]
    for call, shapes in enumerate((first, second)):
        log(f"noalloc {dt} call {call}: {len(shapes)} problems")
        v1, f1, p1 = make_batch(89 + call, shapes, dtype=dtype, alpha=1.5, beta=0.5)
        v2, f2, p2 = make_batch(89 + call, shapes, dtype=dtype, alpha=1.5, beta=0.5)
        C0 = [C.clone() for _, _, C in v1]
        torch.cuda.synchronize()
        mg.gemm_batched(p1, code)
        mg.gemm_batched_noalloc(p2, code)
        torch.cuda.synchronize()
        assert all(torch.equal(a[2], b[2]) for a, b in zip(v1, v2)), call
        _check_oracle(v2, C0, 1.5, 0.5, dt == "f32")


def test_noalloc_rejects_oversized_list():
    """About 100 000 tiles of 64 x 64 do not fit the 8 MiB list: the call
    fails with MG_ERR_INVALID_ARG before enqueueing, and C is untouched."""
    A = torch.zeros(64, 8, dtype=torch.float64, device="cuda")
    B = torch.zeros(8, 64, dtype=torch.float64, device="cuda")
    Cs = torch.full((100000, 64, 64), 7.0, dtype=torch.float64, device="cuda")
    arr = (mg.Problem * 100000)()
    for i in range(100000):
        arr[i] = mg.problem(A, B, Cs[i], 1.0, 0.0)
    rc = mg.lib().mg_gemm_batched_noalloc(mg.F64, 100000, arr, None)
    assert rc == mg.ERR_INVALID_ARG
    assert "static buffer" in mg.last_error()
    torch.cuda.synchronize()
    assert bool((Cs == 7.0).all())
