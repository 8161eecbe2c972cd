"""The continuous-batching GEMM server (needs a GPU).

Checks: results against the oracle; every request's result is bit-identical
when it runs alone and when it runs inside a Poisson mix (the per-request
arithmetic depends only on its own shape); admission keeps the admitted
bytes within the budget and the slot limit; oversized requests and a full
queue are rejected; batches really contain several requests and batches on
different streams overlap in time.
"""

import ctypes

import numpy as np
import pytest

import oracle
import synth
from helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")


def make_trace(seed, count, rate, lo, hi, split_frac=0.3):
    """Poisson arrivals, square n log-uniform in [lo, hi], a split_frac share
    of split-INT8 requests, operands U[-1,1) per request."""
    gaps = synth.poisson_gaps(seed, synth.STREAM_ARRIVALS, count, rate)
    t = np.cumsum(gaps) - gaps[0]
    ns = synth.log_uniform_int(seed, synth.STREAM_SIZES, count, lo, hi)
    mix = synth.uniform_unit(seed, synth.STREAM_MIX, count)
    algos = np.where(mix < split_frac, mg.SPLIT_I8, mg.NATIVE)
    ops = []
    for i, n in enumerate(ns):
        n = int(n)
        A = synth.uniform_pm1(seed + i, 0, n * n, device="cuda").view(n, n)
        B = synth.uniform_pm1(seed + i, 1, n * n, device="cuda").view(n, n)
        C = synth.uniform_pm1(seed + i, 2, n * n, device="cuda").view(n, n)
        ops.append((A, B, C, C.clone()))
    reqs = (mg.Request * count)()
    for i, (A, B, C, _) in enumerate(ops):
        reqs[i] = mg.Request(mg.F64, int(algos[i]), mg.problem(A, B, C, 1.0, 1.0),
                             int(t[i] * 1e9))
    return reqs, ops, algos


def test_submit_wait_matches_oracle():
    with mg.Server(n_streams=2) as srv:
        cases = []
        for i, (n, algo) in enumerate([(33, mg.NATIVE), (200, mg.SPLIT_I8), (129, mg.NATIVE),
                                       (64, mg.SPLIT_BF16)]):
            A = synth.matrix(90 + i, 0, n, n + 3, device="cuda")
            B = synth.matrix(90 + i, 1, n + 3, n, device="cuda")
            C = synth.matrix(90 + i, 2, n, n, device="cuda")
            C0 = C.clone()
            t = srv.submit(A, B, C, 1.5, 0.5, algo=algo)
            cases.append((t, A, B, C, C0, algo))
        for t, A, B, C, C0, algo in cases:
            r = srv.wait(t)
            assert r["status"] == mg.OK
            assert r["t_arrival_ns"] <= r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_launch_ns"] \
                <= r["t_done_ns"]
            ref = oracle.dgemm(1.5, A.cpu().numpy(), B.cpu().numpy(), 0.5, C0.cpu().numpy())
            err = oracle.rel_fro_err(C.cpu().numpy(), ref)
            assert err <= (1e-13 if algo == mg.NATIVE else 1e-12), (algo, err)
        with pytest.raises(mg.MgError):
            srv.poll(cases[0][0])  # ticket released after the result was taken


def test_alone_equals_in_mix_and_oracle():
    seed = synth.config_seed(5, 1)
    count = 400
    reqs, ops, algos = make_trace(seed, count, 4000.0, 32, 256)
    with mg.Server(n_streams=4, max_batch=32) as srv:
        res = srv.replay(reqs)
        st = srv.stats()
    log(f"mix stats: {st}")
    assert all(r.status == mg.OK for r in res)
    assert st["completed"] == count and st["max_batch_seen"] > 1
    mixed = [C.clone() for _, _, C, _ in ops]
    # every request alone, on a fresh server, from the same initial C
    with mg.Server(n_streams=1) as alone:
        for i, (A, B, C, C0) in enumerate(ops):
            C.copy_(C0)
            t = alone.submit(A, B, C, 1.0, 1.0, algo=int(algos[i]))
            assert alone.wait(t)["status"] == mg.OK
            assert torch.equal(C, mixed[i]), f"request {i} differs alone vs in the mix"
    # every request against the oracle (well over 1 % and 200 of the mix)
    for i in range(count):
        A, B, _, C0 = ops[i]
        ref = oracle.dgemm(1.0, A.cpu().numpy(), B.cpu().numpy(), 1.0, C0.cpu().numpy())
        err = oracle.rel_fro_err(mixed[i].cpu().numpy(), ref)
        assert err <= (1e-13 if algos[i] == mg.NATIVE else 1e-12), (i, err)
    # batches on different streams overlapped in time
    iv = sorted({(r.batch_id, r.t_launch_ns, r.t_done_ns) for r in res}, key=lambda x: x[1])
    overlaps = sum(1 for a, b in zip(iv, iv[1:]) if b[1] < a[2])
    log(f"batches {len(iv)}, overlapping consecutive batches {overlaps}")
    assert overlaps > 0


def test_admission_respects_budget_and_slots():
    n = 256
    per_req = 3 * n * n * 8
    budget = 3 * per_req + 1000
    with mg.Server(n_streams=4, max_slots=2, hbm_budget_bytes=budget) as srv:
        ops, tickets = [], []
        for i in range(24):
            A = synth.matrix(95, 0, n, n, device="cuda")
            B = synth.matrix(95, 1, n, n, device="cuda")
            C = torch.zeros(n, n, dtype=torch.float64, device="cuda")
            ops.append((A, B, C))
            tickets.append(srv.submit(A, B, C))
        for t in tickets:
            assert srv.wait(t)["status"] == mg.OK
        st = srv.stats()
        assert st["max_inflight_bytes"] <= budget
        assert st["max_slots_used"] <= 2
        An, Bn = ops[0][0].cpu().numpy(), ops[0][1].cpu().numpy()
        ref = oracle.dgemm(1.0, An, Bn, 0.0, None)
        assert oracle.rel_fro_err(ops[0][2].cpu().numpy(), ref) <= 1e-13
        # the same problem 24 times: every copy has the same bits
        assert all(torch.equal(C, ops[0][2]) for _, _, C in ops)
        big = torch.zeros(512, 512, dtype=torch.float64, device="cuda")
        with pytest.raises(mg.MgError) as ei:
            srv.submit(big, big.clone(), big.clone())
        assert ei.value.code == mg.ERR_NO_MEMORY
        assert srv.stats()["rejected_memory"] == 1


def test_queue_full_is_busy():
    n = 4096
    A = synth.matrix(96, 0, n, n, device="cuda")
    B = synth.matrix(96, 1, n, n, device="cuda")
    Cs = [torch.zeros(n, n, dtype=torch.float64, device="cuda") for _ in range(8)]
    with mg.Server(n_streams=1, max_slots=1, max_queue=2) as srv:
        tickets, busy = [], 0
        for C in Cs:
            try:
                tickets.append(srv.submit(A, B, C))
            except mg.MgError as e:
                assert e.code == mg.ERR_BUSY
                busy += 1
        for t in tickets:
            assert srv.wait(t)["status"] == mg.OK
        assert busy > 0 and srv.stats()["rejected_busy"] == busy


def test_invalid_request_rejected_before_queueing():
    with mg.Server(n_streams=1) as srv:
        A = torch.zeros(8, 8, dtype=torch.float64, device="cuda")
        r = mg.Request(mg.F64, mg.NATIVE, mg.Problem(8, 8, 8, 1.0, 0.0, A.data_ptr(), 8,
                                                       A.data_ptr(), 8, A.data_ptr(), 8), 0)
        t = ctypes.c_uint64()
        assert mg.lib().mg_gemm_submit(srv._h, ctypes.byref(r), ctypes.byref(t)) \
            == mg.ERR_INVALID_ARG
        r.algo = mg.SPLIT_I8
        r.dtype = mg.F32
        assert mg.lib().mg_gemm_submit(srv._h, ctypes.byref(r), ctypes.byref(t)) \
            == mg.ERR_UNSUPPORTED
        assert srv.stats()["submitted"] == 0


def test_large_native_requests_run_direct_and_match():
    """Native requests of at least 1024^3 multiply-adds run as their own
    launch inside a batch; the result equals the library call alone (bit for
    bit) and the oracle on sampled outputs."""
    m, n, k = 1100, 1030, 1000
    A = synth.matrix(97, 0, m, k, device="cuda")
    B = synth.matrix(97, 1, k, n, device="cuda")
    C = synth.matrix(97, 2, m, n, device="cuda")
    C0 = C.clone()
    small = [(synth.matrix(98 + i, 0, 64, 64, device="cuda"),
              synth.matrix(98 + i, 1, 64, 64, device="cuda"),
              torch.zeros(64, 64, dtype=torch.float64, device="cuda")) for i in range(4)]
    with mg.Server(n_streams=1, max_batch=16) as srv:
        ts = [srv.submit(a, b, c) for a, b, c in small]
        tl = srv.submit(A, B, C, 1.0, 1.0)
        for t in ts:
            assert srv.wait(t)["status"] == mg.OK
        assert srv.wait(tl)["status"] == mg.OK
    alone = C0.clone()
    mg.gemm(A, B, alone, 1.0, 1.0)
    torch.cuda.synchronize()
    assert torch.equal(alone, C)
    rows = np.array([0, 1, 517, m - 1])
    cols = np.array([0, 3, 640, n - 1])
    ref = oracle.dgemm_sampled(1.0, A.cpu().numpy(), B.cpu().numpy(), 1.0, C0.cpu().numpy(),
                               rows, cols)
    got = C.cpu().numpy()[np.ix_(rows, cols)]
    assert oracle.rel_fro_err(got, ref) <= 1e-13
    for a, b, c in small:
        ref = oracle.dgemm(1.0, a.cpu().numpy(), b.cpu().numpy(), 0.0, None)
        assert oracle.rel_fro_err(c.cpu().numpy(), ref) <= 1e-13


def test_config5_trace_alone_equals_mix_and_oracle():
    """Workload 5 as run: 2 s of Poisson arrivals at 2000 requests/s, square
    n log-uniform in [32, 2048], 70 % native / 30 % split INT8, alpha = beta
    = 1, every request with its own C (A and B are views of resident
    operand pools).  Every request must give the same bits alone as in the
    mix; 1 % of the requests (at least 200) and every request with n >= 1024
    are checked against the oracle (full outputs below n = 512, sampled
    rows and columns above)."""
    seed = synth.config_seed(5, 3)
    rate, seconds = 2000.0, 2.0
    count = int(rate * seconds)
    gaps = synth.poisson_gaps(seed, synth.STREAM_ARRIVALS, count, rate)
    t_arr = np.cumsum(gaps) - gaps[0]
    ns = synth.log_uniform_int(seed, synth.STREAM_SIZES, count, 32, 2048).astype(np.int64)
    mix = synth.uniform_unit(seed, synth.STREAM_MIX, count)
    algos = np.where(mix < 0.3, mg.SPLIT_I8, mg.NATIVE)
    pool = 1 << 25
    pa = synth.flat_uniform(seed, 0, pool, device="cuda")
    pb = synth.flat_uniform(seed, 1, pool, device="cuda")
    offs = (synth.uniform_unit(seed, 12, count) * (pool - ns * ns)).astype(np.int64) // 32 * 32
    c_off = np.concatenate([[0], np.cumsum((ns * ns + 31) // 32 * 32)])
    log(f"config5 trace: {count} requests, C arena {c_off[-1] * 8 / 2**30:.1f} GiB, "
        f"n >= 1024: {int((ns >= 1024).sum())}, split: {int((algos != mg.NATIVE).sum())}")
    C0 = synth.flat_uniform(seed, 2, int(c_off[-1]), device="cuda")
    C = C0.clone()

    def views(i):
        n = int(ns[i])
        a = pa[offs[i]: offs[i] + n * n].view(n, n)
        b = pb[offs[i]: offs[i] + n * n].view(n, n)
        c = C[c_off[i]: c_off[i] + n * n].view(n, n)
        c0 = C0[c_off[i]: c_off[i] + n * n].view(n, n)
        return a, b, c, c0

    reqs = (mg.Request * count)()
    for i in range(count):
        a, b, c, _ = views(i)
        reqs[i] = mg.Request(mg.F64, int(algos[i]), mg.problem(a, b, c, 1.0, 1.0),
                             int(t_arr[i] * 1e9))
    with mg.Server(n_streams=4, max_batch=64, hbm_budget_bytes=64 << 30) as srv:
        res = srv.replay(reqs)
        st = srv.stats()
    log(f"config5 mix stats: {st}")
    assert all(r.status == mg.OK for r in res)
    assert st["completed"] == count
    mixed = C.clone()
    C.copy_(C0)
    torch.cuda.synchronize()
    with mg.Server(n_streams=1, max_batch=1) as alone:
        for i in range(count):
            a, b, c, _ = views(i)
            assert alone.wait(alone.submit(a, b, c, 1.0, 1.0, algo=int(algos[i])))["status"] \
                == mg.OK
    torch.cuda.synchronize()
    for i in range(count):
        lo, hi = int(c_off[i]), int(c_off[i] + ns[i] * ns[i])
        assert torch.equal(C[lo:hi], mixed[lo:hi]), f"request {i} (n={ns[i]}) alone != mix"
    # oracle: a seeded 1 % sample (at least 200) plus every n >= 1024
    pick = np.unique(np.concatenate([
        (synth.uniform_unit(seed, 13, max(200, count // 100)) * count).astype(np.int64),
        np.nonzero(ns >= 1024)[0]]))
    worst = {mg.NATIVE: 0.0, mg.SPLIT_I8: 0.0}
    for i in pick:
        n = int(ns[i])
        a, b, _, c0 = views(i)
        lo = int(c_off[i])
        got = mixed[lo: lo + n * n].view(n, n)
        if n < 512:
            ref = oracle.dgemm(1.0, a.cpu().numpy(), b.cpu().numpy(), 1.0, c0.cpu().numpy())
            g = got.cpu().numpy()
        else:
            r = np.unique(np.concatenate([[0, n - 1],
                                          (synth.uniform_unit(seed + int(i), 14, 14) * n).astype(int)]))
            cidx = np.unique(np.concatenate([[0, n - 1],
                                             (synth.uniform_unit(seed + int(i), 15, 14) * n).astype(int)]))
            rt, ct = torch.from_numpy(r).cuda(), torch.from_numpy(cidx).cuda()
            ref = oracle.dgemm(1.0, a[rt].cpu().numpy(), b[:, ct].cpu().numpy(), 1.0,
                               c0[rt][:, ct].cpu().numpy())
            g = got[rt][:, ct].cpu().numpy()
        err = oracle.rel_fro_err(g, ref)
        assert err <= (1e-13 if algos[i] == mg.NATIVE else 1e-12), (int(i), n, int(algos[i]), err)
        worst[int(algos[i])] = max(worst[int(algos[i])], err)
    log(f"config5: {count} requests bit-identical alone vs mix; {len(pick)} checked against the "
        f"oracle, worst native {worst[mg.NATIVE]:.3e}, split {worst[mg.SPLIT_I8]:.3e}")


def test_submit_waits_for_producer_writes():
    """A request submitted right after torch enqueued the writes of its C
    (a long product on the current stream, no synchronisation) runs after
    them: the server's lane waits on the event Server.submit records."""
    n = 256
    X = synth.matrix(99, 3, 4096, 4096, device="cuda")
    A = synth.matrix(99, 0, n, n, device="cuda")
    B = synth.matrix(99, 1, n, n, device="cuda")
    C = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with mg.Server(n_streams=2) as srv:
        for rep in range(3):
            C.zero_()
            Y = X @ X  # several milliseconds of work ahead of the write of C
            C.copy_(Y[:n, :n])
            t = srv.submit(A, B, C, 1.0, 1.0)
            assert srv.wait(t)["status"] == mg.OK
            torch.cuda.synchronize()
            ref = oracle.dgemm(1.0, A.cpu().numpy(), B.cpu().numpy(), 1.0,
                               Y[:n, :n].cpu().numpy())
            assert oracle.rel_fro_err(C.cpu().numpy(), ref) <= 1e-13, rep
