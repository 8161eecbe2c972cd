"""Host logic of the serving loop, run in the server's host-simulation mode
(no GPU: batches "run" for a modeled duration, operands are never touched).

Covers admission against the byte budget and slot limit, FIFO admission,
rejection of oversized requests and of submissions to a full queue,
continuous batching (requests that arrive while a batch runs go out
together in the next one), open-loop replay, and draining on destroy.
"""

import ctypes
import time

import numpy as np
import pytest

import paper_1602_08477_amd as mg
import synth

BASE = 0x100000000  # fake device addresses, validated but never dereferenced


class FakeOperands:
    """Distinct, aligned, non-overlapping fake address ranges per request."""

    def __init__(self):
        self.next = BASE

    def take(self, nbytes):
        p = self.next
        self.next += (nbytes + 4095) // 4096 * 4096 + 4096
        return p

    def request(self, n, algo=mg.NATIVE, t_arrival_ns=0, m=None, k=None):
        m = m or n
        k = k or n
        A = self.take(m * k * 8)
        B = self.take(k * n * 8)
        C = self.take(m * n * 8)
        return mg.Request(mg.F64, algo, mg.Problem(m, n, k, 1.0, 1.0, A, k, B, n, C, n),
                          t_arrival_ns)


def req_bytes(n):
    return 3 * n * n * 8


def test_budget_slots_and_fifo():
    ops = FakeOperands()
    n = 512
    budget = 3 * req_bytes(n) + 100
    with mg.Server(n_streams=4, max_slots=3, hbm_budget_bytes=budget, simulate=True,
                   sim_tflops=2.0, sim_launch_ns=50000) as srv:
        tickets = [srv.submit_request(ops.request(n)) for _ in range(40)]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(r["status"] == mg.OK for r in res)
    assert st["completed"] == 40 and st["submitted"] == 40
    assert st["max_inflight_bytes"] <= budget
    assert st["max_slots_used"] <= 3
    admits = [r["t_admit_ns"] for r in res]
    assert admits == sorted(admits), "admission must follow submission order"
    for r in res:
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_launch_ns"] <= r["t_done_ns"]


def test_oversized_request_rejected():
    ops = FakeOperands()
    with mg.Server(hbm_budget_bytes=req_bytes(256), simulate=True) as srv:
        with pytest.raises(mg.MgError) as ei:
            srv.submit_request(ops.request(512))
        assert ei.value.code == mg.ERR_NO_MEMORY
        # split requests also count their workspace
        L = mg.split_layout(mg.SPLIT_I8, mg.split_default_slices(mg.SPLIT_I8), 200, 200, 200)
        assert req_bytes(200) + L["total_bytes"] > req_bytes(256)
        with pytest.raises(mg.MgError):
            srv.submit_request(ops.request(200, algo=mg.SPLIT_I8))
        t = srv.submit_request(ops.request(200))
        assert srv.wait(t)["status"] == mg.OK
        assert srv.stats()["rejected_memory"] == 2


def test_full_queue_is_busy():
    ops = FakeOperands()
    with mg.Server(n_streams=1, max_slots=1, max_queue=2, simulate=True, sim_tflops=0.001,
                   sim_launch_ns=0) as srv:
        ok, busy = [], 0
        for _ in range(10):
            try:
                ok.append(srv.submit_request(ops.request(64)))
            except mg.MgError as e:
                assert e.code == mg.ERR_BUSY
                busy += 1
        assert busy >= 6 and srv.stats()["rejected_busy"] == busy
        for t in ok:
            assert srv.wait(t)["status"] == mg.OK


def test_continuous_batching_groups_late_arrivals():
    ops = FakeOperands()
    with mg.Server(n_streams=1, max_batch=64, simulate=True, sim_tflops=1.0,
                   sim_launch_ns=0) as srv:
        # ~17 ms modeled: the late requests all arrive while it runs, even on
        # a loaded host
        first = srv.submit_request(ops.request(2048))
        deadline = time.time() + 5.0
        while srv.stats()["batches"] < 1 and time.time() < deadline:
            time.sleep(0.0002)  # the first request is taken as a batch of its own
        assert srv.stats()["batches"] == 1
        late = [srv.submit_request(ops.request(64)) for _ in range(10)]
        r0 = srv.wait(first)
        rl = [srv.wait(t) for t in late]
    assert r0["batch_size"] == 1
    assert len({r["batch_id"] for r in rl}) == 1 and rl[0]["batch_size"] == 10
    assert rl[0]["batch_id"] != r0["batch_id"]
    assert all(r["t_launch_ns"] >= r0["t_done_ns"] for r in rl)


def test_batches_overlap_across_streams():
    ops = FakeOperands()
    # each simulated batch lasts ~3 ms, far longer than the scheduler needs
    # to hand the next request to a free lane even on a loaded host
    with mg.Server(n_streams=3, max_batch=1, simulate=True, sim_tflops=0.01,
                   sim_launch_ns=0) as srv:
        ts = [srv.submit_request(ops.request(256)) for _ in range(6)]
        res = [srv.wait(t) for t in ts]
    # with max_batch 1 and 3 lanes, up to three batches are in flight at once
    iv = sorted((r["t_launch_ns"], r["t_done_ns"]) for r in res)
    assert any(b[0] < a[1] for a, b in zip(iv, iv[1:]))


def test_replay_poisson_open_loop():
    seed = synth.config_seed(5, 7)
    count, rate = 600, 3000.0
    gaps = synth.poisson_gaps(seed, synth.STREAM_ARRIVALS, count, rate)
    t = np.cumsum(gaps) - gaps[0]
    ns = synth.log_uniform_int(seed, synth.STREAM_SIZES, count, 32, 512)
    mix = synth.uniform_unit(seed, synth.STREAM_MIX, count)
    ops = FakeOperands()
    reqs = (mg.Request * count)()
    for i in range(count):
        reqs[i] = ops.request(int(ns[i]), mg.SPLIT_I8 if mix[i] < 0.3 else mg.NATIVE,
                              int(t[i] * 1e9))
    with mg.Server(n_streams=4, simulate=True, sim_tflops=20.0, sim_launch_ns=20000) as srv:
        res = srv.replay(reqs)
        st = srv.stats()
    assert st["completed"] == count and all(r.status == mg.OK for r in res)
    arr = np.array([r.t_arrival_ns for r in res], dtype=np.int64)
    d = np.diff(arr) / 1e9
    # submitted on schedule (open loop); a loaded host may delay a few
    dev = np.abs(d - np.diff(t))
    assert np.median(dev) < 2e-4 and np.quantile(dev, 0.99) < 5e-3
    lat = np.array([(r.t_done_ns - r.t_arrival_ns) / 1e6 for r in res])
    assert (lat > 0.019).all() and np.percentile(lat, 50) < 50
    assert st["max_batch_seen"] >= 1


def test_destroy_drains_pending_requests():
    ops = FakeOperands()
    srv = mg.Server(n_streams=2, simulate=True, sim_tflops=5.0)
    for _ in range(20):
        srv.submit_request(ops.request(256))
    srv.close()  # returns only after all 20 have completed


def test_bad_options_and_requests():
    with pytest.raises(mg.MgError):
        mg.Server(n_streams=0, simulate=True)
    with pytest.raises(mg.MgError):
        mg.Server(simulate=True, sim_tflops=0.0)
    ops = FakeOperands()
    with mg.Server(simulate=True) as srv:
        r = ops.request(64)
        r.p.C = r.p.A  # output overlapping an operand
        with pytest.raises(mg.MgError):
            srv.submit_request(r)
        r = ops.request(64)
        r.dtype = mg.F32
        r.algo = mg.SPLIT_I8
        with pytest.raises(mg.MgError) as ei:
            srv.submit_request(r)
        assert ei.value.code == mg.ERR_UNSUPPORTED
        with pytest.raises(mg.MgError) as ei:
            srv.poll(12345)
        assert ei.value.code == mg.ERR_NOT_FOUND
        assert srv.stats()["submitted"] == 0
