"""Batched uneven GEMMs in one persistent launch (needs a GPU).

Each problem must match the oracle (FP64: 1e-13 and the per-element rounding
bound; FP32: 1e-5 on FP32-rounded inputs).  Every tile runs the same k-loop as
the single-problem kernel whatever its tile class, so each batched result must
also equal the single-problem library call bit for bit ("alone" vs "in the
mix").  Graph replays are checked against eager launches, several times, with
eager work in between.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import U32, elementwise_bound, log, make_batch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")


def check_problem(A, B, C0, got, alpha, beta, f32=False):
    A = A.double().cpu().numpy()
    B = B.double().cpu().numpy()
    C0 = C0.double().cpu().numpy()
    got = got.double().cpu().numpy()
    ref = oracle.dgemm(alpha, A, B, beta, C0)
    err = oracle.rel_fro_err(got, ref)
    bound = elementwise_bound(alpha, A, B, beta, C0, A.shape[1], u=U32 if f32 else 2.0 ** -53)
    assert err <= (1e-5 if f32 else 1e-13), err
    assert (np.abs(got - ref) <= bound).all()
    return err


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batch_matches_oracle_and_single_calls(dt):
    dtype = torch.float64 if dt == "f64" else torch.float32
    code = mg.F64 if dt == "f64" else mg.F32
    shapes = [tuple(int(x) for x in s) for s in synth.batch_shapes(81, 60, 1, 300)]
    shapes += [(1, 1, 1), (33, 1, 7), (1, 40, 513), (128, 64, 16), (65, 65, 65)]
    views, flats, probs = make_batch(81, shapes, dtype=dtype, alpha=1.5, beta=0.5)
    C0 = [c.clone() for _, _, c in views]
    plan = mg.Plan(code, probs)
    plan.launch()
    torch.cuda.synchronize()
    st = plan.stats()
    log(f"batch {dt}: {st}")
    assert st["problems"] == len(shapes) and st["graph"] == 1
    worst = 0.0
    for (A, B, C), c0 in zip(views, C0):
        worst = max(worst, check_problem(A, B, c0, C, 1.5, 0.5, f32=(dt == "f32")))
        alone = c0.clone()
        mg.gemm(A, B, alone, 1.5, 0.5)
        torch.cuda.synchronize()
        assert torch.equal(alone, C), "batched result differs from the single call"
    log(f"batch {dt}: worst rel_fro_err {worst:.3e}")


def test_tile_classes_agree_bitwise():
    """Forcing each tile class through the tuning table gives identical bits."""
    shapes = [(97, 131, 77), (200, 64, 300), (31, 257, 45)]
    outs = []
    for c in range(mg.NUM_GROUPED_CLASSES):
        views, flats, probs = make_batch(82, shapes)
        t = mg.TuneTable.from_list(mg.F64, [c] * mg.TUNE_BUCKETS)
        plan = mg.Plan(mg.F64, probs, t)
        plan.launch()
        torch.cuda.synchronize()
        assert plan.stats()["tiles_per_class"][c] == plan.stats()["tiles"]
        outs.append([C.clone() for _, _, C in views])
    for o in outs[1:]:
        assert all(torch.equal(a, b) for a, b in zip(outs[0], o))


def padded_copy(X, aligned, dtype):
    """X in a buffer whose row pitch is a multiple of 8 elements (16-byte rows
    for FP64 and FP32) or odd; the padding holds NaN."""
    r, c = X.shape
    pitch = (c + 7) // 8 * 8 + 8 if aligned else c + 1 + (c % 2)
    big = torch.full((r, pitch), float("nan"), dtype=dtype, device="cuda")
    big[:, :c] = X
    return big, big[:, :c]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_operand_alignment_paths_agree_bitwise(dt):
    """A with 16-byte rows streams through 16-byte loads (so does FP64 B,
    which then lands row-major in LDS), odd pitches through 4-byte loads;
    every class gives the same bits for all four combinations (m, n, k
    ragged against the 16-byte chunks and the tiles)."""
    dtype = torch.float64 if dt == "f64" else torch.float32
    code = mg.F64 if dt == "f64" else mg.F32
    shapes = [(97, 131, 78), (200, 64, 300), (31, 257, 46), (64, 64, 16), (5, 3, 2), (70, 33, 129)]
    for c in range(mg.NUM_GROUPED_CLASSES):
        t = mg.TuneTable.from_list(code, [c] * mg.TUNE_BUCKETS)
        outs = []
        for a_al, b_al in ((True, True), (False, False), (True, False), (False, True)):
            probs, Cs, keep = [], [], []
            for i, (m_, n_, k_) in enumerate(shapes):
                A = synth.matrix(85 + i, 0, m_, k_, device="cuda").to(dtype)
                B = synth.matrix(85 + i, 1, k_, n_, device="cuda").to(dtype)
                C = synth.matrix(85 + i, 2, m_, n_, device="cuda").to(dtype)
                Abig, Av = padded_copy(A, a_al, dtype)
                Bbig, Bv = padded_copy(B, b_al, dtype)
                keep += [Abig, Bbig]
                probs.append(mg.problem(Av, Bv, C, 1.25, 0.5))
                Cs.append(C)
            plan = mg.Plan(code, probs, t)
            plan.launch()
            torch.cuda.synchronize()
            outs.append([C.clone() for C in Cs])
            plan.close()
        for o in outs[1:]:
            assert all(torch.equal(a, b) for a, b in zip(outs[0], o)), (dt, c)
        # and against the oracle, so that all four are not wrong alike
        if dt == "f64":
            for i, (m_, n_, k_) in enumerate(shapes):
                A = synth.matrix(85 + i, 0, m_, k_)
                B = synth.matrix(85 + i, 1, k_, n_)
                C0 = synth.matrix(85 + i, 2, m_, n_)
                check_problem(torch.from_numpy(A), torch.from_numpy(B), torch.from_numpy(C0),
                              outs[0][i], 1.25, 0.5)


def test_graph_replays_match_eager():
    shapes = [tuple(int(x) for x in s) for s in synth.batch_shapes(83, 40, 16, 256)]
    views, flats, probs = make_batch(83, shapes, beta=0.0)
    plan = mg.Plan(mg.F64, probs)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    eager = [C.clone() for _, _, C in views]
    for rep in range(4):
        for _, _, C in views:
            C.fill_(float("nan"))  # eager work between replays; beta=0 ignores it
        torch.cuda.synchronize()
        plan.launch(graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(e, C) for e, (_, _, C) in zip(eager, views)), rep


def test_special_problems_in_batch():
    dev = "cuda"
    d = torch.float64
    A = synth.matrix(84, 0, 50, 40, device=dev)
    B = synth.matrix(84, 1, 40, 30, device=dev)
    nanC = torch.full((50, 30), float("nan"), dtype=d, device=dev)
    C1 = synth.matrix(84, 2, 50, 30, device=dev)
    C1_0 = C1.clone()
    C2 = synth.matrix(84, 3, 50, 30, device=dev)
    C2_0 = C2.clone()
    nanA = torch.full((50, 40), float("nan"), dtype=d, device=dev)
    big = torch.zeros(60, 45, dtype=d, device=dev)
    Cu = big[1:51, 1:31]  # 8-byte aligned, odd pitch: scalar path
    empty = torch.empty(0, 30, dtype=d, device=dev)
    probs = [mg.problem(A, B, nanC, 1.0, 0.0),          # beta = 0 ignores NaN C
             mg.problem(nanA, B, C1, 0.0, 2.0),         # alpha = 0 ignores NaN A
             mg.Problem(50, 30, 0, 1.0, 0.5, None, 1, None, 1, C2.data_ptr(), 30),  # k = 0
             mg.problem(A, B, Cu, 1.0, 0.0),
             mg.problem(torch.empty(0, 40, dtype=d, device=dev), B, empty, 1.0, 0.0)]
    plan = mg.Plan(mg.F64, probs)
    plan.launch()
    torch.cuda.synchronize()
    An, Bn = A.cpu().numpy(), B.cpu().numpy()
    ref = oracle.dgemm(1.0, An, Bn, 0.0, None)
    bound = elementwise_bound(1.0, An, Bn, 0.0, None, 40)
    assert torch.isfinite(nanC).all()
    assert oracle.rel_fro_err(nanC.cpu().numpy(), ref) <= 1e-13
    assert (np.abs(nanC.cpu().numpy() - ref) <= bound).all()
    assert torch.equal(C1, 2.0 * C1_0)
    assert torch.equal(C2, 0.5 * C2_0)
    assert oracle.rel_fro_err(Cu.cpu().numpy(), ref) <= 1e-13
    assert (np.abs(Cu.cpu().numpy() - ref) <= bound).all()
    assert plan.stats()["scale_tiles"] > 0


def test_overlapping_outputs_rejected():
    C = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    A = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    p1 = mg.problem(A[:40], A, C[:40], 1.0, 0.0)
    p2 = mg.problem(A[:30], A, C[30:60], 1.0, 0.0)
    with pytest.raises(mg.MgError, match="overlap"):
        mg.Plan(mg.F64, [p1, p2])
    p3 = mg.problem(A, A, A, 1.0, 0.0)  # C overlaps its own A
    with pytest.raises(mg.MgError, match="overlaps"):
        mg.Plan(mg.F64, [p3])


def test_one_shot_batched_matches_plan():
    shapes = [tuple(int(x) for x in s) for s in synth.batch_shapes(85, 30, 16, 200)]
    v1, f1, p1 = make_batch(85, shapes)
    v2, f2, p2 = make_batch(85, shapes)
    mg.Plan(mg.F64, p1).launch()
    mg.gemm_batched(p2, mg.F64)
    torch.cuda.synchronize()
    assert all(torch.equal(a[2], b[2]) for a, b in zip(v1, v2))


def test_autotune_table_valid():
    t = mg.autotune(mg.F64, reps=1)
    vals = t.to_list()
    assert len(vals) == mg.TUNE_BUCKETS and all(0 <= v < mg.NUM_GROUPED_CLASSES for v in vals)
    log(f"autotune classes histogram: {np.bincount(vals, minlength=3).tolist()}")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_config4_2000_problems_all(dt):
    """Workload 4: 2000 problems, m, n, k log-uniform in [16, 512], one
    persistent graph launch with an autotuned table; every problem against
    the oracle element by element (1e-13 / 1e-5 and the per-element rounding
    bound), so a dropped or doubled tile fails."""
    dtype = torch.float64 if dt == "f64" else torch.float32
    code = mg.F64 if dt == "f64" else mg.F32
    seed = synth.config_seed(4)
    shapes = [tuple(int(x) for x in s) for s in synth.batch_shapes(seed, 2000)]
    views, flats, probs = make_batch(seed, shapes, dtype=dtype)
    C0 = [C.double().cpu().numpy() for _, _, C in views]
    table = mg.autotune(code, reps=1)
    plan = mg.Plan(code, probs, table)
    plan.launch()
    torch.cuda.synchronize()
    log(f"config4 {dt}: {plan.stats()}")
    worst = 0.0
    for i, (A, B, C) in enumerate(views):
        A = A.double().cpu().numpy()
        B = B.double().cpu().numpy()
        got = C.double().cpu().numpy()
        ref = oracle.dgemm(1.0, A, B, 1.0, C0[i])
        err = oracle.rel_fro_err(got, ref)
        assert err <= (1e-5 if dt == "f32" else 1e-13), (i, shapes[i], err)
        bound = elementwise_bound(1.0, A, B, 1.0, C0[i], A.shape[1],
                                  u=U32 if dt == "f32" else 2.0 ** -53)
        assert (np.abs(got - ref) <= bound).all(), (i, shapes[i])
        worst = max(worst, err)
    log(f"config4 {dt}: all 2000 problems within the bars, worst rel_fro_err {worst:.3e}")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_large_problems_in_batch_contract(dt):
    """Problems of 1024^3 and 1536^3 in one batch (with small ones): each
    equals the oracle; each is bit-identical to the single-problem call with
    a one-k-group division (the 64x64 ring, 23); mg_gemm picks a two-k-group
    division there (26-29), whose result agrees with the batched one within
    the per-element rounding bound."""
    dtype = torch.float64 if dt == "f64" else torch.float32
    code = mg.F64 if dt == "f64" else mg.F32
    shapes = [(1024, 1024, 1024), (1536, 1536, 1536), (40, 70, 90), (300, 17, 512)]
    views, flats, probs = make_batch(86, shapes, dtype=dtype)
    C0 = [C.clone() for _, _, C in views]
    plan = mg.Plan(code, probs)
    plan.launch()
    torch.cuda.synchronize()
    u = U32 if dt == "f32" else 2.0 ** -53
    for (A, B, C), c0, (m, n, k) in zip(views, C0, shapes):
        check_problem(A, B, c0, C, 1.0, 1.0, f32=(dt == "f32"))
        one = c0.clone()
        mg.gemm(A, B, one, 1.0, 1.0, cfg=23)
        pick = mg.pick_tile_cfg(m, n, k, code)
        dflt = c0.clone()
        mg.gemm(A, B, dflt, 1.0, 1.0)
        torch.cuda.synchronize()
        assert torch.equal(one, C), (m, n, k)
        if m * n >= 1 << 20:
            assert pick in (26, 27, 28, 29), pick
            An, Bn, Cn = (x.double().cpu().numpy() for x in (A, B, c0))
            bound = elementwise_bound(1.0, An, Bn, 1.0, Cn, k, u=u)
            diff = np.abs(dflt.double().cpu().numpy() - C.double().cpu().numpy())
            assert (diff <= 2 * bound).all()
            log(f"{dt} {m}x{n}x{k}: mg_gemm picks {pick}; differing elements vs batched "
                f"{int((diff > 0).sum())} of {m * n}")
        else:
            assert torch.equal(dflt, C), (m, n, k)


def test_autotune_cache_roundtrip(tmp_path):
    """The tuned table persists as JSON keyed by device, CU count, dtype and
    library version: the first call times and writes, the second reads the
    same table without timing; entries of other keys survive a rewrite."""
    import json
    path = str(tmp_path / "tune.json")
    info = {}
    t1 = mg.autotune(mg.F64, reps=1, cache=path, info=info)
    assert info["from_cache"] is False
    doc = json.load(open(path))
    assert doc["format"] == "mg-autotune-1" and len(doc["tables"]) == 1
    e = doc["tables"][0]
    assert e["dtype"] == "f64" and e["classes"] == t1.to_list() and e["cus"] > 0
    t2 = mg.autotune(mg.F64, reps=1, cache=path, info=info)
    assert info["from_cache"] is True and t2.to_list() == t1.to_list()
    t3 = mg.autotune(mg.F32, reps=1, cache=path, info=info)
    assert info["from_cache"] is False
    doc = json.load(open(path))
    assert sorted(x["dtype"] for x in doc["tables"]) == ["f32", "f64"]
    assert mg.autotune(mg.F32, reps=1, cache=path, info=info).to_list() == t3.to_list()
    assert info["from_cache"] is True


def test_one_shot_repeat_replays_graph_and_reads_current_data():
    """mg_gemm_batched keeps the plan of each distinct problem set: a repeated
    set replays its graph (a hit), and the replay reads the operands' current
    contents; more than 8 other sets evict it (a miss again)."""
    shapes = [tuple(int(x) for x in s) for s in synth.batch_shapes(93, 50, 1, 300)]
    views, flats, probs = make_batch(93, shapes, beta=0.0)
    s0 = mg.gemm_batched_cache_stats()
    mg.gemm_batched(probs)
    torch.cuda.synchronize()
    first = [C.clone() for _, _, C in views]
    for (A, B, _), got in zip(views, first):
        check_problem(A, B, torch.zeros_like(got), got, 1.0, 0.0)
    flats["A"].mul_(2.0)  # new operand values behind the same descriptors
    mg.gemm_batched(probs)
    torch.cuda.synchronize()
    s1 = mg.gemm_batched_cache_stats()
    assert s1["hits"] == s0["hits"] + 1 and s1["misses"] == s0["misses"] + 1
    assert all(torch.equal(C, 2.0 * f) for (_, _, C), f in zip(views, first))
    others = []
    for i in range(9):
        v, f, p = make_batch(94 + i, [(40 + i, 30, 20)], beta=0.0)
        mg.gemm_batched(p)
        others.append((v, f))
    mg.gemm_batched(probs)
    torch.cuda.synchronize()
    s2 = mg.gemm_batched_cache_stats()
    assert s2["misses"] == s1["misses"] + 10 and s2["hits"] == s1["hits"]
    assert all(torch.equal(C, 2.0 * f) for (_, _, C), f in zip(views, first))
    for v, _ in others:
        A, B, C = v[0]
        check_problem(A, B, torch.zeros_like(C), C, 1.0, 0.0)
