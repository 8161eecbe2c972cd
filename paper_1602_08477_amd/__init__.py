"""Python binding of libmg, the MI355X (gfx950) GEMM library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libmg.so.  PyTorch supplies device memory and streams.  If the
shared library is missing this module raises on first use; there is no
fallback path.

The operation is the paper's DGEMM, C <- alpha*A*B + beta*C (Section 4.2),
on row-major matrices with a row pitch (``tensor.stride(0)``).
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MG_LIBRARY selects another build of the library (the LDS-poison debug
# build, libmg_poison.so, for race checks); default: the release build.
LIB_PATH = os.environ.get("MG_LIBRARY") or os.path.join(_HERE, "libmg.so")

# status codes (include/mg.h)
NAIVE_CFG = 25  # the one-output-per-lane work division (MG_NAIVE_CFG)
OK = 0
PENDING = 1
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED = -2
ERR_HIP = -3
ERR_NO_MEMORY = -4
ERR_BUSY = -5
ERR_NOT_FOUND = -6

F64 = 0
F32 = 1
NATIVE = 0
SPLIT_I8 = 1
SPLIT_BF16 = 2
BUILD_LDS_POISON = 1


class MgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libmg error {code}: {msg}")
        self.code = code


class SplitLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("mp", "np", "kp", "elem_bytes", "e_off", "f_off", "a_off", "b_off", "p_off",
                 "total_bytes")]


_lib = None
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_vp = ctypes.c_void_p
_int = ctypes.c_int


def lib() -> ctypes.CDLL:
    """The loaded libmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.mg_last_error.restype = ctypes.c_char_p
        L.mg_version.restype = _int
        L.mg_num_tile_cfgs.restype = _int
        L.mg_tile_cfg_info.argtypes = [_int, _int] + [ctypes.POINTER(_int)] * 4
        L.mg_pick_tile_cfg.argtypes = [_int, _i64, _i64, _i64]
        gemm_args = [_i64, _i64, _i64, _dbl, _vp, _i64, _vp, _i64, _dbl, _vp, _i64, _vp]
        L.mg_gemm.argtypes = [_int, _int] + gemm_args
        L.mg_gemm_cfg.argtypes = [_int, _int] + gemm_args
        L.mg_gemm_ex.argtypes = [_int, _int, _int, _int] + gemm_args
        L.mg_daxpy.argtypes = [_i64, _dbl, _vp, _i64, _vp, _i64, _vp]
        L.mg_split_default_slices.argtypes = [_int]
        L.mg_split_layout_query.argtypes = [_int, _int, _i64, _i64, _i64,
                                            ctypes.POINTER(SplitLayout)]
        L.mg_split_prepare.argtypes = [_int, _int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp,
                                       _i64, _vp]
        L.mg_gemm_split.argtypes = [_int, _int, _i64, _i64, _i64, _dbl, _vp, _i64, _vp, _i64,
                                    _dbl, _vp, _i64, _vp, _i64, _vp]
        L.mg_gemm_split_cfg.argtypes = [_int, _int, _int, _i64, _i64, _i64, _dbl, _vp, _i64, _vp,
                                        _i64, _dbl, _vp, _i64, _vp, _i64, _vp]
        _bind_batched(L)
        _bind_server(L)
        _lib = L
    return _lib


def last_error() -> str:
    return lib().mg_last_error().decode()


def check(rc: int) -> int:
    if rc < 0:
        raise MgError(rc, last_error())
    return rc


# ------------------------------------------------------------------ helpers
def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _mat(t, name):
    """(pointer, rows, cols, ld) of a row-major 2-D tensor with unit column stride."""
    if t is None:
        return None, 0, 0, 1
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride (row-major)")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)
    return ctypes.c_void_p(t.data_ptr()), t.shape[0], t.shape[1], max(ld, t.shape[1], 1)


def _mnk(A, B, C, k):
    pa, am, ak, lda = _mat(A, "A")
    pb, bk, bn, ldb = _mat(B, "B")
    pc, cm, cn, ldc = _mat(C, "C")
    m, n = cm, cn
    if A is not None:
        k = ak
        if am != m:
            raise ValueError("A rows != C rows")
    if B is not None:
        if bn != n or bk != k:
            raise ValueError("B shape mismatch")
    return (pa, lda), (pb, ldb), (pc, ldc), m, n, k


# --------------------------------------------------------------------- API
def gemm(A, B, C, alpha: float = 1.0, beta: float = 0.0, algo: int = NATIVE,
         cfg: int | None = None, stream=None, k: int | None = None):
    """C <- alpha*A@B + beta*C in place on the GPU (mg_gemm / mg_gemm_cfg).
    A may be None only with k == 0.  Returns C."""
    (pa, lda), (pb, ldb), (pc, ldc), m, n, kk = _mnk(A, B, C, k)
    dt = _dtype_code(C)
    s = _stream_handle(stream)
    if cfg is None:
        check(lib().mg_gemm(dt, algo, m, n, kk, alpha, pa, lda, pb, ldb, beta, pc, ldc, s))
    else:
        check(lib().mg_gemm_cfg(dt, cfg, m, n, kk, alpha, pa, lda, pb, ldb, beta, pc, ldc, s))
    return C


def gemm_ex(A, B, C, alpha: float = 1.0, beta: float = 0.0, transa: bool = False,
            transb: bool = False, cfg: int | None = None, stream=None):
    """C <- alpha*op(A)@op(B) + beta*C in place (mg_gemm_ex).  A and B are the
    stored matrices: A is k x m when transa (m x k otherwise), B is n x k when
    transb (k x n otherwise).  Returns C."""
    pa, ar, ac, lda = _mat(A, "A")
    pb, br, bc, ldb = _mat(B, "B")
    pc, m, n, ldc = _mat(C, "C")
    am, k = (ac, ar) if transa else (ar, ac)
    bk, bn = (bc, br) if transb else (br, bc)
    if am != m or bn != n or bk != k:
        raise ValueError("op(A), op(B), C shape mismatch")
    s = _stream_handle(stream)
    check(lib().mg_gemm_ex(_dtype_code(C), -1 if cfg is None else cfg, int(transa), int(transb),
                           m, n, k, alpha, pa, lda, pb, ldb, beta, pc, ldc, s))
    return C


def daxpy(alpha: float, x, y, stream=None):
    """y <- alpha*x + y in place (mg_daxpy).  x and y are 1-D float64 CUDA
    tensors of equal length; their strides (>= 1) are the increments.
    Returns y."""
    for t, name in ((x, "x"), (y, "y")):
        if t.dim() != 1:
            raise ValueError(f"{name} must be 1-D")
    if x.shape[0] != y.shape[0]:
        raise ValueError("x and y lengths differ")
    n = y.shape[0]
    incx = x.stride(0) if n > 1 else 1
    incy = y.stride(0) if n > 1 else 1
    check(lib().mg_daxpy(n, alpha, ctypes.c_void_p(x.data_ptr()), incx,
                         ctypes.c_void_p(y.data_ptr()), incy, _stream_handle(stream)))
    return y


def num_tile_cfgs() -> int:
    return lib().mg_num_tile_cfgs()


def tile_cfg_info(cfg: int, dtype: int = F64) -> dict:
    v = [_int() for _ in range(4)]
    check(lib().mg_tile_cfg_info(dtype, cfg, *[ctypes.byref(x) for x in v]))
    return dict(zip(("bm", "bn", "bk", "threads"), (x.value for x in v)))


def pick_tile_cfg(m: int, n: int, k: int, dtype: int = F64) -> int:
    return lib().mg_pick_tile_cfg(dtype, m, n, k)


def split_default_slices(algo: int) -> int:
    return check(lib().mg_split_default_slices(algo))


def split_layout(algo: int, slices: int, m: int, n: int, k: int) -> dict:
    L = SplitLayout()
    check(lib().mg_split_layout_query(algo, slices, m, n, k, ctypes.byref(L)))
    return {f: getattr(L, f) for f, _ in SplitLayout._fields_}


def split_workspace(algo: int, slices: int, m: int, n: int, k: int, device="cuda"):
    """A uint8 device tensor large enough for mg_gemm_split's workspace."""
    import torch
    return torch.empty(split_layout(algo, slices, m, n, k)["total_bytes"], dtype=torch.uint8,
                       device=device)


def split_prepare(algo: int, slices: int, A, B, workspace, stream=None):
    """Steps 1-2 of the split method into ``workspace`` (mg_split_prepare)."""
    pa, m, k, lda = _mat(A, "A")
    pb, kb, n, ldb = _mat(B, "B")
    if kb != k:
        raise ValueError("inner dimensions differ")
    check(lib().mg_split_prepare(algo, slices, m, n, k, pa, lda, pb, ldb,
                                 ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                 _stream_handle(stream)))
    return workspace


def split_num_cfgs() -> int:
    return lib().mg_split_num_cfgs()


def build_flags() -> int:
    """mg_build_flags: 1 (MG_BUILD_LDS_POISON) for the LDS-poison debug build."""
    return lib().mg_build_flags()


def release_cached_memory() -> None:
    """Trim the library's split-workspace pools (mg_release_cached_memory)."""
    check(lib().mg_release_cached_memory())


def gemm_split(A, B, C, alpha: float = 1.0, beta: float = 0.0, algo: int = SPLIT_I8,
               slices: int | None = None, workspace=None, stream=None, cfg: int = -1):
    """C <- alpha*A@B + beta*C through the split-precision path
    (mg_gemm_split_cfg; cfg -1 lets the library pick the work division)."""
    (pa, lda), (pb, ldb), (pc, ldc), m, n, k = _mnk(A, B, C, None)
    if slices is None:
        slices = split_default_slices(algo)
    if workspace is None:
        workspace = split_workspace(algo, slices, m, n, k, device=C.device)
    check(lib().mg_gemm_split_cfg(algo, slices, cfg, m, n, k, alpha, pa, lda, pb, ldb, beta, pc,
                                  ldc, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                  _stream_handle(stream)))
    return C


# ------------------------------------------------------------ batched GEMM
NUM_GROUPED_CLASSES = 3
TUNE_EDGES = 6
TUNE_BUCKETS = 216


class Problem(ctypes.Structure):
    _fields_ = [("m", _i64), ("n", _i64), ("k", _i64), ("alpha", _dbl), ("beta", _dbl),
                ("A", _vp), ("lda", _i64), ("B", _vp), ("ldb", _i64), ("C", _vp), ("ldc", _i64)]


class TuneTable(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("cls", ctypes.c_int32 * TUNE_BUCKETS)]

    def to_list(self):
        return [int(x) for x in self.cls]

    @classmethod
    def from_list(cls, dtype, values):
        t = cls()
        t.dtype = dtype
        for i, v in enumerate(values):
            t.cls[i] = int(v)
        return t


class PlanStats(ctypes.Structure):
    _fields_ = [("problems", _i64), ("tiles", _i64), ("workgroups", _i64), ("occupancy", _i64),
                ("tiles_per_class", _i64 * NUM_GROUPED_CLASSES), ("scale_tiles", _i64),
                ("flops", _dbl), ("bytes", _dbl), ("graph", _i64)]


def _bind_batched(L):
    L.mg_grouped_class_info.argtypes = [_int, ctypes.POINTER(_int), ctypes.POINTER(_int)]
    L.mg_tune_bucket.argtypes = [_i64, _i64, _i64]
    L.mg_tune_default.argtypes = [_int, ctypes.POINTER(TuneTable)]
    L.mg_autotune.argtypes = [_int, _int, _vp, ctypes.POINTER(TuneTable)]
    L.mg_autotune_cached.argtypes = [_int, _int, ctypes.c_char_p, _vp, ctypes.POINTER(TuneTable),
                                     ctypes.POINTER(_int)]
    L.mg_plan_create.argtypes = [_int, _i64, ctypes.POINTER(Problem), ctypes.POINTER(TuneTable),
                                 ctypes.POINTER(_vp)]
    L.mg_plan_launch.argtypes = [_vp, _vp]
    L.mg_plan_launch_direct.argtypes = [_vp, _vp]
    L.mg_plan_get_stats.argtypes = [_vp, ctypes.POINTER(PlanStats)]
    L.mg_plan_destroy.argtypes = [_vp]
    L.mg_gemm_batched.argtypes = [_int, _int, _i64, ctypes.POINTER(Problem), _vp]
    L.mg_gemm_batched_cache_stats.argtypes = [ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
    L.mg_gemm_batched_noalloc.argtypes = [_int, _i64, ctypes.POINTER(Problem), _vp]


def problem(A, B, C, alpha=1.0, beta=0.0) -> Problem:
    """Problem descriptor from row-major device tensors (kept alive by the caller)."""
    (pa, lda), (pb, ldb), (pc, ldc), m, n, k = _mnk(A, B, C, None)
    return Problem(m, n, k, alpha, beta, pa, lda, pb, ldb, pc, ldc)


def problems_array(probs):
    """A ctypes array of Problem descriptors, built once: the batched calls
    take it in place of a list and pass it through without copying (for a
    batch launched many times, this takes the per-call marshalling out)."""
    return (Problem * max(1, len(probs)))(*probs), len(probs)


def _problems(probs):
    if isinstance(probs, tuple) and len(probs) == 2 and isinstance(probs[0], ctypes.Array):
        return probs  # from problems_array
    return problems_array(probs)


def grouped_class_info(cls: int) -> tuple:
    a, b = _int(), _int()
    check(lib().mg_grouped_class_info(cls, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def tune_bucket(m: int, n: int, k: int) -> int:
    return lib().mg_tune_bucket(m, n, k)


def tune_default(dtype: int = F64) -> TuneTable:
    t = TuneTable()
    check(lib().mg_tune_default(dtype, ctypes.byref(t)))
    return t


def autotune(dtype: int = F64, reps: int = 3, stream=None, cache: str | None = None,
             info: dict | None = None) -> TuneTable:
    """mg_autotune, or mg_autotune_cached when ``cache`` names a JSON file;
    ``info["from_cache"]`` tells whether the table came from it."""
    t = TuneTable()
    if cache is None:
        check(lib().mg_autotune(dtype, reps, _stream_handle(stream), ctypes.byref(t)))
        return t
    hit = ctypes.c_int(0)
    check(lib().mg_autotune_cached(dtype, reps, os.fsencode(cache), _stream_handle(stream),
                                   ctypes.byref(t), ctypes.byref(hit)))
    if info is not None:
        info["from_cache"] = bool(hit.value)
    return t


class Plan:
    """A batch of problems prepared for one persistent (graph-replayed) launch."""

    def __init__(self, dtype, probs, table: TuneTable | None = None, keep=None):
        arr, n = _problems(probs)
        h = _vp()
        check(lib().mg_plan_create(dtype, n, arr, None if table is None else ctypes.byref(table),
                                   ctypes.byref(h)))
        self._h = h
        self._keep = keep  # tensors the plan points into

    def launch(self, stream=None, graph: bool = True):
        f = lib().mg_plan_launch if graph else lib().mg_plan_launch_direct
        check(f(self._h, _stream_handle(stream)))

    def stats(self) -> dict:
        s = PlanStats()
        check(lib().mg_plan_get_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in PlanStats._fields_}
        d["tiles_per_class"] = list(s.tiles_per_class)
        return d

    def close(self):
        if self._h:
            lib().mg_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_batched_noalloc(probs, dtype: int = F64, stream=None):
    """One-shot batched launch with no device allocation
    (mg_gemm_batched_noalloc: work list in the library's static buffer)."""
    arr, n = _problems(probs)
    check(lib().mg_gemm_batched_noalloc(dtype, n, arr, _stream_handle(stream)))


def gemm_batched(probs, dtype: int = F64, stream=None, algo: int = NATIVE):
    """One-shot batched launch (mg_gemm_batched).  NATIVE: a repeated problem
    set replays its kept graph; SPLIT_I8 / SPLIT_BF16 (FP64 only): batched
    split-precision launches, each result the single call's bits."""
    arr, n = _problems(probs)
    check(lib().mg_gemm_batched(dtype, algo, n, arr, _stream_handle(stream)))


def gemm_batched_cache_stats() -> dict:
    h, m = _i64(), _i64()
    check(lib().mg_gemm_batched_cache_stats(ctypes.byref(h), ctypes.byref(m)))
    return {"hits": h.value, "misses": m.value}


# ------------------------------------------------------------------ serving
class ServerOpts(ctypes.Structure):
    _fields_ = [("n_streams", _int), ("max_slots", _int), ("max_queue", _int),
                ("max_batch", _int), ("hbm_budget_bytes", _i64),
                ("table", ctypes.POINTER(TuneTable)), ("simulate", ctypes.c_int32),
                ("sim_tflops", _dbl), ("sim_launch_ns", _i64)]


class Request(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("algo", ctypes.c_int32), ("p", Problem),
                ("t_arrival_ns", _i64), ("ready_event", _vp)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32), ("batch_id", _i64),
                ("t_arrival_ns", _i64), ("t_submit_ns", _i64), ("t_admit_ns", _i64),
                ("t_launch_ns", _i64), ("t_done_ns", _i64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, _i64) for f in ("submitted", "completed", "rejected_busy", "rejected_memory",
                                    "failed", "batches", "max_batch_seen", "max_inflight_bytes",
                                    "max_slots_used")]


def _bind_server(L):
    L.mg_now_ns.restype = _i64
    L.mg_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]
    L.mg_server_destroy.argtypes = [_vp]
    L.mg_gemm_submit.argtypes = [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.mg_gemm_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.mg_gemm_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.mg_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    L.mg_server_replay.argtypes = [_vp, _i64, ctypes.POINTER(Request), ctypes.POINTER(Result)]


def now_ns() -> int:
    return lib().mg_now_ns()


def result_dict(r: Result) -> dict:
    return {f: getattr(r, f) for f, _ in Result._fields_}


class Server:
    """Continuous-batching GEMM server (mg_server_*)."""

    def __init__(self, n_streams=4, max_slots=256, max_queue=1 << 20, max_batch=64,
                 hbm_budget_bytes=64 << 30, table: TuneTable | None = None,
                 simulate: bool = False, sim_tflops: float = 50.0, sim_launch_ns: int = 20000):
        """``simulate=True``: host simulation, no GPU work (see mg_server_opts)."""
        self._table = table
        o = ServerOpts(n_streams, max_slots, max_queue, max_batch, hbm_budget_bytes,
                       None if table is None else ctypes.pointer(table), int(simulate),
                       sim_tflops, sim_launch_ns)
        h = _vp()
        check(lib().mg_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._simulate = bool(simulate)
        self._events = {}

    def submit(self, A, B, C, alpha=1.0, beta=0.0, algo=NATIVE, t_arrival_ns=0,
               stream=None) -> int:
        """Queues one request.  Its kernels wait for an event recorded here on
        ``stream`` (torch's current stream by default), so they run after
        every write to A, B and C already enqueued there."""
        import torch
        ev = None
        if not self._simulate:
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream() if stream is None else stream)
        r = Request(_dtype_code(C), algo, problem(A, B, C, alpha, beta), t_arrival_ns,
                    None if ev is None else ev.cuda_event)
        t = self.submit_request(r)
        if ev is not None:
            self._events[t] = ev  # alive until the request is reported done
        return t

    def submit_request(self, r: Request) -> int:
        t = ctypes.c_uint64()
        check(lib().mg_gemm_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """None while pending, else the result dict."""
        r = Result()
        rc = check(lib().mg_gemm_poll(self._h, ticket, ctypes.byref(r)))
        if rc == PENDING:
            return None
        self._events.pop(ticket, None)
        return result_dict(r)

    def wait(self, ticket: int) -> dict:
        r = Result()
        check(lib().mg_gemm_wait(self._h, ticket, ctypes.byref(r)))
        self._events.pop(ticket, None)
        return result_dict(r)

    def stats(self) -> dict:
        s = ServerStats()
        check(lib().mg_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def replay(self, reqs) -> "ctypes.Array":
        """Open-loop replay of a ctypes Request array (arrival offsets in ns).
        Every write already enqueued on the device is finished first, so
        requests without a ready_event see their operands complete."""
        n = len(reqs)
        if not self._simulate:
            import torch
            torch.cuda.synchronize()
        res = (Result * max(1, n))()
        check(lib().mg_server_replay(self._h, n, reqs, res))
        return res

    def close(self):
        if self._h:
            lib().mg_server_destroy(self._h)
            self._h = _vp()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
