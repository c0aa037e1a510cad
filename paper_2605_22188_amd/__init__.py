"""Python binding of libkbnb (include/kbnb.h): argument marshalling only.

Every computation happens in the HIP library; this module converts numpy
arrays to the C structures and back.  There is no fallback: if libkbnb.so is
missing or cannot be loaded, importing the functions raises.

Functions carry the C names: create_problem, destroy_problem, submit_nodes,
poll_bounds, branch_and_bound, last_error, prox_batch, certify_batch,
problem_info.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkbnb.so")

OK, TIMEOUT = 0, 1
SQUARED, LOGISTIC = 0, 1
DTYPE_F64, DTYPE_F32, DTYPE_BF16 = 0, 1, 2
MEM_HOST_COPY, MEM_DEVICE_COPY, MEM_DEVICE_BORROW = 0, 1, 2
CONVERGED, PRUNED, MAXITER, ERROR, UNPRUNABLE = 0, 1, 2, 3, 4
_DTYPES = {"f64": DTYPE_F64, "f32": DTYPE_F32, "bf16": DTYPE_BF16}
ITER_AUTO, ITER_F32, ITER_F64, ITER_ANCHORED = 0, 1, 2, 3
_ITERS = {0: ITER_AUTO, "auto": ITER_AUTO, "f32": ITER_F32, "f64": ITER_F64,
          "anchored": ITER_ANCHORED}


class KbnbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kbnb error {code}: {msg}")
        self.code = code


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32), ("k", ctypes.c_int32),
                ("loss", ctypes.c_int32), ("lambda2", ctypes.c_double), ("M", ctypes.c_double),
                ("x_dtype", ctypes.c_int32), ("mem_flags", ctypes.c_int32),
                ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("y", ctypes.c_void_p),
                ("hip_stream", ctypes.c_void_p), ("hbm_budget_bytes", ctypes.c_uint64),
                ("batch_width", ctypes.c_int32), ("cert_period", ctypes.c_int32),
                ("iter_dtype", ctypes.c_int32), ("admit_timeout_ms", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("split_rows", ctypes.c_int32),
                ("reopt_groups", ctypes.c_int32)]


class NodeDesc(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("n_in", ctypes.c_int32),
                ("fixed_in", ctypes.c_void_p), ("n_out", ctypes.c_int32),
                ("fixed_out", ctypes.c_void_p), ("warm_start", ctypes.c_void_p),
                ("upper_bound", ctypes.c_double), ("rel_tol", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("stop_unprunable", ctypes.c_int32),
                ("warm_nnz", ctypes.c_int32), ("warm_idx", ctypes.c_void_p),
                ("warm_val", ctypes.c_void_p)]


class BoundResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("lower_bound", ctypes.c_double),
                ("primal_value", ctypes.c_double), ("rel_gap", ctypes.c_double),
                ("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("branch_index", ctypes.c_int32), ("support_len", ctypes.c_int32),
                ("queue_seconds", ctypes.c_double), ("solve_seconds", ctypes.c_double)]


class BnbOptions(ctypes.Structure):
    _fields_ = [("time_limit_s", ctypes.c_double), ("rel_gap_tol", ctypes.c_double),
                ("node_rel_tol", ctypes.c_double), ("max_fista_iters", ctypes.c_int32),
                ("max_nodes", ctypes.c_int64), ("log_every_s", ctypes.c_double),
                ("rashomon", ctypes.c_int32), ("rashomon_n", ctypes.c_int32),
                ("rashomon_eps", ctypes.c_double), ("node_order", ctypes.c_int32),
                ("audit", ctypes.c_int32), ("support_path", ctypes.c_int32)]


class BnbResult(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_double), ("lower_bound", ctypes.c_double),
                ("rel_gap", ctypes.c_double), ("nodes", ctypes.c_int64),
                ("status", ctypes.c_int32), ("support_len", ctypes.c_int32),
                ("support", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("incumbent_updates", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("rashomon_size", ctypes.c_int64), ("audit_leaves", ctypes.c_int64)]


class TuneOptions(ctypes.Structure):
    _fields_ = [("widths", ctypes.c_void_p), ("n_widths", ctypes.c_int32),
                ("periods", ctypes.c_void_p), ("n_periods", ctypes.c_int32),
                ("sample_nodes", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("rel_tol", ctypes.c_double), ("time_limit_s", ctypes.c_double),
                ("tie_frac", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("tune_tiles", ctypes.c_int32), ("refresh", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("batch_width", ctypes.c_int32), ("cert_period", ctypes.c_int32),
                ("rate", ctypes.c_double), ("trials", ctypes.c_int32),
                ("sample_nodes", ctypes.c_int32), ("seconds", ctypes.c_double),
                ("tile_rows", ctypes.c_int32), ("split_rows", ctypes.c_int32),
                ("cached", ctypes.c_int32), ("tile_trials", ctypes.c_int32)]


EXPORTS = ["create_problem", "destroy_problem", "submit_nodes", "poll_bounds",
           "branch_and_bound", "rashomon_entry", "autotune", "last_error", "prox_batch",
           "certify_batch", "problem_info", "kernel_stats", "pool_create", "pool_destroy",
           "pool_add", "pool_info", "pool_export", "pool_record", "rashomon_pool",
           "rashomon_reliance", "pool_summary", "evaluate_supports", "cancel_nodes",
           "bnb_audit_leaf", "certify_batch_noalloc", "device_budget",
           "engine_streams"]

_lib = None


def load():
    """Load libkbnb.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_22188_amd.build`")
        # PyTorch ships its own HIP runtime library under the same soname;
        # loading torch first makes this process hold one runtime, whichever
        # of the two the caller touches first
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        lib.create_problem.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(vp)]
        lib.destroy_problem.argtypes = [vp]
        lib.submit_nodes.argtypes = [vp, ctypes.POINTER(NodeDesc), i32]
        lib.poll_bounds.argtypes = [vp, ctypes.POINTER(BoundResult), i32,
                                    ctypes.POINTER(i32), vp, vp, i32]
        lib.branch_and_bound.argtypes = [vp, ctypes.POINTER(BnbOptions), ctypes.POINTER(BnbResult)]
        lib.last_error.restype = ctypes.c_char_p
        lib.last_error.argtypes = []
        lib.prox_batch.argtypes = [vp, i32, vp, vp, dbl, vp]
        lib.certify_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        lib.problem_info.argtypes = [vp, vp, vp]
        lib.kernel_stats.argtypes = [vp, i32, vp]
        lib.pool_create.argtypes = [ctypes.POINTER(vp)]
        lib.pool_destroy.argtypes = [vp]
        lib.pool_add.argtypes = [vp, vp, i32, vp, dbl]
        lib.pool_info.argtypes = [vp, vp, vp, vp]
        lib.pool_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        lib.pool_record.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp]
        lib.rashomon_pool.argtypes = [vp, ctypes.POINTER(vp)]
        lib.rashomon_reliance.argtypes = [vp, vp, vp]
        lib.pool_summary.argtypes = [vp, i32, vp, vp]
        lib.evaluate_supports.argtypes = [vp, i32, vp, dbl, i32, vp, vp, vp, vp, vp]
        lib.cancel_nodes.argtypes = [vp]
        lib.bnb_audit_leaf.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp]
        lib.certify_batch_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        lib.device_budget.argtypes = [ctypes.c_int64, vp]
        lib.engine_streams.argtypes = [i32]
        for name in EXPORTS:
            if name != "last_error":
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def last_error() -> str:
    return load().last_error().decode()


def _check(rc):
    if rc < 0:
        raise KbnbError(rc, last_error())
    return rc


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Handle:
    """Owns a problem handle and the host arrays the library may still read."""

    def __init__(self, ptr, n, p, k, keep):
        self.ptr = ptr
        self.n, self.p, self.k = n, p, k
        self._keep = keep

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                destroy_problem(self)
            except Exception:
                pass


def _problem_desc(X, y, k, loss, lambda2, M, dtype, batch_width, cert_period, hbm_budget_bytes,
                  iter_dtype=0, admit_timeout_ms=0, tile_rows=0, split_rows=0, reopt_groups=0):
    """Marshal a problem description; returns (desc, arrays to keep alive, mem flag)."""
    xd = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    keep = []
    if hasattr(X, "is_cuda") and X.is_cuda:
        n, p = X.shape
        Xc = X.contiguous()
        keep.append(Xc)
        xptr, ldx, mem = ctypes.c_void_p(Xc.data_ptr()), p, MEM_DEVICE_COPY
        yc = y.contiguous().double()
        keep.append(yc)
        yptr = ctypes.c_void_p(yc.data_ptr())
        # the library waits for the work queued on the producing stream
        import torch
        stream = ctypes.c_void_p(torch.cuda.current_stream(X.device).cuda_stream)
    else:
        want = {DTYPE_F64: np.float64, DTYPE_F32: np.float32, DTYPE_BF16: np.uint16}[xd]
        Xa = np.ascontiguousarray(X, dtype=want)
        n, p = Xa.shape
        ya = np.ascontiguousarray(y, dtype=np.float64)
        keep += [Xa, ya]
        xptr, ldx, mem, yptr = _p(Xa), p, MEM_HOST_COPY, _p(ya)
        stream = None
    d = ProblemDesc(n=n, p=p, k=int(k), loss=int(loss), lambda2=float(lambda2), M=float(M),
                    x_dtype=xd, mem_flags=mem, X=xptr, ldx=ldx, y=yptr, hip_stream=stream,
                    hbm_budget_bytes=int(hbm_budget_bytes), batch_width=int(batch_width),
                    cert_period=int(cert_period),
                    iter_dtype=_ITERS[iter_dtype] if iter_dtype in _ITERS else int(iter_dtype),
                    admit_timeout_ms=int(admit_timeout_ms), tile_rows=int(tile_rows),
                    split_rows=int(split_rows), reopt_groups=int(reopt_groups))
    return d, keep, mem


def create_problem(X, y, k, loss, lambda2, M, dtype="f32", batch_width=0, cert_period=0,
                   hbm_budget_bytes=0, iter_dtype=0, admit_timeout_ms=0, tile_rows=0, split_rows=0,
                   reopt_groups=0):
    """X: host array holding the stored entries (float64 / float32 / uint16
    bfloat16 bits), or a torch CUDA tensor (copied on the device).
    iter_dtype: "auto" (0), "f32", "f64" or "anchored" (precision of the
    iteration).  admit_timeout_ms: wait for the process-wide device budget.
    reopt_groups: workgroups per support in the support re-optimisation (0:
    automatic, 1: one)."""
    lib = load()
    d, keep, mem = _problem_desc(X, y, k, loss, lambda2, M, dtype, batch_width, cert_period,
                                 hbm_budget_bytes, iter_dtype, admit_timeout_ms, tile_rows,
                                 split_rows, reopt_groups)
    out = ctypes.c_void_p()
    _check(lib.create_problem(ctypes.byref(d), ctypes.byref(out)))
    return Handle(out, d.n, d.p, int(k), keep if mem != MEM_HOST_COPY else [])


def autotune(X, y, k, loss, lambda2, M, dtype="f32", nodes=None, widths=None, periods=None,
             sample_nodes=0, max_iters=0, rel_tol=0.0, time_limit_s=0.0, tie_frac=0.0, seed=0,
             hbm_budget_bytes=0, iter_dtype=0, tune_tiles=False, refresh=False):
    """Measure every (batch width, certificate period) candidate on a node
    sample and return the choice plus the table of rates (node bounds/s)."""
    lib = load()
    d, keep, _ = _problem_desc(X, y, k, loss, lambda2, M, dtype, 0, 0, hbm_budget_bytes,
                               iter_dtype)
    w = np.ascontiguousarray(widths if widths is not None else [64, 128, 256, 512, 1024, 2048],
                             dtype=np.int32)
    pr = np.ascontiguousarray(periods if periods is not None else [4, 8, 16], dtype=np.int32)
    o = TuneOptions(widths=_p(w), n_widths=len(w), periods=_p(pr), n_periods=len(pr),
                    sample_nodes=int(sample_nodes), max_iters=int(max_iters),
                    rel_tol=float(rel_tol), time_limit_s=float(time_limit_s),
                    tie_frac=float(tie_frac), seed=int(seed), tune_tiles=1 if tune_tiles else 0,
                    refresh=1 if refresh else 0)
    arr, count = None, 0
    if nodes is not None:
        arr, nkeep = _node_array(nodes, math.inf, 0.0, 0, None, None)
        keep += nkeep
        count = len(nodes)
    r = TuneResult()
    rates = np.zeros((len(w), len(pr)))
    _check(lib.autotune(ctypes.byref(d), arr, count, ctypes.byref(o), ctypes.byref(r), _p(rates)))
    return dict(batch_width=r.batch_width, cert_period=r.cert_period, rate=r.rate,
                trials=r.trials, sample_nodes=r.sample_nodes, seconds=r.seconds,
                tile_rows=r.tile_rows, split_rows=r.split_rows, cached=bool(r.cached),
                tile_trials=r.tile_trials, widths=w.tolist(), periods=pr.tolist(), rates=rates)


def destroy_problem(h: Handle):
    if h.ptr:
        ptr, h.ptr = h.ptr, None
        _check(load().destroy_problem(ptr))


def _node_array(nodes, upper_bound, rel_tol, max_iters, tags, warm_starts, stop_unprunable=0):
    """Marshal node descriptors; returns (ctypes array, arrays to keep alive)."""
    count = len(nodes)
    arr = (NodeDesc * max(count, 1))()
    keep = []

    def pick(v, i):
        return v[i] if hasattr(v, "__len__") else v
    for i, nd in enumerate(nodes):
        fin, fout = (nd.fixed_in, nd.fixed_out) if hasattr(nd, "fixed_in") else nd
        fin = np.ascontiguousarray(fin, dtype=np.int32)
        fout = np.ascontiguousarray(fout, dtype=np.int32)
        keep += [fin, fout]
        # a warm start is a length-p array, or a sparse (indices, values) pair
        w = wi = wv = None
        if warm_starts is not None and warm_starts[i] is not None:
            ws = warm_starts[i]
            if isinstance(ws, tuple):
                wi = np.ascontiguousarray(ws[0], dtype=np.int32)
                wv = np.ascontiguousarray(ws[1], dtype=np.float64)
                keep += [wi, wv]
            else:
                w = np.ascontiguousarray(ws, dtype=np.float64)
                keep.append(w)
        arr[i] = NodeDesc(tag=int(tags[i]) if tags is not None else i, n_in=len(fin),
                          fixed_in=_p(fin) if len(fin) else None, n_out=len(fout),
                          fixed_out=_p(fout) if len(fout) else None,
                          warm_start=_p(w) if w is not None else None,
                          warm_nnz=len(wi) if wi is not None else 0,
                          warm_idx=_p(wi) if wi is not None and len(wi) else None,
                          warm_val=_p(wv) if wv is not None and len(wv) else None,
                          upper_bound=float(pick(upper_bound, i)),
                          rel_tol=float(pick(rel_tol, i)), max_iters=int(pick(max_iters, i)),
                          stop_unprunable=int(pick(stop_unprunable, i)))
    return arr, keep


class PreparedNodes:
    """Node descriptors marshalled once, for repeated or timed submission."""

    def __init__(self, nodes, upper_bound=math.inf, rel_tol=0.0, max_iters=0, tags=None,
                 warm_starts=None):
        self.count = len(nodes)
        self.arr, self._keep = _node_array(nodes, upper_bound, rel_tol, max_iters, tags,
                                           warm_starts)


def submit_prepared(h: Handle, prep: PreparedNodes):
    _check(load().submit_nodes(h.ptr, prep.arr, prep.count))


def poll_raw(h: Handle, out, cap, timeout_us=-1):
    """poll_bounds into a caller-owned (BoundResult * cap) array, no supports
    or iterates; returns (count, return code)."""
    n = ctypes.c_int32(0)
    rc = load().poll_bounds(h.ptr, out, int(cap), ctypes.byref(n), None, None, int(timeout_us))
    if rc < 0:
        _check(rc)
    return n.value, rc


def submit_nodes(h: Handle, nodes, upper_bound=math.inf, rel_tol=0.0, max_iters=0, tags=None,
                 warm_starts=None, stop_unprunable=0):
    """nodes: sequence of (fixed_in, fixed_out) index arrays (or objects with
    .fixed_in / .fixed_out).  Per-node upper_bound / rel_tol / max_iters /
    stop_unprunable may be scalars or sequences."""
    arr, keep = _node_array(nodes, upper_bound, rel_tol, max_iters, tags, warm_starts,
                            stop_unprunable)
    _check(load().submit_nodes(h.ptr, arr, len(nodes)))
    del keep


def poll_bounds(h: Handle, cap=1024, timeout_us=-1, supports=True, betas=True):
    """Returns a list of dicts (tag, lower_bound, primal_value, rel_gap, status,
    iterations, branch_index, support, beta)."""
    out = (BoundResult * cap)()
    n = ctypes.c_int32(0)
    sup = np.empty((cap, h.k), np.int32) if supports else None
    bet = np.empty((cap, h.p), np.float64) if betas else None
    rc = _check(load().poll_bounds(h.ptr, out, cap, ctypes.byref(n), _p(sup), _p(bet),
                                   int(timeout_us)))
    res = []
    for i in range(n.value):
        r = out[i]
        d = dict(tag=r.tag, lower_bound=r.lower_bound, primal_value=r.primal_value,
                 rel_gap=r.rel_gap, status=r.status, iterations=r.iterations,
                 branch_index=r.branch_index, support_len=r.support_len,
                 queue_seconds=r.queue_seconds, solve_seconds=r.solve_seconds)
        if supports:
            d["support"] = sup[i, :r.support_len].copy()
        if betas:
            d["beta"] = bet[i].copy()
        res.append(d)
    return res, rc


def device_budget(bytes_=-1):
    """Set (bytes_ >= 0; 0 = unlimited) or read (-1) the process-wide device
    budget of problem arenas on the current device; returns the bytes in use."""
    used = ctypes.c_int64(0)
    _check(load().device_budget(int(bytes_), ctypes.byref(used)))
    return used.value


def engine_streams(count):
    """Problems created afterwards share `count` streams (0: one each)."""
    _check(load().engine_streams(int(count)))


def cancel_nodes(h: Handle):
    """Drop every queued, running or unpolled node of h; returns when h is idle."""
    _check(load().cancel_nodes(h.ptr))


def bound_nodes(h: Handle, nodes, **kw):
    """Submit `nodes` and wait for all of them; results ordered like `nodes`."""
    submit_nodes(h, nodes, tags=list(range(len(nodes))), **kw)
    got = {}
    while len(got) < len(nodes):
        res, rc = poll_bounds(h, cap=max(1, len(nodes)), timeout_us=-1)
        for r in res:
            got[r["tag"]] = r
        if not res and rc == TIMEOUT:
            raise KbnbError(-4, "engine idle with nodes outstanding")
    return [got[i] for i in range(len(nodes))]


def branch_and_bound(h: Handle, time_limit_s=0.0, rel_gap_tol=0.0, node_rel_tol=0.0,
                     max_fista_iters=0, max_nodes=0, log_every_s=0.0, rashomon_eps=None,
                     rashomon_n=0, node_order=0, audit=False, support_path=0):
    """rashomon_eps (>= 0): also collect the support-level Rashomon set (the
    best rashomon_n when nonzero), returned as "rashomon": a list of
    (support tuple, value, beta) ordered by value.  node_order: 0 best bound,
    1 depth first.  audit: also return "leaves", the discarded subtrees with the
    certificates of their bounds (see bnb_audit_leaf).  support_path: 0
    automatic, 1 the re-optimisation kernel, 2 the node engine."""
    sup = np.full(h.k, -1, np.int32)
    beta = np.zeros(h.p)
    o = BnbOptions(time_limit_s=time_limit_s, rel_gap_tol=rel_gap_tol,
                   node_rel_tol=node_rel_tol, max_fista_iters=max_fista_iters,
                   max_nodes=max_nodes, log_every_s=log_every_s,
                   rashomon=0 if rashomon_eps is None else 1, rashomon_n=int(rashomon_n),
                   rashomon_eps=0.0 if rashomon_eps is None else float(rashomon_eps),
                   node_order=int(node_order), audit=1 if audit else 0,
                   support_path=int(support_path))
    r = BnbResult(support=_p(sup), beta=_p(beta))
    _check(load().branch_and_bound(h.ptr, ctypes.byref(o), ctypes.byref(r)))
    out = dict(objective=r.objective, lower_bound=r.lower_bound, rel_gap=r.rel_gap,
               nodes=r.nodes, status=r.status, support=sup[:r.support_len].copy(),
               beta=beta, incumbent_updates=r.incumbent_updates, seconds=r.seconds)
    if rashomon_eps is not None:
        out["rashomon"] = [rashomon_entry(h, i) for i in range(r.rashomon_size)]
    if audit:
        out["leaves"] = [bnb_audit_leaf(h, i) for i in range(r.audit_leaves)]
    return out


def bnb_audit_leaf(h: Handle, i):
    """Leaf i of the last audited search: dict(kind, bound, state, cert_state,
    cert_beta, cert_bound)."""
    kind = ctypes.c_int32(0)
    bound = ctypes.c_double(0.0)
    cb = ctypes.c_double(0.0)
    st = np.zeros(h.p, np.int8)
    cst = np.zeros(h.p, np.int8)
    beta = np.zeros(h.p)
    _check(load().bnb_audit_leaf(h.ptr, ctypes.c_int64(int(i)), ctypes.byref(kind),
                                 ctypes.byref(bound), _p(st), _p(cst), _p(beta), ctypes.byref(cb)))
    return dict(kind=kind.value, bound=bound.value, state=st, cert_state=cst, cert_beta=beta,
                cert_bound=cb.value)


def rashomon_entry(h: Handle, i):
    """Entry i of the last collected Rashomon set: (support tuple, value, beta)."""
    sup = np.full(h.k, -1, np.int32)
    beta = np.zeros(h.p)
    n = ctypes.c_int32(0)
    v = ctypes.c_double(0.0)
    _check(load().rashomon_entry(h.ptr, ctypes.c_int64(int(i)), _p(sup), ctypes.byref(n),
                                 _p(beta), ctypes.byref(v)))
    return tuple(int(j) for j in sup[:n.value]), v.value, beta


class Pool:
    """A compact support pool (trie + offsets + flat coefficients), owned here."""

    def __init__(self, ptr=None):
        if ptr is None:
            ptr = ctypes.c_void_p()
            _check(load().pool_create(ctypes.byref(ptr)))
        self.ptr = ptr

    @classmethod
    def from_problem(cls, h: Handle):
        """A copy of the set collected by the last Rashomon call on h."""
        ptr = ctypes.c_void_p()
        _check(load().rashomon_pool(h.ptr, ctypes.byref(ptr)))
        return cls(ptr)

    def close(self):
        if self.ptr is not None and self.ptr.value:
            load().pool_destroy(self.ptr)
        self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, seq, coef=None, value=0.0):
        sq = np.ascontiguousarray(seq, dtype=np.int32)
        c = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64)
        assert c is None or c.shape == sq.shape
        _check(load().pool_add(self.ptr, _p(sq) if sq.size else None, int(sq.size),
                               None if c is None else _p(c), float(value)))

    def info(self):
        """(records N, trie nodes T, stored coefficients o_N)."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().pool_info(self.ptr, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def __len__(self):
        return self.info()[0]

    def export(self):
        """The stored arrays: parent p(v), label a(v), end nodes, values, offsets o, coefficients c."""
        N, T, C = self.info()
        out = dict(parent=np.empty(T, np.int32), label=np.empty(T, np.int32),
                   end_node=np.empty(N, np.int32), values=np.empty(N),
                   offsets=np.empty(N + 1, np.int64), coef=np.empty(C))
        _check(load().pool_export(self.ptr, _p(out["parent"]), _p(out["label"]),
                                  _p(out["end_node"]), _p(out["values"]), _p(out["offsets"]),
                                  _p(out["coef"])))
        return out

    def record(self, m):
        """Record m: (path labels root first, coefficients in that order, value)."""
        n = ctypes.c_int32(0)
        _check(load().pool_record(self.ptr, int(m), None, ctypes.byref(n), None, None))
        seq = np.empty(max(n.value, 1), np.int32)
        coef = np.empty(max(n.value, 1))
        v = ctypes.c_double(0.0)
        _check(load().pool_record(self.ptr, int(m), _p(seq), ctypes.byref(n), _p(coef),
                                  ctypes.byref(v)))
        return tuple(int(j) for j in seq[:n.value]), coef[:n.value].copy(), v.value


def evaluate_supports(h: Handle, supports, rel_tol=0.0, max_iters=0):
    """Batched re-optimisation of supports (each a sequence of feature
    indices); returns dict of arrays: value, lower_bound, beta (count x p),
    status, iterations."""
    count = len(supports)
    sup = np.full((max(count, 1), h.k), -1, np.int32)
    for i, S in enumerate(supports):
        S = list(S)
        assert len(S) <= h.k
        sup[i, :len(S)] = S
    val = np.zeros(max(count, 1))
    low = np.zeros(max(count, 1))
    bet = np.zeros((max(count, 1), h.p))
    st = np.zeros(max(count, 1), np.int32)
    it = np.zeros(max(count, 1), np.int32)
    _check(load().evaluate_supports(h.ptr, count, _p(sup), float(rel_tol), int(max_iters), _p(val),
                                    _p(low), _p(bet), _p(st), _p(it)))
    return dict(value=val[:count], lower_bound=low[:count], beta=bet[:count], status=st[:count],
                iterations=it[:count])


SUMMARY_ROWS = ("freq", "mean", "abs_mean", "pos_frac", "coef_min", "coef_max",
                "reliance_min", "reliance_max", "reliance_mean")


def rashomon_reliance(h: Handle, pool: Pool):
    """Fixed-model reliance of every stored coefficient of `pool` on h's
    instance, laid out like the pool's coefficient vector."""
    C = pool.info()[2]
    out = np.zeros(max(C, 1))
    _check(load().rashomon_reliance(h.ptr, pool.ptr, _p(out)))
    return out[:C]


def pool_summary(pool: Pool, p, reliance=None):
    """Per-feature summaries over the pool's records (dict of length-p arrays)."""
    out = np.zeros((9, int(p)))
    rel = None if reliance is None else np.ascontiguousarray(reliance, dtype=np.float64)
    _check(load().pool_summary(pool.ptr, int(p), None if rel is None else _p(rel), _p(out)))
    return dict(zip(SUMMARY_ROWS, out))


def prox_batch(h: Handle, states, u, eta):
    st = np.ascontiguousarray(states, dtype=np.int8)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    m = st.shape[0]
    assert st.shape == (m, h.p) and uu.shape == (m, h.p)
    out = np.empty((m, h.p))
    _check(load().prox_batch(h.ptr, m, _p(st), _p(uu), float(eta), _p(out)))
    return out


def certify_batch(h: Handle, states, betas):
    st = np.ascontiguousarray(states, dtype=np.int8)
    bb = np.ascontiguousarray(betas, dtype=np.float64)
    m = st.shape[0]
    assert st.shape == (m, h.p) and bb.shape == (m, h.p)
    phi, psi = np.empty(m), np.empty(m)
    sup = np.empty((m, h.k), np.int32)
    br = np.empty(m, np.int32)
    _check(load().certify_batch(h.ptr, m, _p(st), _p(bb), _p(phi), _p(psi), _p(sup), _p(br)))
    return phi, psi, sup, br


def certify_batch_noalloc(h: Handle, states, betas, phi, psi, supports=None, branch=None,
                          stream=None):
    """certify_batch on torch device tensors without any allocation: states
    (m, p) int8, betas (m, p) float64; writes phi, psi (m,) float64 and, when
    given, supports (m, k) int32 and branch (m,) int32.  Enqueued on `stream`
    (a torch stream; None: the problem's own stream); the caller
    synchronises."""
    m = states.shape[0]
    assert tuple(states.shape) == (m, h.p) and tuple(betas.shape) == (m, h.p)
    for t in (states, betas, phi, psi, supports, branch):
        assert t is None or t.is_contiguous()

    def ptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(load().certify_batch_noalloc(h.ptr, int(m), ptr(states), ptr(betas), ptr(phi), ptr(psi),
                                        ptr(supports), ptr(branch), st))


def problem_info(h: Handle):
    i = np.zeros(11, np.int64)
    d = np.zeros(4)
    _check(load().problem_info(h.ptr, _p(i), _p(d)))
    return dict(n=int(i[0]), p=int(i[1]), k=int(i[2]), batch_width=int(i[3]),
                cert_period=int(i[4]), loss=int(i[5]), gsplit=int(i[6]), rounds=int(i[7]),
                iteration={1: "f32", 2: "f64", 3: "anchored"}.get(int(i[8]), "?"),
                tile_rows=int(i[9]), split_rows=int(i[10]),
                L=float(d[0]), lambda2=float(d[1]), M=float(d[2]), device_bytes=float(d[3]))


def create_from_instance(inst, **kw):
    """Convenience: create a problem from a workloads.Instance-like object
    (fields X_store, dtype, y, k, loss, lambda2, M)."""
    return create_problem(inst.X_store, inst.y, inst.k, inst.loss, inst.lambda2, inst.M,
                          dtype=inst.dtype, **kw)


KERNEL_NAMES = ["fwd_xy", "bwd_xtr", "prox", "cert_xb", "cert_xtz", "cert_finish", "admit",
                "reduce"]


def kernel_stats(h: Handle, mode=-1):
    """mode 1: reset and start timing kernels; 0: stop; -1: read only.
    Returns the counters as they were before the mode change."""
    out = np.zeros(18)
    _check(load().kernel_stats(h.ptr, int(mode), _p(out)))
    ms = dict(zip(KERNEL_NAMES, out[0:8]))
    cnt = dict(zip(KERNEL_NAMES, out[8:16].astype(np.int64)))
    return dict(total_ms=ms, launches=cnt, useful_cols=float(out[16]), running_cols=float(out[17]))
