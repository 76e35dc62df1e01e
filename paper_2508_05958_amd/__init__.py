"""Python binding of the HTLR library for MI355X (libhtlr.so).

Argument marshalling only: every step of construction, product and solve
runs in the library's HIP kernels.  PyTorch supplies device memory and
streams.  The names follow the C ABI in include/htlr.h.

Loading fails loudly when the library has not been built
(``python -m paper_2508_05958_amd.build`` or ``__graft_entry__.build()``);
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhtlr.so")

HTLR_OK = 0
STATUS = {0: "HTLR_OK", -1: "HTLR_ERR_INVALID", -2: "HTLR_ERR_UNSUPPORTED", -3: "HTLR_ERR_OOM",
          -4: "HTLR_ERR_HIP", -5: "HTLR_ERR_NOT_CONVERGED", -6: "HTLR_ERR_NUMERIC"}
KERNELS = {"inv_r": 0, "neg_log": 1, "exp": 2, "gauss": 3, "poly_test": 100}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
VEC_F64, VEC_F32 = 0, 1
ADM = {"strong": 0, "weak": 1}


class HTLRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _BuildOpts(ctypes.Structure):
    _fields_ = [("eta2", ctypes.c_double), ("admissibility", ctypes.c_int), ("gl_order", ctypes.c_int),
                ("a", ctypes.POINTER(ctypes.c_double)), ("precisions", ctypes.c_int),
                ("orthonormalize", ctypes.c_int), ("rank_tol", ctypes.c_double),
                ("edges", ctypes.POINTER(ctypes.c_double))]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("max_inner", ctypes.c_int), ("inner_prec", ctypes.c_int), ("inner_tol", ctypes.c_double)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int), ("matvecs_fp64", ctypes.c_int),
                ("matvecs_inner", ctypes.c_int), ("rel_residual", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int), ("p", ctypes.c_int), ("leaf_side", ctypes.c_int),
                ("levels", ctypes.c_int), ("uniform", ctypes.c_int), ("adm_pairs", ctypes.c_int64 * 16),
                ("unique_cores", ctypes.c_int64 * 16), ("near_pairs", ctypes.c_int64),
                ("device_bytes", ctypes.c_size_t), ("diag0", ctypes.c_double), ("uniform_m", ctypes.c_int),
                ("rank", ctypes.c_int), ("level_rank", ctypes.c_int * 16)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("ks_target", ctypes.c_int), ("near_kind", ctypes.c_int), ("near_waves", ctypes.c_int),
                ("candidates", ctypes.c_int), ("ms_default", ctypes.c_double), ("ms_best", ctypes.c_double)]


class _ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double)]


_lib = None
_c_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        L.htlr_last_error.restype = ctypes.c_char_p
        L.htlr_build.argtypes = [_c_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(_BuildOpts), ctypes.POINTER(_vp)]
        L.htlr_build_quasi.argtypes = [_c_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(_BuildOpts), ctypes.POINTER(_vp)]
        L.htlr_footprint.argtypes = [_c_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(_BuildOpts), ctypes.POINTER(ctypes.c_size_t)]
        L.htlr_workspace_bytes.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.htlr_matvec.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]
        L.htlr_matvec_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]
        L.htlr_solve.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(_SolveOpts),
                                 ctypes.POINTER(_SolveInfo), _vp]
        L.htlr_info.argtypes = [_vp, ctypes.POINTER(_Info)]
        L.htlr_exact_rows.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp]
        L.htlr_free.argtypes = [_vp]
        L.htlr_free.restype = None
        L.htlr_plan_counts.argtypes = [_c_dp, _c_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]
        L.htlr_plan_pairs.argtypes = [_c_dp, _c_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.htlr_autotune.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_TuneResult)]
        L.htlr_profile_enable.argtypes = [_vp, ctypes.c_int]
        L.htlr_profile_read.argtypes = [_vp, ctypes.POINTER(_ProfEntry), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        for name in ("htlr_build", "htlr_build_quasi", "htlr_footprint", "htlr_workspace_bytes", "htlr_matvec",
                     "htlr_solve", "htlr_exact_rows",
                     "htlr_info", "htlr_plan_counts", "htlr_plan_pairs", "htlr_profile_enable",
                     "htlr_profile_read", "htlr_autotune"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != HTLR_OK:
        raise HTLRError(status, lib().htlr_last_error().decode())


def _points_arg(points, d, n):
    if points is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(d * n))
    return arr, arr.ctypes.data_as(_c_dp)


ORTH = {"none": 0, "qr": 1, "qrcp": 2}


def _edges_arg(edges, d, n):
    if edges is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
    if arr.size != d * (n + 1):
        raise HTLRError(-1, f"edges must hold d*(n+1) = {d * (n + 1)} values")
    arr = arr.reshape(d * (n + 1))
    return arr, arr.ctypes.data_as(_c_dp)


def _opts(eta2, admissibility, gl_order, a, precisions, orthonormalize=0, rank_tol=0.0, edges=None):
    """Build options; returns (options, arrays the options point into)."""
    o = _BuildOpts()
    o.orthonormalize = ORTH[orthonormalize] if isinstance(orthonormalize, str) else int(orthonormalize)
    o.rank_tol = float(rank_tol)
    o.eta2 = float(eta2)
    o.admissibility = ADM[admissibility] if isinstance(admissibility, str) else int(admissibility)
    o.gl_order = int(gl_order)
    keep = None
    if a is not None:
        keep = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        o.a = keep.ctypes.data_as(_c_dp)
    if isinstance(precisions, (list, tuple)):
        precisions = sum(1 << PRECISIONS[p] for p in precisions)
    o.precisions = int(precisions)
    keep_e = None
    if edges is not None:
        keep_e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64).reshape(-1))
        o.edges = keep_e.ctypes.data_as(_c_dp)
    return o, (keep, keep_e)


def _stream_ptr(stream):
    if stream is None:
        return None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


@dataclass
class SolveInfo:
    outer_iters: int
    inner_iters: int
    matvecs_fp64: int
    matvecs_inner: int
    rel_residual: float


class HTLRMatrix:
    """An HTLR matrix resident on the current GPU (wraps htlr_matrix).

    With ``m`` given, the quasi-uniform transfer form of htlr_build_quasi:
    diag(a) + T Ahat S, Ahat on the uniform grid of m cells per dimension."""

    def __init__(self, points, kernel, d, n, p, leaf, eta2=1.0, admissibility="strong", gl_order=0,
                 a=None, precisions=0, m=None, orthonormalize=0, rank_tol=0.0, edges=None):
        self.d, self.n, self.p, self.leaf, self.m = d, n, p, leaf, m
        self.N = n ** d
        self.kernel = kernel
        if a is not None and np.asarray(a).size != self.N:
            raise HTLRError(-1, f"a must hold {self.N} values (one per grid point)")
        keep_pts, pts = _points_arg(points, d, n)
        if edges is not None:
            _edges_arg(edges, d, n)
        o, keep_a = _opts(eta2, admissibility, gl_order, a, precisions, orthonormalize, rank_tol, edges)
        h = _vp()
        kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        if m is None:
            _check(lib().htlr_build(pts, kid, d, n, p, leaf, ctypes.byref(o), ctypes.byref(h)))
        else:
            _check(lib().htlr_build_quasi(pts, kid, d, n, int(m), p, leaf, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        del keep_pts, keep_a

    def _check_vec(self, x, name, dt, nrhs=None):
        """x must be a CUDA tensor of dtype dt holding N x nrhs values in the
        library's layout: (N,) contiguous, or (N, nrhs) column-major."""
        if not hasattr(x, "is_cuda") or not x.is_cuda or x.dtype != dt:
            raise HTLRError(-1, f"{name} must be a {dt} CUDA tensor")
        if x.dim() == 1:
            ok = x.shape[0] == self.N and x.is_contiguous()
        elif x.dim() == 2:
            ok = x.shape[0] == self.N and x.stride(0) == 1 and (x.shape[1] == 1 or x.stride(1) == self.N)
        else:
            ok = False
        if not ok:
            raise HTLRError(-1, f"{name} must hold {self.N} rows, contiguous (one right-hand side) or column-major "
                                f"(each right-hand side contiguous)")
        cols = 1 if x.dim() == 1 else x.shape[1]
        if nrhs is not None and cols != nrhs:
            raise HTLRError(-1, f"{name} has {cols} right-hand sides, expected {nrhs}")
        return cols

    def matvec(self, u, f=None, prec="fp64", stream=None):
        """f = A u for device tensors u (N,) or (N, nrhs), column-major for nrhs > 1."""
        return self._product(lib().htlr_matvec, u, f, prec, stream)

    def matvec_noalloc(self, u, f, prec="fp64", stream=None):
        """f = A u into a caller-given f, with the work buffers in the library's
        fixed device scratch (htlr_matvec_noalloc): no device allocation."""
        if f is None:
            raise HTLRError(-1, "matvec_noalloc writes into a caller-given f")
        return self._product(lib().htlr_matvec_noalloc, u, f, prec, stream)

    def _product(self, fn, u, f, prec, stream):
        import torch
        pr = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        dt = torch.float64 if pr == 0 else torch.float32
        nrhs = self._check_vec(u, "u", dt)
        if f is None:
            f = torch.empty_like(u)
        else:
            self._check_vec(f, "f", dt, nrhs)
            if f.data_ptr() == u.data_ptr():
                raise HTLRError(-1, "f and u must not overlap")
        _check(fn(self._h, u.data_ptr(), f.data_ptr(), nrhs, pr, VEC_F64 if pr == 0 else VEC_F32,
                  _stream_ptr(stream)))
        return f

    def solve(self, f, u=None, tol=1e-10, restart=30, max_outer=20, max_inner=300, inner_prec="fp32",
              inner_tol=0.0, stream=None, check=True):
        import torch
        self._check_vec(f, "f", torch.float64, 1)
        if u is None:
            u = torch.zeros_like(f)
        else:
            self._check_vec(u, "u", torch.float64, 1)
            if u.data_ptr() == f.data_ptr():
                raise HTLRError(-1, "f and u must not overlap")
        o = _SolveOpts(tol, restart, max_outer, max_inner,
                       PRECISIONS[inner_prec] if isinstance(inner_prec, str) else int(inner_prec), inner_tol)
        info = _SolveInfo()
        st = lib().htlr_solve(self._h, f.data_ptr(), u.data_ptr(), 1, ctypes.byref(o), ctypes.byref(info),
                              _stream_ptr(stream))
        res = SolveInfo(info.outer_iters, info.inner_iters, info.matvecs_fp64, info.matvecs_inner,
                        info.rel_residual)
        if check:
            _check(st)
        return u, res, st

    def exact_rows(self, u, rows, stream=None):
        """Rows ``rows`` (int64 CUDA tensor) of the uncompressed Nystrom
        product A u (eq. 1.3-1.4), FP64; u is (N,) or (N, nrhs) column-major."""
        import torch
        nrhs = self._check_vec(u, "u", torch.float64)
        if not rows.is_cuda or rows.dtype != torch.int64 or rows.dim() != 1 or not rows.is_contiguous():
            raise HTLRError(-1, "rows must be a contiguous 1-D int64 CUDA tensor")
        out = torch.empty((nrhs, rows.numel()), dtype=torch.float64, device=u.device).t()
        _check(lib().htlr_exact_rows(self._h, u.data_ptr(), rows.data_ptr(), rows.numel(), out.data_ptr(), nrhs,
                                     _stream_ptr(stream)))
        return out if u.dim() == 2 else out[:, 0]

    def info(self) -> dict:
        i = _Info()
        _check(lib().htlr_info(self._h, ctypes.byref(i)))
        return {"d": i.d, "n": i.n, "p": i.p, "leaf_side": i.leaf_side, "levels": i.levels,
                "uniform": bool(i.uniform), "adm_pairs": list(i.adm_pairs[: i.levels + 1]),
                "unique_cores": list(i.unique_cores[: i.levels + 1]), "near_pairs": i.near_pairs,
                "device_bytes": i.device_bytes, "diag0": i.diag0, "uniform_m": i.uniform_m, "rank": i.rank,
                "level_rank": list(i.level_rank[: i.levels + 1])}

    def workspace_bytes(self, nrhs=1, prec="fp64") -> int:
        b = ctypes.c_size_t()
        _check(lib().htlr_workspace_bytes(self._h, nrhs, PRECISIONS[prec], ctypes.byref(b)))
        return b.value

    def autotune(self, nrhs=1, prec="fp64") -> dict:
        """Time kernel variants for products of this shape; keep the fastest."""
        r = _TuneResult()
        _check(lib().htlr_autotune(self._h, nrhs, PRECISIONS[prec] if isinstance(prec, str) else int(prec),
                                   ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in _TuneResult._fields_}

    def profile(self, enable: bool = True):
        """Start (or stop) per-launch hipEvent timing of products; clears the record."""
        _check(lib().htlr_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{step name: (launches, total ms)} since the last profile() call."""
        cnt = ctypes.c_int()
        _check(lib().htlr_profile_read(self._h, None, 0, ctypes.byref(cnt)))
        arr = (_ProfEntry * max(cnt.value, 1))()
        _check(lib().htlr_profile_read(self._h, arr, cnt.value, ctypes.byref(cnt)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(cnt.value)}

    def free(self):
        if getattr(self, "_h", None):
            lib().htlr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class _ServerOpts(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_size_t), ("max_active", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("restart", ctypes.c_int), ("inner_prec", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("autotune", ctypes.c_int), ("no_group_fusion", ctypes.c_int), ("inner_tol", ctypes.c_double)]


class _Request(ctypes.Structure):
    _fields_ = [("points", _c_dp), ("kernel", ctypes.c_int), ("d", ctypes.c_int), ("n", ctypes.c_int),
                ("p", ctypes.c_int), ("leaf", ctypes.c_int), ("eta2", ctypes.c_double),
                ("admissibility", ctypes.c_int), ("a", _c_dp), ("f", _c_dp), ("tol", ctypes.c_double),
                ("max_outer", ctypes.c_int)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("inner_iters", ctypes.c_int), ("rel_residual", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("fused_products", ctypes.c_int64), ("graph_launches", ctypes.c_int64),
                ("structures_built", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("resident_structures", ctypes.c_int), ("active", ctypes.c_int), ("queued", ctypes.c_int),
                ("resident_bytes", ctypes.c_size_t), ("group_products", ctypes.c_int64),
                ("grouped_launches", ctypes.c_int64)]


def _declare_server(L):
    if getattr(L, "_server_declared", False):
        return
    L.htlr_server_create.argtypes = [ctypes.POINTER(_ServerOpts), ctypes.POINTER(_vp)]
    L.htlr_server_submit.argtypes = [_vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_int64)]
    L.htlr_server_step.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.htlr_server_result.argtypes = [_vp, ctypes.c_int64, _c_dp, ctypes.POINTER(_RequestInfo)]
    L.htlr_server_stats.argtypes = [_vp, ctypes.POINTER(_ServerStats)]
    L.htlr_server_clock.argtypes = [_vp]
    L.htlr_server_clock.restype = ctypes.c_double
    L.htlr_server_destroy.argtypes = [_vp]
    L.htlr_server_destroy.restype = None
    for name in ("htlr_server_create", "htlr_server_submit", "htlr_server_step", "htlr_server_result",
                 "htlr_server_stats"):
        getattr(L, name).restype = ctypes.c_int
    L._server_declared = True


class Server:
    """Continuous-batching request server (wraps htlr_server)."""

    def __init__(self, memory_budget=0, max_active=64, max_batch=16, restart=30, inner_prec="fp32",
                 use_graphs=True, autotune=False, group_fusion=True, inner_tol=0.0):
        L = lib()
        _declare_server(L)
        o = _ServerOpts(int(memory_budget), max_active, max_batch, restart,
                        PRECISIONS[inner_prec] if isinstance(inner_prec, str) else int(inner_prec),
                        1 if use_graphs else 0, 1 if autotune else 0, 0 if group_fusion else 1, float(inner_tol))
        h = _vp()
        _check(L.htlr_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def submit(self, f, kernel, d, n, p, leaf, points=None, a=None, tol=1e-8, eta2=1.0, admissibility="strong",
               max_outer=0) -> int:
        N = n ** d
        fa = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(N))
        keep = [fa]
        r = _Request()
        r.f = fa.ctypes.data_as(_c_dp)
        if points is not None:
            pa = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(d * n))
            keep.append(pa)
            r.points = pa.ctypes.data_as(_c_dp)
        if a is not None:
            aa = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(N))
            keep.append(aa)
            r.a = aa.ctypes.data_as(_c_dp)
        r.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        r.d, r.n, r.p, r.leaf = d, n, p, leaf
        r.eta2 = float(eta2)
        r.admissibility = ADM[admissibility] if isinstance(admissibility, str) else int(admissibility)
        r.tol = float(tol)
        r.max_outer = int(max_outer)
        rid = ctypes.c_int64()
        _check(lib().htlr_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._sizes = getattr(self, "_sizes", {})
        self._sizes[rid.value] = N
        return rid.value

    def step(self):
        a, q = ctypes.c_int(), ctypes.c_int()
        _check(lib().htlr_server_step(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def result(self, rid):
        """(u, info) for a finished request, else (None, info)."""
        i = _RequestInfo()
        u = np.empty(self._sizes[rid])
        st = lib().htlr_server_result(self._h, rid, u.ctypes.data_as(_c_dp), ctypes.byref(i))
        info = {"state": i.state, "status": i.status, "outer_iters": i.outer_iters, "inner_iters": i.inner_iters,
                "rel_residual": i.rel_residual, "t_submit": i.t_submit, "t_admit": i.t_admit, "t_done": i.t_done}
        if st != HTLR_OK:
            return None, info
        return u, info

    def stats(self) -> dict:
        s = _ServerStats()
        _check(lib().htlr_server_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}

    def clock(self) -> float:
        return lib().htlr_server_clock(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().htlr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def htlr_build(points, kernel, d, n, p, leaf, **kw) -> HTLRMatrix:
    return HTLRMatrix(points, kernel, d, n, p, leaf, **kw)


def htlr_build_quasi(points, kernel, d, n, m, p, leaf, **kw) -> HTLRMatrix:
    return HTLRMatrix(points, kernel, d, n, p, leaf, m=m, **kw)


def htlr_footprint(points, kernel, d, n, p, leaf, eta2=1.0, admissibility="strong", gl_order=0,
                   precisions=0, orthonormalize=0, rank_tol=0.0, edges=None) -> int:
    keep_pts, pts = _points_arg(points, d, n)
    if edges is not None:
        _edges_arg(edges, d, n)
    o, keep = _opts(eta2, admissibility, gl_order, None, precisions, orthonormalize, rank_tol, edges)
    b = ctypes.c_size_t()
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    _check(lib().htlr_footprint(pts, kid, d, n, p, leaf, ctypes.byref(o), ctypes.byref(b)))
    return b.value


def htlr_plan_counts(points, d, n, leaf, eta2=1.0, admissibility="strong", edges=None):
    keep, pts = _points_arg(points, d, n)
    keep_e, e = _edges_arg(edges, d, n)
    L = ctypes.c_int()
    adm = (ctypes.c_int64 * 16)()
    near = ctypes.c_int64()
    _check(lib().htlr_plan_counts(pts, e, d, n, leaf, float(eta2), ADM[admissibility], ctypes.byref(L), adm,
                                  ctypes.byref(near)))
    return L.value, list(adm[: L.value + 1]), near.value


def htlr_plan_pairs(points, d, n, leaf, level, eta2=1.0, admissibility="strong", edges=None):
    keep, pts = _points_arg(points, d, n)
    keep_e, e = _edges_arg(edges, d, n)
    cnt = ctypes.c_int64()
    _check(lib().htlr_plan_pairs(pts, e, d, n, leaf, float(eta2), ADM[admissibility], level, None, None, 0,
                                 ctypes.byref(cnt)))
    tau = np.empty(cnt.value, dtype=np.int32)
    sig = np.empty(cnt.value, dtype=np.int32)
    _check(lib().htlr_plan_pairs(pts, e, d, n, leaf, float(eta2), ADM[admissibility], level,
                                 tau.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 sig.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cnt.value, ctypes.byref(cnt)))
    return tau, sig
