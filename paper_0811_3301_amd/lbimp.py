"""Thin ctypes binding of liblbimp.so (C-ABI in include/lbimp.h).

Functions carry the C names and only marshal arguments: torch tensors (float32, contiguous,
on the context's GPU) are passed as device pointers, outputs are allocated with torch when
not given, and every call is enqueued on torch's current stream.  All compute runs in the
HIP library; if the library is missing, loading fails with an error (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbimp.so")

LBIMP_OK, LBIMP_E_INVALID, LBIMP_E_NOMEM, LBIMP_E_DEVICE, LBIMP_E_UNSUPPORTED = 0, 1, 2, 3, 4
LBIMP_MODE_BRUTE, LBIMP_MODE_KEOGH, LBIMP_MODE_IMPROVED = 0, 1, 2
LBIMP_P_INF = 0x7FFFFFFF  # the exponent p = infinity
MODES = {"brute": LBIMP_MODE_BRUTE, "keogh": LBIMP_MODE_KEOGH, "improved": LBIMP_MODE_IMPROVED}
STAGES = ("envelope", "lb_keogh", "select_seeds", "seed_dtw", "compact", "lb_improved", "dtw", "finalize")

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


class LbimpStats(ctypes.Structure):
    _fields_ = [("candidates", _i64), ("seeded", _i64), ("pruned_keogh", _i64), ("pruned_improved", _i64),
                ("dtw_started", _i64), ("dtw_abandoned", _i64), ("pruned_pd", _i64)]


STATS_FIELDS = [f for f, _ in LbimpStats._fields_]

# name -> (restype, argtypes); the C-ABI surface, one entry per declaration in lbimp.h
SIGNATURES = {
    "lbimp_last_error": (ctypes.c_char_p, []),
    "lbimp_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "lbimp_ctx_set_stream": (ctypes.c_int, [_vp, _vp]),
    "lbimp_ctx_destroy": (None, [_vp]),
    "lbimp_ctx_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lbimp_ctx_set_option": (ctypes.c_int, [_vp, ctypes.c_char_p, _i64]),
    "lbimp_ctx_stage_times": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
    "lbimp_db_create": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.POINTER(_vp)]),
    "lbimp_db_destroy": (None, [_vp]),
    "lbimp_db_size": (_i64, [_vp]),
    "lbimp_db_length": (_i32, [_vp]),
    "lbimp_envelope": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _vp, _vp]),
    "lbimp_lb_keogh": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, _i32, _vp]),
    "lbimp_db_lb_keogh": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, _vp]),
    "lbimp_db_pd_bound": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, _vp]),
    "lbimp_lb_improved": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _i32, _i32, _vp]),
    "lbimp_dtw_band": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i32, _i32, _i32, _vp]),
    "lbimp_dtw_pairs": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _vp]),
    "lbimp_nn_search": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp,
                                       ctypes.POINTER(LbimpStats)]),
    "lbimp_nn_search_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp]),
    "lbimp_nn_search_ragged": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), _i32, _vp, ctypes.POINTER(_i64),
                                              ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i64, _i32,
                                              ctypes.POINTER(_i32), _i32, _vp, _vp, ctypes.POINTER(LbimpStats)]),
    "lbimp_nn_search_ragged_workspace": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), _i32, ctypes.POINTER(_i32),
                                                        ctypes.POINTER(_i32), _i64, _i32, ctypes.POINTER(_i32), _i32,
                                                        ctypes.POINTER(ctypes.c_uint64)]),
    "lbimp_ctx_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint64)]),
    "lbimp_autotune": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32, ctypes.POINTER(_i32)]),
    "lbimp_ctx_copy_tuning": (ctypes.c_int, [_vp, _vp]),
}
TUNE_KNOBS = ("seeds", "sweep_shape", "lbi_pipeline", "dtw_group", "seed_lane", "cascade", "pd", "lbi_abandon",
              "lbi_buckets", "dtw_split")

_lib = None


class LbimpError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.lbimp_last_error().decode() if _lib is not None else ""
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run `python -m paper_0811_3301_amd.build` first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != LBIMP_OK:
        raise LbimpError(rc, where)


def _dev(t: torch.Tensor, name: str, dtype=torch.float32) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _p(p) -> int:
    """The exponent as the C-ABI takes it: math.inf (or LBIMP_P_INF) selects p = infinity."""
    return LBIMP_P_INF if p == float("inf") else int(p)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Ctx:
    """Owning handle of an lbimp_ctx; calls follow torch's current stream."""

    def __init__(self, device: int = 0):
        lib = load()
        self.device = device
        h = _vp()
        with torch.cuda.device(device):
            _check(lib.lbimp_ctx_create(device, _stream(), ctypes.byref(h)), "lbimp_ctx_create")
        self.h = h

    def sync_stream(self):
        _check(_lib.lbimp_ctx_set_stream(self.h, _stream()), "lbimp_ctx_set_stream")
        return self.h

    def close(self):
        if getattr(self, "h", None):
            _lib.lbimp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Db:
    """Owning handle of a device-resident database (copied from a [N][n] float32 GPU tensor)."""

    def __init__(self, ctx: Ctx, rows: torch.Tensor):
        if rows.dim() != 2:
            raise ValueError("rows must be [N][n]")
        N, n = rows.shape
        h = _vp()
        _check(_lib.lbimp_db_create(ctx.sync_stream(), _dev(rows, "rows") if N else None, N, n, ctypes.byref(h)),
               "lbimp_db_create")
        self.h, self.N, self.n = h, N, n

    def close(self):
        if getattr(self, "h", None):
            _lib.lbimp_db_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbimp_ctx_create(device: int = 0) -> Ctx:
    return Ctx(device)


def lbimp_db_create(ctx: Ctx, rows: torch.Tensor) -> Db:
    return Db(ctx, rows)


def lbimp_ctx_set_timing(ctx: Ctx, enable: bool):
    _check(_lib.lbimp_ctx_set_timing(ctx.h, int(bool(enable))), "lbimp_ctx_set_timing")


def lbimp_ctx_set_option(ctx: Ctx, name: str, value: int):
    _check(_lib.lbimp_ctx_set_option(ctx.h, name.encode(), int(value)), "lbimp_ctx_set_option")


def lbimp_ctx_stage_times(ctx: Ctx) -> dict:
    buf = (ctypes.c_float * len(STAGES))()
    m = _lib.lbimp_ctx_stage_times(ctx.h, buf, len(STAGES))
    if m < 0:
        raise LbimpError(-m, "lbimp_ctx_stage_times")
    return {STAGES[i]: float(buf[i]) for i in range(m)}


def _out(out, shape, dtype, like):
    if out is None:
        return torch.empty(shape, dtype=dtype, device=like.device)
    return out


def lbimp_envelope(ctx: Ctx, y: torch.Tensor, w: int, U=None, L=None):
    y2 = y.reshape(-1, y.shape[-1])
    B, n = y2.shape
    U = _out(U, y.shape, torch.float32, y)
    L = _out(L, y.shape, torch.float32, y)
    _check(_lib.lbimp_envelope(ctx.sync_stream(), _dev(y2, "y"), B, n, w, _dev(U, "U"), _dev(L, "L")),
           "lbimp_envelope")
    return U, L


def lbimp_lb_keogh(ctx: Ctx, x: torch.Tensor, U: torch.Tensor, L: torch.Tensor, p: int, out=None):
    N, n = x.shape
    out = _out(out, (N,), torch.float32, x)
    _check(_lib.lbimp_lb_keogh(ctx.sync_stream(), _dev(x, "x"), N, n, _dev(U, "U"), _dev(L, "L"), _p(p),
                               _dev(out, "lb")), "lbimp_lb_keogh")
    return out


def lbimp_db_lb_keogh(ctx: Ctx, db: Db, U: torch.Tensor, L: torch.Tensor, p: int, out=None):
    U2 = U.reshape(-1, db.n)
    Q = U2.shape[0]
    out = _out(out, (Q, db.N), torch.float32, U)
    _check(_lib.lbimp_db_lb_keogh(ctx.sync_stream(), db.h, _dev(U2, "U"), _dev(L.reshape(-1, db.n), "L"), Q, _p(p),
                                  _dev(out, "lb")), "lbimp_db_lb_keogh")
    return out


def lbimp_db_pd_bound(ctx: Ctx, db: Db, U: torch.Tensor, L: torch.Tensor, p, out=None):
    """Piecewise-sum lower bound (Sec. 9) of every database row for Q envelopes: [Q][N]."""
    U2 = U.reshape(-1, db.n)
    Q = U2.shape[0]
    out = _out(out, (Q, db.N), torch.float32, U)
    _check(_lib.lbimp_db_pd_bound(ctx.sync_stream(), db.h, _dev(U2, "U"), _dev(L.reshape(-1, db.n), "L"), Q, _p(p),
                                  _dev(out, "lb")), "lbimp_db_pd_bound")
    return out


def lbimp_lb_improved(ctx: Ctx, x: torch.Tensor, y: torch.Tensor, U: torch.Tensor, L: torch.Tensor, w: int, p: int,
                      out=None):
    N, n = x.shape
    out = _out(out, (N,), torch.float32, x)
    _check(_lib.lbimp_lb_improved(ctx.sync_stream(), _dev(x, "x"), N, n, _dev(y, "y"), _dev(U, "U"), _dev(L, "L"),
                                  w, _p(p), _dev(out, "lb")), "lbimp_lb_improved")
    return out


def lbimp_dtw_band(ctx: Ctx, x: torch.Tensor, y: torch.Tensor, w: int, p: int, out=None):
    N, n = x.shape
    out = _out(out, (N,), torch.float32, x)
    _check(_lib.lbimp_dtw_band(ctx.sync_stream(), _dev(x, "x"), N, _dev(y, "y"), n, w, _p(p), _dev(out, "dist")),
           "lbimp_dtw_band")
    return out


def lbimp_dtw_pairs(ctx: Ctx, x: torch.Tensor, y: torch.Tensor, w: int, p, out=None):
    """DTW_p of row c of x against row c of y for every c (x, y: [N][n] float32 GPU tensors)."""
    N, n = x.shape
    if tuple(y.shape) != (N, n):
        raise ValueError("x and y must have the same [N][n] shape")
    out = _out(out, (N,), torch.float32, x)
    _check(_lib.lbimp_dtw_pairs(ctx.sync_stream(), _dev(x, "x") if N else None, _dev(y, "y") if N else None, N, n, w,
                                _p(p), _dev(out, "dist")), "lbimp_dtw_pairs")
    return out


def lbimp_nn_search(ctx: Ctx, db: Db, queries: torch.Tensor, w: int, p: int, k: int = 1, mode="improved",
                    idx=None, dist=None, stats: bool = True):
    """Returns (idx [Q][k] int64, dist [Q][k] float32, stats) with stats a structured numpy array or None."""
    if isinstance(mode, str):
        mode = MODES[mode]
    Q = queries.shape[0]
    idx = _out(idx, (Q, k), torch.int64, queries)
    dist = _out(dist, (Q, k), torch.float32, queries)
    st = (LbimpStats * max(Q, 1))() if stats else None
    _check(_lib.lbimp_nn_search(ctx.sync_stream(), db.h, _dev(queries, "queries") if Q else None, Q, w, _p(p), k, mode,
                                _dev(idx, "idx", torch.int64), _dev(dist, "dist"), st), "lbimp_nn_search")
    return idx, dist, (_stats_array(st, Q) if stats else None)


def lbimp_nn_search_noalloc(ctx: Ctx, db: Db, queries: torch.Tensor, w: int, p: int, k: int = 1, mode="improved",
                            idx=None, dist=None):
    """lbimp_nn_search on the library's fixed device scratch (no allocation inside the call).
    Returns (idx [Q][k] int64, dist [Q][k] float32)."""
    if isinstance(mode, str):
        mode = MODES[mode]
    Q = queries.shape[0]
    idx = _out(idx, (Q, k), torch.int64, queries)
    dist = _out(dist, (Q, k), torch.float32, queries)
    _check(_lib.lbimp_nn_search_noalloc(ctx.sync_stream(), db.h, _dev(queries, "queries") if Q else None, Q, w, _p(p),
                                        k, mode, _dev(idx, "idx", torch.int64), _dev(dist, "dist")),
           "lbimp_nn_search_noalloc")
    return idx, dist


def _stats_array(st, Q):
    return np.array([[getattr(s, f) for f in STATS_FIELDS] for s in st[:Q]], dtype=np.int64).reshape(
        Q, len(STATS_FIELDS))


def _per_query(v, Q, name):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.int32), (Q,)))
    if a.shape != (Q,):
        raise ValueError(f"{name} must be one value or one per query")
    return a


def lbimp_nn_search_ragged(ctx: Ctx, dbs, queries: torch.Tensor, offsets, db_of, w, p: int, k=1,
                           mode="improved", idx=None, dist=None, stats: bool = True):
    """Ragged batch: `queries` is a 1-D device tensor holding the queries end to end, query q at
    [offsets[q], offsets[q+1]); db_of[q] indexes `dbs`; w and k are one value or one per query.
    Returns (idx [Q][kmax], dist [Q][kmax], stats) with kmax the largest k; row q holds query
    q's k nearest neighbours, then -1 / +inf."""
    if isinstance(mode, str):
        mode = MODES[mode]
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    Q = off.shape[0] - 1
    if Q < 0:
        raise ValueError("offsets must hold Q + 1 entries")
    dof = np.ascontiguousarray(db_of, dtype=np.int32)
    wq = _per_query(w, Q, "w")
    kq = _per_query(k, Q, "k")
    if dof.shape != (Q,):
        raise ValueError("db_of must hold Q entries")
    kmax = int(kq.max()) if Q else 1
    idx = _out(idx, (Q, kmax), torch.int64, queries)
    dist = _out(dist, (Q, kmax), torch.float32, queries)
    handles = (_vp * max(len(dbs), 1))(*[d.h for d in dbs])
    st = (LbimpStats * max(Q, 1))() if stats else None
    _check(_lib.lbimp_nn_search_ragged(
        ctx.sync_stream(), handles, len(dbs), _dev(queries, "queries") if queries.numel() else None,
        off.ctypes.data_as(ctypes.POINTER(_i64)), dof.ctypes.data_as(ctypes.POINTER(_i32)),
        wq.ctypes.data_as(ctypes.POINTER(_i32)), Q, _p(p), kq.ctypes.data_as(ctypes.POINTER(_i32)), mode,
        _dev(idx, "idx", torch.int64), _dev(dist, "dist"), st), "lbimp_nn_search_ragged")
    return idx, dist, (_stats_array(st, Q) if stats else None)


def lbimp_nn_search_ragged_workspace(ctx: Ctx, dbs, db_of, w, p: int, k=1, mode="improved") -> int:
    """Device workspace (bytes) lbimp_nn_search_ragged needs for this batch on `ctx`."""
    if isinstance(mode, str):
        mode = MODES[mode]
    dof = np.ascontiguousarray(db_of, dtype=np.int32)
    Q = dof.shape[0]
    wq = _per_query(w, Q, "w")
    kq = _per_query(k, Q, "k")
    handles = (_vp * max(len(dbs), 1))(*[d.h for d in dbs])
    out = ctypes.c_uint64(0)
    _check(_lib.lbimp_nn_search_ragged_workspace(ctx.h, handles, len(dbs), dof.ctypes.data_as(ctypes.POINTER(_i32)),
                                                 wq.ctypes.data_as(ctypes.POINTER(_i32)), Q, _p(p),
                                                 kq.ctypes.data_as(ctypes.POINTER(_i32)), mode, ctypes.byref(out)),
           "lbimp_nn_search_ragged_workspace")
    return int(out.value)


def lbimp_ctx_workspace_bytes(ctx: Ctx) -> int:
    out = ctypes.c_uint64(0)
    _check(_lib.lbimp_ctx_workspace_bytes(ctx.h, ctypes.byref(out)), "lbimp_ctx_workspace_bytes")
    return int(out.value)


def lbimp_autotune(ctx: Ctx, db: Db, queries: torch.Tensor, w: int, p: int, k: int = 1, mode="improved") -> dict:
    """Tune the search of this batch shape; returns the chosen knobs by name."""
    if isinstance(mode, str):
        mode = MODES[mode]
    out = (_i32 * len(TUNE_KNOBS))()
    _check(_lib.lbimp_autotune(ctx.sync_stream(), db.h, _dev(queries, "queries"), queries.shape[0], w, _p(p), k, mode,
                               out), "lbimp_autotune")
    return {name: int(out[i]) for i, name in enumerate(TUNE_KNOBS)}


def lbimp_ctx_copy_tuning(dst: Ctx, src: Ctx):
    _check(_lib.lbimp_ctx_copy_tuning(dst.h, src.h), "lbimp_ctx_copy_tuning")
