"""ctypes binding of ``liblsamg.so`` (the C-ABI declared in ``include/lsamg.h``).

Argument marshalling only: every step of setup and solve runs in the native
library (host C++ setup, HIP kernels for the solve).  PyTorch is used for
device memory and the current HIP stream; importing this module fails loudly
if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsamg.so")

LSAMG_OK, LSAMG_EINVAL, LSAMG_EBADINPUT, LSAMG_ENOTSPD = 0, -1, -2, -3
LSAMG_ENOMEM, LSAMG_EHIP, LSAMG_ENOCONV, LSAMG_ENODEV = -4, -5, -6, -7
FP64, MIXED = 0, 1
OP_A, OP_RAS, OP_RAST, OP_VCYCLE = 0, 1, 2, 3
AGG_LATTICE, AGG_STANDARD = 0, 1
CYCLE_V, CYCLE_ADDITIVE = 0, 1
SETUP_HOST, SETUP_DEVICE, SETUP_AUTO = 0, 1, 2
OPT_BATCHED, OPT_MFMA, OPT_GRAPH, OPT_MFMA_TILE, OPT_ONEPASS_ATA, OPT_DENSE_SPLIT = 0, 1, 2, 3, 4, 5
OPT_ATA_TILES, OPT_BGROUP, OPT_KRYLOV = 6, 7, 8
KRYLOV_CG, KRYLOV_FCG, KRYLOV_BLOCK = 0, 1, 2

ERROR_NAMES = {0: "OK", -1: "EINVAL", -2: "EBADINPUT", -3: "ENOTSPD",
               -4: "ENOMEM", -5: "EHIP", -6: "ENOCONV", -7: "ENODEV"}


class LsamgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lsamg {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("max_levels", C.c_int32), ("max_coarse", C.c_int64),
                ("ndim", C.c_int32), ("grid", C.c_int32 * 3),
                ("block", C.c_int32), ("omega_max", C.c_int32),
                ("n_eig_fixed", C.c_int32), ("kappa", C.c_double),
                ("cmin", C.c_int32 * 8), ("ncmin", C.c_int32),
                ("tie_rtol", C.c_double), ("tie_atol", C.c_double),
                ("pinv_rtol", C.c_double), ("thresh_margin", C.c_double),
                ("stall_ratio", C.c_double), ("precision", C.c_int32),
                ("device", C.c_int32), ("nthreads", C.c_int32),
                ("verbose", C.c_int32), ("dense_tail", C.c_int64),
                ("aggregation", C.c_int32), ("agg_passes", C.c_int32 * 8),
                ("nagg_passes", C.c_int32), ("cycle", C.c_int32),
                ("setup_device", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32),
                ("rel_res", C.c_double), ("true_rel_res", C.c_double),
                ("rho", C.c_double), ("seconds", C.c_double),
                ("restarts", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LevelInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nagg", C.c_int64), ("g_rows", C.c_int64),
                ("g_nnz", C.c_int64), ("a_nnz", C.c_int64),
                ("smoother_entries", C.c_int64), ("p_entries", C.c_int64),
                ("block", C.c_int32), ("n_color", C.c_int32),
                ("n_mult", C.c_int32), ("kmin", C.c_int32), ("kmax", C.c_int32),
                ("thresh", C.c_double), ("hazards", C.c_int64)]


class Info(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("n0", C.c_int64), ("m0", C.c_int64),
                ("setup_seconds", C.c_double), ("device_bytes", C.c_size_t),
                ("op_complexity", C.c_double),
                ("smoother_complexity", C.c_double),
                ("level", LevelInfo * 16), ("tail_level", C.c_int32)]


class SetupView(C.Structure):
    _fields_ = [("n", C.c_int64), ("nagg", C.c_int64),
                ("agg", C.POINTER(C.c_int32)), ("optr", C.POINTER(C.c_int64)),
                ("oidx", C.POINTER(C.c_int64)), ("k", C.POINTER(C.c_int32)),
                ("M", C.POINTER(C.c_int32)), ("mu", C.POINTER(C.c_double)),
                ("muptr", C.POINTER(C.c_int64)), ("block", C.c_int32),
                ("n_color", C.c_int32), ("n_mult", C.c_int32),
                ("thresh", C.c_double)]


class KProf(C.Structure):
    _fields_ = [("name", C.c_char * 80), ("launches", C.c_int64),
                ("ms", C.c_double), ("bytes", C.c_double), ("flops", C.c_double)]


class Request(C.Structure):
    _fields_ = [("id", C.c_uint64), ("op_key", C.c_uint64),
                ("G", C.POINTER(Csr)), ("params", C.POINTER(Params)),
                ("b", C.c_void_p), ("x", C.c_void_p), ("nrhs", C.c_int32),
                ("maxit", C.c_int32), ("tol", C.c_double)]


class Done(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("cache_hit", C.c_int32),
                ("batch_rhs", C.c_int32), ("iters_max", C.c_int32),
                ("true_rel_res_max", C.c_double), ("t_queue", C.c_double),
                ("t_setup", C.c_double), ("t_solve", C.c_double),
                ("t_total", C.c_double), ("joined_at", C.c_int32),
                ("reserved", C.c_int32), ("msg", C.c_char * 96)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64),
                ("hits", C.c_int64), ("misses", C.c_int64),
                ("evictions", C.c_int64), ("resident_bytes", C.c_size_t),
                ("peak_bytes", C.c_size_t), ("budget", C.c_size_t),
                ("queued", C.c_int32), ("active", C.c_int32),
                ("joins", C.c_int64), ("reserve_misses", C.c_int64),
                ("iterations", C.c_int64)]


# every symbol the header declares, with its ctypes signature
_SIGS = {
    "lsamg_params_default": (None, [C.POINTER(Params)]),
    "lsamg_setup": (C.c_int, [C.POINTER(Csr), C.POINTER(Params),
                              C.POINTER(C.c_void_p)]),
    "lsamg_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                              C.c_int64, C.c_double, C.c_int32, C.c_void_p,
                              C.POINTER(Stats)]),
    "lsamg_apply_op": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "lsamg_apply_op_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    "lsamg_set_precision": (C.c_int, [C.c_void_p, C.c_int32]),
    "lsamg_set_option": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64]),
    "lsamg_apply_vcycle_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_int32, C.c_int64, C.c_void_p]),
    "lsamg_profile": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p]),
    "lsamg_profile_read": (C.c_int, [C.c_void_p, C.POINTER(KProf), C.c_int32,
                                     C.POINTER(C.c_int32)]),
    "lsamg_info_get": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "lsamg_export_setup": (C.c_int, [C.c_void_p, C.c_int32,
                                     C.POINTER(SetupView)]),
    "lsamg_device_bytes": (C.c_size_t, [C.c_void_p]),
    "lsamg_destroy": (None, [C.c_void_p]),
    "lsamg_last_error": (C.c_char_p, []),
    "lsamg_server_create": (C.c_int, [C.c_int32, C.c_size_t, C.c_int32,
                                      C.POINTER(C.c_void_p)]),
    "lsamg_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request)]),
    "lsamg_server_poll": (C.c_int, [C.c_void_p, C.POINTER(Done), C.c_int32,
                                    C.POINTER(C.c_int32), C.c_int32]),
    "lsamg_server_stats_get": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "lsamg_server_destroy": (None, [C.c_void_p]),
}

_lib = None


def load() -> C.CDLL:
    """Load the built library (raises if it is missing: there is no fallback).

    torch is imported first: its ROCm build carries its own HIP and HSA
    runtimes, which then also serve the library (whose libamdhip64.so.7 the
    loader finds already present).  Loaded the other way round, the process
    would hold two HIP/HSA runtimes, the library's could not open the GPU, and
    device pointers from torch would be foreign to it."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run "
                          "python -m paper_2601_04112_amd.build")
    import torch  # noqa: F401  (HIP runtime first, see above)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, allow=()):
    if rc != LSAMG_OK and rc not in allow:
        msg = load().lsamg_last_error()
        raise LsamgError(rc, msg.decode() if msg else "")
    return rc


def default_params() -> Params:
    p = Params()
    load().lsamg_params_default(C.byref(p))
    return p


def make_params(ndim: int, grid: Sequence[int], *, block: int = 4,
                max_levels: int = 10, max_coarse: int = 2000,
                omega_max: int = 800, n_eig_fixed: int = 0,
                kappa: float = 50.0, cmin: Sequence[int] = (2,),
                tie_rtol: float = 1e-8, tie_atol: float = 1e-12,
                pinv_rtol: float = 1e-6, thresh_margin: float = 1e-10,
                stall_ratio: float = 0.9, precision: int = FP64,
                device: int = 0, nthreads: int = 0, verbose: bool = False,
                dense_tail: int = 16384, aggregation: str = "lattice",
                agg_passes: Sequence[int] = (1,), cycle: str = "v",
                setup_device="auto") -> Params:
    p = default_params()
    p.ndim = ndim
    for d in range(3):
        p.grid[d] = int(grid[d]) if d < len(grid) else 1
    p.block, p.max_levels, p.max_coarse = block, max_levels, max_coarse
    p.omega_max, p.n_eig_fixed, p.kappa = omega_max, n_eig_fixed, kappa
    cm = list(cmin)[:8]
    for i, c in enumerate(cm):
        p.cmin[i] = int(c)
    p.ncmin = len(cm)
    p.tie_rtol, p.tie_atol, p.pinv_rtol = tie_rtol, tie_atol, pinv_rtol
    p.thresh_margin, p.stall_ratio = thresh_margin, stall_ratio
    p.precision, p.device, p.nthreads = precision, device, nthreads
    p.verbose = 1 if verbose else 0
    p.dense_tail = int(dense_tail)
    if aggregation not in ("lattice", "standard"):
        raise ValueError("aggregation must be 'lattice' or 'standard'")
    p.aggregation = AGG_STANDARD if aggregation == "standard" else AGG_LATTICE
    ap = list(agg_passes)[:8]
    for i, c in enumerate(ap):
        p.agg_passes[i] = int(c)
    p.nagg_passes = len(ap)
    if cycle not in ("v", "additive"):
        raise ValueError("cycle must be 'v' or 'additive'")
    p.cycle = CYCLE_ADDITIVE if cycle == "additive" else CYCLE_V
    # True / "device": the setup's dense local problems on the GPU; False /
    # "host": on the host; "auto": on the GPU from 100,000 unknowns on
    if setup_device in ("auto", None):
        p.setup_device = SETUP_AUTO
    elif setup_device in (True, "device", 1):
        p.setup_device = SETUP_DEVICE
    elif setup_device in (False, "host", 0):
        p.setup_device = SETUP_HOST
    else:
        raise ValueError("setup_device must be 'auto', 'device' or 'host'")
    return p


class Solver:
    """Handle over one hierarchy: ``setup(G, params)`` then ``solve(b, tol)``."""

    def __init__(self, G, ndim: int, grid: Sequence[int], **params):
        lib = load()
        G = G.tocsr()
        self._rowptr = np.ascontiguousarray(G.indptr, dtype=np.int64)
        self._col = np.ascontiguousarray(G.indices, dtype=np.int32)
        self._val = np.ascontiguousarray(G.data, dtype=np.float64)
        csr = Csr(G.shape[0], G.shape[1], int(self._val.size),
                  self._rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                  self._col.ctypes.data_as(C.POINTER(C.c_int32)),
                  self._val.ctypes.data_as(C.POINTER(C.c_double)))
        self.params = make_params(ndim, grid, **params)
        h = C.c_void_p()
        _check(lib.lsamg_setup(C.byref(csr), C.byref(self.params), C.byref(h)))
        self._h = h
        self.n = G.shape[1]
        self.device = self.params.device
        del self._rowptr, self._col, self._val

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            load().lsamg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ----------------------------------------------------------
    @staticmethod
    def _stream(stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        return C.c_void_p(stream.cuda_stream)

    def _dev_vec(self, t):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda
                and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("expected a contiguous float64 CUDA/HIP tensor")
        return t

    # -- solve ------------------------------------------------------------
    def solve(self, b, tol: float = 1e-8, maxit: int = 1000, out=None,
              stream=None, raise_on_noconv: bool = False):
        """Solve A x = b.  ``b``: device float64 tensor of shape (n,) or
        (nrhs, n) (each row one right-hand side).  Returns (x, stats)."""
        import torch
        b = self._dev_vec(b)
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        if b.shape[-1] != self.n:
            raise ValueError("length mismatch")
        x = torch.empty_like(b) if out is None else self._dev_vec(out)
        st = (Stats * nrhs)()
        rc = load().lsamg_solve(self._h, C.c_void_p(b.data_ptr()),
                                C.c_void_p(x.data_ptr()), nrhs, self.n, tol,
                                maxit, self._stream(stream), st)
        _check(rc, allow=() if raise_on_noconv else (LSAMG_ENOCONV,))
        return x, [s.as_dict() for s in st]

    def apply(self, op: int, x, out=None, stream=None):
        """y = op(x) on the finest level (OP_A, OP_RAS, OP_RAST, OP_VCYCLE)."""
        import torch
        x = self._dev_vec(x)
        y = torch.empty_like(x) if out is None else self._dev_vec(out)
        _check(load().lsamg_apply_op(self._h, op, C.c_void_p(x.data_ptr()),
                                     C.c_void_p(y.data_ptr()),
                                     self._stream(stream)))
        return y

    def apply_noalloc(self, op: int, x, out, stream=None):
        """The allocation-free form of ``apply``: ``out`` must be given; the
        call only enqueues its kernels on the stream (no synchronisation) and
        allocates nothing (its staging is the library's per-GPU array)."""
        x = self._dev_vec(x)
        y = self._dev_vec(out)
        _check(load().lsamg_apply_op_noalloc(self._h, op, C.c_void_p(x.data_ptr()),
                                             C.c_void_p(y.data_ptr()),
                                             self._stream(stream)))
        return y

    def apply_vcycle_batch(self, X, out=None, stream=None):
        """Y = B X for the rows of X (shape (nrhs, n), nrhs <= 64) through
        the multi-right-hand-side V-cycle."""
        import torch
        X = self._dev_vec(X)
        if X.dim() != 2 or X.shape[1] != self.n:
            raise ValueError("expected shape (nrhs, n)")
        Y = torch.empty_like(X) if out is None else self._dev_vec(out)
        _check(load().lsamg_apply_vcycle_batch(
            self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
            X.shape[0], self.n, self._stream(stream)))
        return Y

    def set_precision(self, precision: int):
        _check(load().lsamg_set_precision(self._h, precision))

    def set_option(self, opt: int, value: int):
        """OPT_BATCHED, OPT_MFMA, OPT_GRAPH, OPT_ONEPASS_ATA (value 0 or 1), OPT_ATA_TILES
        (0 off, 1 per precision, 2 row form, 3 expanded form), OPT_MFMA_TILE
        (0: autotune, else 100*rt + 10*u + split) or OPT_DENSE_SPLIT (0: autotune,
        1..16: LDS-staged dense GEMM with that many loop ranges, 17: never) or OPT_BGROUP
        (0: autotune, 1: row-group pass, 2: CSR passes) or OPT_KRYLOV (KRYLOV_CG,
        KRYLOV_FCG: flexible CG, or KRYLOV_BLOCK: block CG on batches of columns)."""
        _check(load().lsamg_set_option(self._h, opt, int(value)))

    # -- kernel timing ----------------------------------------------------
    def profile(self, on: bool = True, only: Optional[str] = None,
                by_level: bool = False):
        """Bracket kernel launches with HIP events (all, or one symbol);
        by_level reports the V-cycle kernels per hierarchy level."""
        mode = (2 if by_level else 1) if on else 0
        _check(load().lsamg_profile(self._h, mode, only.encode() if only else None))

    def profile_read(self) -> list:
        """Per-kernel totals since profiling was enabled (then reset)."""
        buf = (KProf * 256)()
        cnt = C.c_int32()
        _check(load().lsamg_profile_read(self._h, buf, 256, C.byref(cnt)))
        return [dict(name=buf[i].name.decode(), launches=buf[i].launches,
                     ms=buf[i].ms, bytes=buf[i].bytes, flops=buf[i].flops)
                for i in range(cnt.value)]

    # -- introspection ----------------------------------------------------
    def info(self) -> dict:
        inf = Info()
        _check(load().lsamg_info_get(self._h, C.byref(inf)))
        levels = []
        for l in range(inf.nlevels):
            L = inf.level[l]
            levels.append({k: getattr(L, k) for k, _ in LevelInfo._fields_})
        return dict(nlevels=inf.nlevels, n0=inf.n0, m0=inf.m0,
                    setup_seconds=inf.setup_seconds,
                    device_bytes=inf.device_bytes,
                    op_complexity=inf.op_complexity,
                    smoother_complexity=inf.smoother_complexity,
                    levels=levels, tail_level=inf.tail_level)

    def export_setup(self, level: int) -> dict:
        v = SetupView()
        _check(load().lsamg_export_setup(self._h, level, C.byref(v)))
        out = dict(n=v.n, nagg=v.nagg, block=v.block, n_color=v.n_color,
                   n_mult=v.n_mult, thresh=v.thresh)
        if v.nagg == 0:
            return out

        def arr(ptr, count, dt):
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt).copy()
        out["agg"] = arr(v.agg, v.n, np.int64)
        out["optr"] = arr(v.optr, v.nagg + 1, np.int64)
        out["oidx"] = arr(v.oidx, int(out["optr"][-1]), np.int64)
        out["k"] = arr(v.k, v.nagg, np.int64)
        out["muptr"] = arr(v.muptr, v.nagg + 1, np.int64)
        out["mu"] = arr(v.mu, int(out["muptr"][-1]), np.float64)
        if bool(v.M):
            out["M"] = arr(v.M, self._m0(), np.int64)
        return out

    def _m0(self) -> int:
        inf = Info()
        _check(load().lsamg_info_get(self._h, C.byref(inf)))
        return inf.m0


def symbols() -> list:
    """Names of every C-ABI entry point (all must be exported)."""
    return list(_SIGS)


class _HostCsr:
    """A CSR of G kept alive (with its ctypes view) while requests use it."""

    def __init__(self, G):
        G = G.tocsr()
        self.rowptr = np.ascontiguousarray(G.indptr, dtype=np.int64)
        self.col = np.ascontiguousarray(G.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(G.data, dtype=np.float64)
        self.csr = Csr(G.shape[0], G.shape[1], int(self.val.size),
                       self.rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                       self.col.ctypes.data_as(C.POINTER(C.c_int32)),
                       self.val.ctypes.data_as(C.POINTER(C.c_double)))
        self.n = G.shape[1]


class Server:
    """Continuous-batching request server (lsamg_server_*).

    ``submit(op_key, G, ndim, grid, b, ...)`` queues a solve with host right-
    hand sides ``b`` (shape (n,) or (nrhs, n)); ``poll()`` returns finished
    requests as dicts carrying the solution ``x`` (host numpy array)."""

    def __init__(self, hbm_budget: int, max_slots: int = 4, device: int = 0):
        h = C.c_void_p()
        _check(load().lsamg_server_create(device, hbm_budget, max_slots, C.byref(h)))
        self._h = h
        self._ops = {}          # op_key -> (_HostCsr, Params)
        self._live = {}         # id -> (b, x, request)
        self._next = 0

    def submit(self, op_key: int, G, ndim: int, grid, b, tol: float = 1e-8,
               maxit: int = 1000, precision: int = MIXED, req_id: Optional[int] = None,
               **params):
        if op_key not in self._ops:
            self._ops[op_key] = (_HostCsr(G), make_params(ndim, grid, precision=precision,
                                                          device=0, **params))
        hc, prm = self._ops[op_key]
        bb = np.ascontiguousarray(np.atleast_2d(b), dtype=np.float64)
        if bb.shape[1] != hc.n:
            raise ValueError("length mismatch")
        x = np.empty_like(bb)
        rid = self._next if req_id is None else req_id
        self._next = max(self._next, rid) + 1
        req = Request(rid, op_key, C.pointer(hc.csr), C.pointer(prm),
                      C.c_void_p(bb.ctypes.data), C.c_void_p(x.ctypes.data),
                      bb.shape[0], maxit, tol)
        _check(load().lsamg_server_submit(self._h, C.byref(req)))
        self._live[rid] = (bb, x, req)
        return rid

    def poll(self, wait_ms: int = 0, cap: int = 256) -> list:
        buf = (Done * cap)()
        cnt = C.c_int32()
        _check(load().lsamg_server_poll(self._h, buf, cap, C.byref(cnt), wait_ms))
        out = []
        for i in range(cnt.value):
            d = buf[i].as_dict()
            d["msg"] = d["msg"].decode(errors="replace")
            bb, x, _ = self._live.pop(d["id"])
            d["x"] = x
            out.append(d)
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().lsamg_server_stats_get(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().lsamg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
