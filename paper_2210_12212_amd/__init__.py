"""MI355X ridge-regularization-path solver (IHS-BIN), Python binding.

Every step of the computation runs in the HIP library behind the C ABI of
include/ihsbin.h; this module only marshals arguments.  PyTorch supplies the
device memory (tensors) and the stream.  The names follow the C calls:

    ctx  = Context(device=0)
    path = ctx.path_build(A, B, lam_min, lam_max, sketch="srht", m=1024)
    X    = path.eval(lambdas)          # T x d x K float64 tensor
    path.free()

A is a dense CUDA tensor (n x d, float32 or float64, row-major) or a CsrInput
of CUDA tensors.  B is n x K (or n) in A's dtype.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L

__all__ = ["Context", "Path", "Server", "CsrInput", "IhsbinError", "solve_path",
           "default_opts", "build_footprint", "sketch_indices_host"]


class IhsbinError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.lib().ihsbin_status_str(status).decode()} ({status}): {msg}")
        self.status = status


@dataclass
class CsrInput:
    """CSR matrix on the device: int32 row_ptr (n+1), int32 col_idx, vals."""
    row_ptr: object
    col_idx: object
    vals: object
    n: int
    d: int

    @property
    def shape(self):
        return (self.n, self.d)


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return L.F32
    if t.dtype == torch.float64:
        return L.F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _require_cuda(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")


def _matrix(A) -> L.Matrix:
    m = L.Matrix()
    if isinstance(A, CsrInput):
        for nm in ("row_ptr", "col_idx", "vals"):
            _require_cuda(getattr(A, nm), nm)
        torch = _torch()
        if A.row_ptr.dtype != torch.int32 or A.col_idx.dtype != torch.int32:
            raise TypeError("CSR indices must be int32")
        m.format, m.dtype = L.CSR, _dtype_code(A.vals)
        m.n, m.d, m.ld, m.nnz = A.n, A.d, A.d, A.vals.numel()
        m.vals, m.row_ptr, m.col_idx = A.vals.data_ptr(), A.row_ptr.data_ptr(), A.col_idx.data_ptr()
    else:
        _require_cuda(A, "A")
        if A.dim() != 2 or A.stride(1) != 1:
            raise ValueError("A must be 2-D with unit column stride")
        m.format, m.dtype = L.DENSE, _dtype_code(A)
        m.n, m.d, m.ld, m.nnz = A.shape[0], A.shape[1], A.stride(0), 0
        m.vals = A.data_ptr()
    return m


def default_opts(**kw) -> L.Opts:
    o = L.Opts()
    L.lib().ihsbin_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "sketch" and isinstance(v, str):
            v = L.SKETCHES[v]
        if k in ("taus", "alg4"):
            continue
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _taus_ptr(taus):
    if taus is None:
        return None, None
    arr = (C.c_double * len(taus))(*[float(t) for t in taus])
    return arr, C.cast(arr, C.POINTER(C.c_double))


def alg4_opts(**kw) -> L.Alg4Opts:
    """ihsbin_alg4_opts_default, then the given fields."""
    a = L.Alg4Opts()
    L.lib().ihsbin_alg4_opts_default(C.byref(a))
    for k, v in kw.items():
        if not hasattr(a, k):
            raise KeyError(f"unknown Algorithm 4 option {k}")
        setattr(a, k, v)
    return a


def _with_pointers(opts):
    """Opts from keyword options plus the host arrays they point to (kept
    alive by the caller for the duration of the call)."""
    o = default_opts(**opts)
    keep_t, ptr = _taus_ptr(opts.get("taus"))
    o.taus = ptr
    keep_a = None
    if opts.get("alg4") is not None:
        keep_a = alg4_opts(**opts["alg4"])
        o.alg4 = C.pointer(keep_a)
    return o, (keep_t, keep_a)


class Context:
    """ihsbin_create / ihsbin_destroy on a device and a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = L.lib().ihsbin_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if rc != L.OK:
            raise IhsbinError(rc, "ihsbin_create")
        self._h = h

    def _check(self, rc, allow=()):
        if rc != L.OK and rc not in allow:
            raise IhsbinError(rc, L.lib().ihsbin_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ihsbin_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- path
    def path_build(self, A, B, lam_min: float, lam_max: float, allow_noconv: bool = True, **opts):
        """ihsbin_path_build; returns (Path, report dict)."""
        Bm = B if B.dim() == 2 else B.reshape(-1, 1)
        _require_cuda(Bm, "B")
        if Bm.stride(1) != 1:
            raise ValueError("B must have unit column stride")
        o, keep = _with_pointers(opts)
        mat = _matrix(A)
        rep = L.Report()
        ph = C.c_void_p()
        rc = L.lib().ihsbin_path_build(self._h, C.byref(mat), C.c_void_p(Bm.data_ptr()), Bm.shape[1],
                                       Bm.stride(0), float(lam_min), float(lam_max), C.byref(o),
                                       C.byref(ph), C.byref(rep))
        self._check(rc, allow=(L.ENOCONV,) if allow_noconv else ())
        r = rep.as_dict()
        r["status"] = rc
        return Path(ph, self), r

    def path_build_batch(self, A, B, lam_min: float, lam_max: float, allow_noconv: bool = True,
                         **opts):
        """ihsbin_path_build_batch for P problems stacked along dim 0: A is a
        P x n x d device tensor (unit column stride), B P x n x K (or P x n).
        Returns (list of P Paths, report dict)."""
        Bm = B if B.dim() == 3 else B.reshape(B.shape[0], B.shape[1], 1)
        _require_cuda(A, "A")
        _require_cuda(Bm, "B")
        if A.dim() != 3 or A.stride(2) != 1 or Bm.stride(2) != 1:
            raise ValueError("A (P x n x d) and B (P x n x K) need unit column stride")
        P = A.shape[0]
        if Bm.shape[0] != P or Bm.shape[1] != A.shape[1]:
            raise ValueError("A and B disagree on P or n")
        o, keep = _with_pointers(opts)
        mat = L.Matrix()
        mat.format, mat.dtype = L.DENSE, _dtype_code(A)
        mat.n, mat.d, mat.ld, mat.nnz = A.shape[1], A.shape[2], A.stride(1), 0
        mat.vals = A.data_ptr()
        handles = (C.c_void_p * P)()
        rep = L.Report()
        rc = L.lib().ihsbin_path_build_batch(self._h, P, C.byref(mat), A.stride(0),
                                             C.c_void_p(Bm.data_ptr()), Bm.shape[2], Bm.stride(1),
                                             Bm.stride(0), float(lam_min), float(lam_max),
                                             C.byref(o), handles, C.byref(rep))
        self._check(rc, allow=(L.ENOCONV,) if allow_noconv else ())
        r = rep.as_dict()
        r["status"] = rc
        return [Path(C.c_void_p(handles[p]), self) for p in range(P)], r

    def solve_path(self, A, B, lambdas, x_dtype=None, **opts):
        """ihsbin_solve_path: build, evaluate at every lambda, free."""
        torch = _torch()
        Bm = B if B.dim() == 2 else B.reshape(-1, 1)
        lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
        x_dtype = x_dtype or torch.float64
        X = torch.empty((len(lam), A.shape[1], Bm.shape[1]), dtype=x_dtype, device=Bm.device)
        o, keep = _with_pointers(opts)
        mat = _matrix(A)
        rep = L.Report()
        rc = L.lib().ihsbin_solve_path(self._h, C.byref(mat), C.c_void_p(Bm.data_ptr()), Bm.shape[1],
                                       Bm.stride(0), lam.ctypes.data_as(C.POINTER(C.c_double)),
                                       len(lam), C.byref(o), C.c_void_p(X.data_ptr()), X.stride(1),
                                       _dtype_code(X), C.byref(rep))
        self._check(rc, allow=(L.ENOCONV,))
        r = rep.as_dict()
        r["status"] = rc
        return X, r

    def sketch_size(self, A, B, lam: float, alg4=None, trace_rows: int = 64, **opts):
        """ihsbin_sketch_size (Algorithm 4 at lam) -> (result dict, X, trace).

        X is the last iterate (d x K float64; n < d: the dual iterate, n x K)
        and trace a (updates x 5) float64 array of (m, tau, delta_k,
        delta_{k+1}, doubled) rows."""
        torch = _torch()
        Bm = B if B.dim() == 2 else B.reshape(-1, 1)
        _require_cuda(Bm, "B")
        if Bm.stride(1) != 1:
            raise ValueError("B must have unit column stride")
        o, keep = _with_pointers(opts)
        a = alg4_opts(**(alg4 or {}))
        n, d = A.shape
        rows = d if n >= d else n
        X = torch.empty((rows, Bm.shape[1]), dtype=torch.float64, device=Bm.device)
        tr = np.zeros((max(trace_rows, 0), 5))
        res = L.Alg4Result()
        mat = _matrix(A)
        self._check(L.lib().ihsbin_sketch_size(
            self._h, C.byref(mat), C.c_void_p(Bm.data_ptr()), Bm.shape[1], Bm.stride(0),
            float(lam), C.byref(o), C.byref(a), C.byref(res), C.c_void_p(X.data_ptr()),
            X.stride(0), tr.ctypes.data_as(C.POINTER(C.c_double)) if trace_rows > 0 else None,
            int(trace_rows)))
        r = res.as_dict()
        return r, X, tr[:min(r["iters"], trace_rows)]

    # --------------------------------------------------------- step calls
    def sketch_draws(self, sketch: str, seed: int, n: int, m: int, sjlt_s: int = 1):
        """ihsbin_sketch_draws -> (idx int32, sign int8) device tensors."""
        torch = _torch()
        code = L.SKETCHES[sketch]
        dev = torch.device("cuda", self.device)
        if code == L.SRHT:
            idx = torch.empty(m, dtype=torch.int32, device=dev)
            sign = torch.empty(n, dtype=torch.int8, device=dev)
        else:
            s = sjlt_s if code == L.SJLT else 1
            idx = torch.empty((n, s), dtype=torch.int32, device=dev)
            sign = torch.empty((n, s), dtype=torch.int8, device=dev)
        self._check(L.lib().ihsbin_sketch_draws(self._h, code, seed, n, m, sjlt_s,
                                                C.c_void_p(idx.data_ptr()), C.c_void_p(sign.data_ptr())))
        return idx, sign

    def sketch_indices_device(self, seed: int, sketch: str, n: int, m: int, sjlt_s: int = 1):
        """ihsbin_sketch_indices_device -> (idx int32, sign int8) device tensors
        (the layouts of sketch_draws)."""
        torch = _torch()
        code = L.SKETCHES[sketch]
        dev = torch.device("cuda", self.device)
        s = sjlt_s if code == L.SJLT else 1
        idx = torch.empty(m if code == L.SRHT else n * s, dtype=torch.int32, device=dev)
        sign = torch.empty(n if code == L.SRHT else n * s, dtype=torch.int8, device=dev)
        self._check(L.lib().ihsbin_sketch_indices_device(
            self._h, seed, code, n, m, sjlt_s, C.c_void_p(idx.data_ptr()),
            C.c_void_p(sign.data_ptr())))
        return idx, sign

    def csr_transpose(self, A):
        """ihsbin_csr_transpose -> (col_ptr, row, vals) device tensors of the
        library's column-major copy of the CSR matrix A."""
        torch = _torch()
        if not isinstance(A, CsrInput):
            raise TypeError("csr_transpose needs a CsrInput")
        nnz = A.vals.numel()
        col_ptr = torch.empty(A.d + 1, dtype=torch.int32, device=A.vals.device)
        row = torch.empty(max(nnz, 1), dtype=torch.int32, device=A.vals.device)
        vals = torch.empty(max(nnz, 1), dtype=A.vals.dtype, device=A.vals.device)
        mat = _matrix(A)
        self._check(L.lib().ihsbin_csr_transpose(self._h, C.byref(mat),
                                                 C.c_void_p(col_ptr.data_ptr()),
                                                 C.c_void_p(row.data_ptr()),
                                                 C.c_void_p(vals.data_ptr())))
        return col_ptr, row[:nnz], vals[:nnz]

    def sketch_apply(self, A, sketch: str, m: int, seed: int, sjlt_s: int = 1,
                     prec: str = "f64"):
        """ihsbin_sketch_apply_prec -> SA (m x d float64); prec "f64" or
        "bf16" or "fp8" (the Gaussian sketch on the BF16 or FP8 matrix cores)."""
        torch = _torch()
        SA = torch.empty((m, A.shape[1]), dtype=torch.float64, device=torch.device("cuda", self.device))
        mat = _matrix(A)
        self._check(L.lib().ihsbin_sketch_apply_prec(
            self._h, C.byref(mat), L.SKETCHES[sketch], sjlt_s, m, seed,
            {"f64": 0, "bf16": 1, "fp8": 2}[prec], C.c_void_p(SA.data_ptr())))
        return SA

    def precond_factor(self, SA, lam0, want_inverse: bool = True):
        """ihsbin_precond_factor -> (Lfac, Linv) as nl x d x d float64 tensors."""
        torch = _torch()
        lam0 = np.ascontiguousarray(np.atleast_1d(np.asarray(lam0, dtype=np.float64)))
        m, d = SA.shape
        Lf = torch.empty((len(lam0), d, d), dtype=torch.float64, device=SA.device)
        Li = torch.empty_like(Lf) if want_inverse else None
        self._check(L.lib().ihsbin_precond_factor(
            self._h, C.c_void_p(SA.contiguous().data_ptr()), m, d,
            lam0.ctypes.data_as(C.POINTER(C.c_double)), len(lam0), C.c_void_p(Lf.data_ptr()),
            C.c_void_p(Li.data_ptr()) if Li is not None else None))
        return Lf, Li

    def gram(self, SA, prec: str = "f64"):
        """ihsbin_gram -> G = SA^T SA (d x d float64; lower triangle and the
        diagonal tiles written).  prec: "f64" or "bf16x3"."""
        torch = _torch()
        SA = SA.contiguous()
        m, d = SA.shape
        G = torch.zeros((d, d), dtype=torch.float64, device=SA.device)
        code = {"f64": 0, "bf16x3": 1}[prec]
        self._check(L.lib().ihsbin_gram(self._h, C.c_void_p(SA.data_ptr()), m, d, code,
                                        C.c_void_p(G.data_ptr())))
        return G

    def sketch_gram(self, A, sketch: str, m: int, seed: int, sjlt_s: int = 1,
                    sketch_prec: str = "f64", gram_prec: str = "f64"):
        """ihsbin_sketch_gram -> G = (SA)^T SA as a path build forms it (d x d
        float64; lower triangle and the diagonal tiles written)."""
        torch = _torch()
        d = A.shape[1]
        dev = A.vals.device if isinstance(A, CsrInput) else A.device
        G = torch.zeros((d, d), dtype=torch.float64, device=dev)
        mat = _matrix(A)
        self._check(L.lib().ihsbin_sketch_gram(
            self._h, C.byref(mat), L.SKETCHES[sketch], sjlt_s, m, seed,
            {"f64": 0, "bf16": 1, "fp8": 2}[sketch_prec], {"f64": 0, "bf16x3": 1}[gram_prec],
            C.c_void_p(G.data_ptr())))
        return G

    def ata_apply_tiled(self, A, U, prec: str = "f64", q: int = 0, splits: int = 0):
        """ihsbin_ata_apply_tiled -> W = A^T A U with a chosen tiling (tuning)."""
        U = U if U.dim() == 2 else U.reshape(-1, 1)
        W = _torch().empty_like(U)
        mat = _matrix(A)
        self._check(L.lib().ihsbin_ata_apply_tiled(
            self._h, C.byref(mat), C.c_void_p(U.data_ptr()), U.shape[1], U.stride(0),
            C.c_void_p(W.data_ptr()), W.stride(0), {"f64": 0, "f32": 1}[prec], int(q), int(splits)))
        return W

    def ata_apply(self, A, U):
        """ihsbin_ata_apply -> W = A^T A U (d x w float64)."""
        U = U if U.dim() == 2 else U.reshape(-1, 1)
        W = _torch().empty_like(U)
        mat = _matrix(A)
        self._check(L.lib().ihsbin_ata_apply(self._h, C.byref(mat), C.c_void_p(U.data_ptr()),
                                             U.shape[1], U.stride(0), C.c_void_p(W.data_ptr()),
                                             W.stride(0)))
        return W


def sketch_indices_host(seed: int, sketch: str, n: int, m: int, sjlt_s: int = 1):
    """ihsbin_sketch_indices_host -> (idx int32, sign int8) numpy arrays: the
    library's host computation of the integer sketch draws (CountSketch/SJLT:
    n*s of each; SRHT: m sampled rows and n signs)."""
    code = L.SKETCHES[sketch]
    s = sjlt_s if code == L.SJLT else 1
    idx = np.zeros(m if code == L.SRHT else n * s, dtype=np.int32)
    sign = np.zeros(n if code == L.SRHT else n * s, dtype=np.int8)
    rc = L.lib().ihsbin_sketch_indices_host(int(seed), code, int(n), int(m), int(sjlt_s),
                                            idx.ctypes.data_as(C.c_void_p),
                                            sign.ctypes.data_as(C.c_void_p))
    if rc != L.OK:
        raise IhsbinError(rc, "ihsbin_sketch_indices_host")
    return idx, sign


def build_footprint(shape, K: int, lam_min: float, lam_max: float, csr: bool = False,
                    dtype: str = "float32", **opts) -> int:
    """ihsbin_build_footprint: upper estimate (bytes) of the device memory one
    build allocates for an n x d problem with K right-hand sides."""
    m = L.Matrix()
    m.format = L.CSR if csr else L.DENSE
    m.dtype = L.F32 if dtype == "float32" else L.F64
    m.n, m.d = int(shape[0]), int(shape[1])
    m.ld = m.d
    o, keep = _with_pointers(opts)
    out = C.c_int64()
    rc = L.lib().ihsbin_build_footprint(C.byref(m), int(K), float(lam_min), float(lam_max),
                                        C.byref(o), C.byref(out))
    if rc != L.OK:
        raise IhsbinError(rc, "ihsbin_build_footprint")
    return int(out.value)


class Server:
    """ihsbin_server_*: concurrent path builds on one device.

    submit() keeps references to A and B until the request is collected by
    wait(), which returns (Path or None, info dict); the path is bound to the
    given torch stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, workers: int = 4, hbm_budget: int = 0,
                 keep_bytes: int | None = None):
        o = L.ServerOpts()
        L.lib().ihsbin_server_opts_default(C.byref(o))
        o.workers, o.hbm_budget = workers, hbm_budget
        if keep_bytes is not None:
            o.keep_bytes = keep_bytes
        h = C.c_void_p()
        rc = L.lib().ihsbin_server_create(C.byref(h), device, C.byref(o))
        if rc != L.OK:
            raise IhsbinError(rc, "ihsbin_server_create")
        self._h = h
        self.device = device
        self._held = {}

    def submit(self, A, B, lam_min: float, lam_max: float, **opts) -> int:
        Bm = B if B.dim() == 2 else B.reshape(-1, 1)
        _require_cuda(Bm, "B")
        if Bm.stride(1) != 1:
            raise ValueError("B must have unit column stride")
        o, keep = _with_pointers(opts)
        mat = _matrix(A)
        # the caller's pending work on A and B must be complete on the device
        _torch().cuda.current_stream(self.device).synchronize()
        rid = C.c_int64()
        rc = L.lib().ihsbin_server_submit(self._h, C.byref(mat), C.c_void_p(Bm.data_ptr()),
                                          Bm.shape[1], Bm.stride(0), float(lam_min),
                                          float(lam_max), C.byref(o), C.byref(rid))
        if rc != L.OK:
            raise IhsbinError(rc, L.lib().ihsbin_server_last_error(self._h).decode())
        self._held[rid.value] = (A, Bm)
        return rid.value

    def wait(self, rid: int, timeout_ms: int = -1, stream=None, allow_noconv: bool = True):
        """-> (Path, info) once finished; (None, None) when timeout_ms runs out."""
        torch = _torch()
        stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ph = C.c_void_p()
        info = L.RequestInfo()
        rc = L.lib().ihsbin_server_wait(self._h, int(rid), int(timeout_ms),
                                        C.c_void_p(stream.cuda_stream), C.byref(ph), C.byref(info))
        if rc == L.EAGAIN:
            return None, None
        self._held.pop(rid, None)
        d = info.as_dict()
        if rc != L.OK and not (allow_noconv and rc == L.ENOCONV):
            if ph.value:
                L.lib().ihsbin_path_free(ph)
            raise IhsbinError(rc, d["message"])
        return Path(ph, device=self.device), d

    def stats(self) -> dict:
        st = L.ServerStats()
        L.lib().ihsbin_server_get_stats(self._h, C.byref(st))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            L.lib().ihsbin_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Path:
    """A built path (ihsbin_path): basis resident on the device."""

    def __init__(self, handle, ctx: Context | None = None, device: int | None = None):
        self._h = handle
        self._ctx = ctx
        self.device = ctx.device if ctx is not None else (device or 0)
        info = L.PathInfo()
        rc = L.lib().ihsbin_path_get_info(self._h, C.byref(info))
        if rc != L.OK:
            raise IhsbinError(rc, "ihsbin_path_get_info")
        self.L, self.K, self.d, self.m_used = info.L, info.K, info.d, info.m_used
        self.lam_min, self.lam_max, self.centred = info.lam_min, info.lam_max, info.centred
        self.dual = info.dual

    def eval(self, lambdas, out=None, dtype=None):
        """ihsbin_path_eval -> X (T x d x K)."""
        torch = _torch()
        lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))
        if out is None:
            out = torch.empty((len(lam), self.d, self.K), dtype=dtype or torch.float64,
                              device=torch.device("cuda", self.device))
        else:
            # the library writes T blocks of d rows with row stride ldx and
            # block stride d * ldx: the tensor must span exactly that
            if tuple(out.shape) != (len(lam), self.d, self.K):
                raise ValueError(f"out must have shape {(len(lam), self.d, self.K)}")
            if not out.is_cuda or out.device.index != self.device:
                raise ValueError(f"out must be on cuda:{self.device}")
            if len(lam) and (out.stride(2) != 1 or out.stride(1) < self.K
                             or out.stride(0) != self.d * out.stride(1)):
                raise ValueError("out needs unit column stride and block stride d * row stride")
        rc = L.lib().ihsbin_path_eval(self._h, lam.ctypes.data_as(C.POINTER(C.c_double)), len(lam),
                                      C.c_void_p(out.data_ptr()), out.stride(1), _dtype_code(out))
        if rc != L.OK:
            raise IhsbinError(rc, "ihsbin_path_eval")
        return out

    def eval_noalloc(self, lambdas, out):
        """ihsbin_path_eval_noalloc into a preallocated out (T x d x K, the
        layout eval accepts); the library allocates no device memory."""
        lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))
        if tuple(out.shape) != (len(lam), self.d, self.K) or not out.is_cuda:
            raise ValueError(f"out must be a device tensor of shape {(len(lam), self.d, self.K)}")
        if len(lam) and (out.stride(2) != 1 or out.stride(1) < self.K
                         or out.stride(0) != self.d * out.stride(1)):
            raise ValueError("out needs unit column stride and block stride d * row stride")
        rc = L.lib().ihsbin_path_eval_noalloc(self._h, lam.ctypes.data_as(C.POINTER(C.c_double)),
                                              len(lam), C.c_void_p(out.data_ptr()), out.stride(1),
                                              _dtype_code(out))
        if rc != L.OK:
            raise IhsbinError(rc, "ihsbin_path_eval_noalloc")
        return out

    def intervals(self):
        """ihsbin_path_intervals -> dict of numpy arrays (lo, hi, lam0, tau, rate, k)."""
        arrs = {k: np.zeros(self.L) for k in ("lo", "hi", "lam0", "tau", "rate")}
        k = np.zeros(self.L, dtype=np.int32)
        ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        rc = L.lib().ihsbin_path_intervals(self._h, ptr(arrs["lo"]), ptr(arrs["hi"]), ptr(arrs["lam0"]),
                                           ptr(arrs["tau"]), ptr(arrs["rate"]),
                                           k.ctypes.data_as(C.POINTER(C.c_int32)))
        if rc != L.OK:
            raise IhsbinError(rc, "ihsbin_path_intervals")
        arrs["k"] = k
        return arrs

    def basis(self, l: int):
        """ihsbin_path_basis -> k_l x d x K float64 tensor."""
        torch = _torch()
        k = int(self.intervals()["k"][l])
        out = torch.empty((k, self.d, self.K), dtype=torch.float64,
                          device=torch.device("cuda", self._ctx.device))
        rc = L.lib().ihsbin_path_basis(self._h, l, C.c_void_p(out.data_ptr()))
        if rc != L.OK:
            raise IhsbinError(rc, "ihsbin_path_basis")
        return out

    def free(self):
        if getattr(self, "_h", None):
            L.lib().ihsbin_path_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solve_path(A, B, lambdas, device: int = 0, **opts):
    """One-shot ihsbin_solve_path on a temporary context."""
    ctx = Context(device)
    try:
        return ctx.solve_path(A, B, lambdas, **opts)
    finally:
        ctx.close()
