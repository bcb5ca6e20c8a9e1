"""ctypes declarations of the C ABI in include/ihsbin.h.

Loading fails loudly (ImportError) when libihsbin.so has not been built: there
is no fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libihsbin.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, ENOCONV, ERANGE, EUNSUP, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7, -8
DENSE, CSR = 0, 1
F32, F64 = 0, 1
GAUSSIAN, SRHT, COUNTSKETCH, SJLT = 0, 1, 2, 3
SKETCHES = {"gaussian": GAUSSIAN, "srht": SRHT, "countsketch": COUNTSKETCH, "sjlt": SJLT}

EXPORTED = [
    "ihsbin_status_str", "ihsbin_version", "ihsbin_opts_default", "ihsbin_create",
    "ihsbin_destroy", "ihsbin_last_error", "ihsbin_path_build", "ihsbin_path_eval",
    "ihsbin_path_get_info", "ihsbin_path_intervals", "ihsbin_path_basis", "ihsbin_path_free",
    "ihsbin_solve_path", "ihsbin_sketch_draws", "ihsbin_sketch_apply", "ihsbin_precond_factor",
    "ihsbin_ata_apply",
    "ihsbin_gram", "ihsbin_sketch_gram", "ihsbin_alg4_opts_default", "ihsbin_sketch_size",
    "ihsbin_build_footprint", "ihsbin_sketch_apply_prec", "ihsbin_path_set_stream", "ihsbin_server_opts_default",
    "ihsbin_server_create", "ihsbin_server_submit", "ihsbin_server_wait",
    "ihsbin_server_get_stats", "ihsbin_server_last_error", "ihsbin_server_destroy",
    "ihsbin_sketch_indices_host", "ihsbin_sketch_indices_device", "ihsbin_csr_transpose",
    "ihsbin_path_eval_noalloc", "ihsbin_path_build_batch", "ihsbin_ata_apply_tiled",
]


class Matrix(C.Structure):
    _fields_ = [("format", C.c_int32), ("dtype", C.c_int32), ("n", C.c_int64), ("d", C.c_int64),
                ("ld", C.c_int64), ("nnz", C.c_int64), ("vals", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p)]


class Alg4Opts(C.Structure):
    _fields_ = [("gamma1", C.c_double), ("gamma2", C.c_double), ("gamma3", C.c_double),
                ("eps", C.c_double), ("max_iter", C.c_int32), ("max_armijo", C.c_int32)]


class Alg4Result(C.Structure):
    _fields_ = [("m", C.c_int64), ("iters", C.c_int32), ("doublings", C.c_int32),
                ("delta0", C.c_double), ("delta", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Opts(C.Structure):
    _fields_ = [("sketch", C.c_int32), ("sjlt_s", C.c_int32), ("m", C.c_int64),
                ("seed", C.c_uint64), ("tol", C.c_double), ("k_max", C.c_int32),
                ("k_fixed", C.c_int32), ("L", C.c_int32), ("centred", C.c_int32),
                ("adaptive_m", C.c_int32), ("rate_target", C.c_double), ("m_max", C.c_int64),
                ("lanczos_steps", C.c_int32), ("timing", C.c_int32),
                ("taus", C.POINTER(C.c_double)), ("gram_prec", C.c_int32),
                ("alg4", C.POINTER(Alg4Opts)), ("sketch_prec", C.c_int32),
                ("sigma_d2", C.c_double), ("basis_prec", C.c_int32), ("f32_switch", C.c_double),
                ("graph_steps", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("m_used", C.c_int64), ("L", C.c_int32), ("k_max_used", C.c_int32),
                ("k_sum", C.c_int32), ("n_unconverged", C.c_int32),
                ("sketch_trials", C.c_int32), ("steps", C.c_int32),
                ("ms_sketch", C.c_double), ("ms_factor", C.c_double),
                ("ms_spectrum", C.c_double), ("ms_basis", C.c_double), ("ms_total", C.c_double),
                ("ata_launches", C.c_int64), ("ata_flops", C.c_double), ("ata_ms_y", C.c_double),
                ("ata_ms_w", C.c_double), ("ata_bytes_a", C.c_double),
                ("peak_bytes", C.c_int64), ("est_rel_err", C.c_double),
                ("ata_f32_launches", C.c_int64), ("ata_f32_flops", C.c_double),
                ("ata_f32_ms_y", C.c_double), ("ata_f32_ms_w", C.c_double),
                ("bytes_moved", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("workers", C.c_int32), ("reserved", C.c_int32), ("hbm_budget", C.c_int64),
                ("keep_bytes", C.c_int64)]


class RequestInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("worker", C.c_int32), ("footprint", C.c_int64),
                ("ms_queue", C.c_double), ("ms_build", C.c_double), ("ms_total", C.c_double),
                ("report", Report), ("message", C.c_char * 160)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("report", "message")}
        d["report"] = self.report.as_dict()
        d["message"] = self.message.decode(errors="replace")
        return d


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("retried", C.c_int64),
                ("workers", C.c_int32), ("queued", C.c_int32), ("inflight", C.c_int32),
                ("max_concurrent", C.c_int32), ("budget", C.c_int64),
                ("inflight_bytes", C.c_int64), ("max_inflight_bytes", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PathInfo(C.Structure):
    _fields_ = [("L", C.c_int32), ("K", C.c_int32), ("d", C.c_int64), ("m_used", C.c_int64),
                ("lam_min", C.c_double), ("lam_max", C.c_double), ("centred", C.c_int32),
                ("dual", C.c_int32)]


def _declare(lib):
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    pd = C.POINTER(C.c_double)
    sig = {
        "ihsbin_status_str": (C.c_char_p, [C.c_int]),
        "ihsbin_version": (C.c_char_p, []),
        "ihsbin_opts_default": (None, [C.POINTER(Opts)]),
        "ihsbin_create": (C.c_int, [C.POINTER(vp), C.c_int, vp]),
        "ihsbin_destroy": (C.c_int, [vp]),
        "ihsbin_last_error": (C.c_char_p, [vp]),
        "ihsbin_path_build": (C.c_int, [vp, C.POINTER(Matrix), vp, i64, i64, dbl, dbl,
                                        C.POINTER(Opts), C.POINTER(vp), C.POINTER(Report)]),
        "ihsbin_path_eval": (C.c_int, [vp, pd, i64, vp, i64, i32]),
        "ihsbin_path_build_batch": (C.c_int, [vp, i32, C.POINTER(Matrix), i64, vp, i64, i64, i64,
                                              dbl, dbl, C.POINTER(Opts), C.POINTER(vp),
                                              C.POINTER(Report)]),
        "ihsbin_path_eval_noalloc": (C.c_int, [vp, pd, i64, vp, i64, i32]),
        "ihsbin_path_get_info": (C.c_int, [vp, C.POINTER(PathInfo)]),
        "ihsbin_path_intervals": (C.c_int, [vp, pd, pd, pd, pd, pd, C.POINTER(C.c_int32)]),
        "ihsbin_path_basis": (C.c_int, [vp, i32, vp]),
        "ihsbin_path_free": (C.c_int, [vp]),
        "ihsbin_solve_path": (C.c_int, [vp, C.POINTER(Matrix), vp, i64, i64, pd, i64,
                                        C.POINTER(Opts), vp, i64, i32, C.POINTER(Report)]),
        "ihsbin_sketch_draws": (C.c_int, [vp, i32, u64, i64, i64, i32, vp, vp]),
        "ihsbin_sketch_apply": (C.c_int, [vp, C.POINTER(Matrix), i32, i32, i64, u64, vp]),
        "ihsbin_sketch_apply_prec": (C.c_int, [vp, C.POINTER(Matrix), i32, i32, i64, u64, i32, vp]),
        "ihsbin_precond_factor": (C.c_int, [vp, vp, i64, i64, pd, i32, vp, vp]),
        "ihsbin_ata_apply": (C.c_int, [vp, C.POINTER(Matrix), vp, i64, i64, vp, i64]),
        "ihsbin_gram": (C.c_int, [vp, vp, i64, i64, i32, vp]),
        "ihsbin_sketch_gram": (C.c_int, [vp, C.POINTER(Matrix), i32, i32, i64, u64, i32, i32, vp]),
        "ihsbin_ata_apply_tiled": (C.c_int, [vp, C.POINTER(Matrix), vp, i64, i64, vp, i64, i32,
                                             i32, i32]),
        "ihsbin_alg4_opts_default": (None, [C.POINTER(Alg4Opts)]),
        "ihsbin_build_footprint": (C.c_int, [C.POINTER(Matrix), i64, dbl, dbl, C.POINTER(Opts),
                                             C.POINTER(C.c_int64)]),
        "ihsbin_path_set_stream": (C.c_int, [vp, vp]),
        "ihsbin_server_opts_default": (None, [C.POINTER(ServerOpts)]),
        "ihsbin_server_create": (C.c_int, [C.POINTER(vp), C.c_int, C.POINTER(ServerOpts)]),
        "ihsbin_server_submit": (C.c_int, [vp, C.POINTER(Matrix), vp, i64, i64, dbl, dbl,
                                           C.POINTER(Opts), C.POINTER(C.c_int64)]),
        "ihsbin_server_wait": (C.c_int, [vp, i64, i64, vp, C.POINTER(vp),
                                         C.POINTER(RequestInfo)]),
        "ihsbin_server_get_stats": (C.c_int, [vp, C.POINTER(ServerStats)]),
        "ihsbin_server_last_error": (C.c_char_p, [vp]),
        "ihsbin_server_destroy": (C.c_int, [vp]),
        "ihsbin_sketch_indices_host": (C.c_int, [u64, i32, i64, i64, i32, vp, vp]),
        "ihsbin_sketch_indices_device": (C.c_int, [vp, u64, i32, i64, i64, i32, vp, vp]),
        "ihsbin_csr_transpose": (C.c_int, [vp, C.POINTER(Matrix), vp, vp, vp]),
        "ihsbin_sketch_size": (C.c_int, [vp, C.POINTER(Matrix), vp, i64, i64, dbl,
                                         C.POINTER(Opts), C.POINTER(Alg4Opts),
                                         C.POINTER(Alg4Result), vp, i64, pd, i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib():
    """The loaded library; raises ImportError when it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: run __graft_entry__.build() first "
                              "(the solver has no non-HIP implementation)")
        _LIB = _declare(C.CDLL(LIB_PATH))
    return _LIB
