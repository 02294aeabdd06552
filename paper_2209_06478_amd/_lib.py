"""ctypes declarations of the C ABI in include/dsm.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsm.so")

COO, CSR, DIA, ELL, HYB, HDC = range(6)
FORMATS = {"coo": COO, "csr": CSR, "dia": DIA, "ell": ELL, "hyb": HYB, "hdc": HDC}
FORMAT_NAMES = {v: k for k, v in FORMATS.items()}
F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}
CG_F64, CG_IR, CG_JACOBI, CG_IR_CONT = 0, 1, 2, 3

OK = 0
E_INVALID, E_NOMEM, E_INFEASIBLE, E_UNSUPPORTED = -1, -2, -3, -4
E_NOT_CONVERGED, E_BREAKDOWN, E_PENDING, E_DEVICE = -5, -6, -7, -8


class ConvertOpts(C.Structure):
    _fields_ = [("value_dtype", C.c_int), ("hdc_theta", C.c_double), ("max_pad_ratio", C.c_double),
                ("hyb_width", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("format", C.c_int32), ("value_dtype", C.c_int32), ("nrows", C.c_int64), ("ncols", C.c_int64),
                ("nnz", C.c_int64), ("ndiag", C.c_int64), ("ell_width", C.c_int64), ("coo_nnz", C.c_int64),
                ("csr_nnz", C.c_int64), ("bytes", C.c_int64), ("pitch", C.c_int64), ("hdc_theta", C.c_double)]


class ExportBufs(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("row", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("offsets", C.c_void_p), ("dia_val", C.c_void_p), ("ell_col", C.c_void_p),
                ("ell_val", C.c_void_p)]


class SelectOpts(C.Structure):
    _fields_ = [("warmup", C.c_int32), ("reps", C.c_int32), ("use_cache", C.c_int32), ("tune_variant", C.c_int32),
                ("vec_dtype", C.c_int), ("value_dtype", C.c_int), ("max_pad_ratio", C.c_double),
                ("bytes_prefilter", C.c_double), ("target", C.c_int32), ("flush_bytes", C.c_int64)]


class SelectReport(C.Structure):
    _fields_ = [("chosen", C.c_int32), ("chosen_variant", C.c_int32), ("cache_hit", C.c_int32),
                ("status", C.c_int32 * 6), ("median_us", C.c_double * 6), ("convert_us", C.c_double * 6),
                ("bytes", C.c_double * 6)]


class CgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int64), ("mode", C.c_int32), ("inner_tol", C.c_double),
                ("check_every", C.c_int32), ("max_outer", C.c_int32)]


class CgResult(C.Structure):
    _fields_ = [("iters", C.c_int64), ("outer_iters", C.c_int64), ("relres", C.c_double),
                ("relres_true", C.c_double), ("status", C.c_int32)]


class ServerOpts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("hbm_budget", C.c_size_t), ("streams", C.c_int32),
                ("small_rows", C.c_int64), ("batch_max", C.c_int32)]


class Timestamps(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("start_s", C.c_double), ("finish_s", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("budget_waits", C.c_uint64),
                ("requeued", C.c_uint64), ("peak_charged_bytes", C.c_uint64), ("workspace_bytes", C.c_uint64),
                ("busy_s", C.c_double), ("elapsed_s", C.c_double)]


STRUCTS = {"dsm_server_stats": ServerStats, "dsm_convert_opts": ConvertOpts, "dsm_info": Info, "dsm_export_bufs": ExportBufs,
           "dsm_select_opts": SelectOpts, "dsm_select_report": SelectReport, "dsm_cg_opts": CgOpts,
           "dsm_cg_result": CgResult, "dsm_server_opts": ServerOpts, "dsm_timestamps": Timestamps}

_p = C.c_void_p
_st = C.c_int32
SIGNATURES = {
    "dsm_status_string": (C.c_char_p, [_st]),
    "dsm_last_error": (C.c_char_p, []),
    "dsm_version": (C.c_int32, []),
    "dsm_ctx_create": (_st, [C.c_int, C.c_size_t, C.POINTER(_p)]),
    "dsm_ctx_destroy": (_st, [_p]),
    "dsm_ctx_bytes_in_use": (_st, [_p, C.POINTER(C.c_size_t)]),
    "dsm_create_csr": (_st, [_p, C.c_int64, C.c_int64, C.c_int64, _p, _p, _p, C.c_int, _p, C.POINTER(_p)]),
    "dsm_create_coo": (_st, [_p, C.c_int64, C.c_int64, C.c_int64, _p, _p, _p, C.c_int, C.c_int, _p,
                             C.POINTER(_p)]),
    "dsm_matrix_destroy": (_st, [_p]),
    "dsm_convert_opts_default": (None, [C.POINTER(ConvertOpts)]),
    "dsm_convert": (_st, [_p, C.c_int, C.POINTER(ConvertOpts), _p]),
    "dsm_get_info": (_st, [_p, C.POINTER(Info)]),
    "dsm_export": (_st, [_p, C.POINTER(ExportBufs), _p]),
    "dsm_row_stats": (_st, [_p, C.POINTER(C.c_int64), _p]),
    "dsm_values_exact": (_st, [_p, C.c_int32, C.POINTER(C.c_int32), _p]),
    "dsm_extract_diagonal": (_st, [_p, _p, _p]),
    "dsm_update_diagonal": (_st, [_p, _p, _p]),
    "dsm_spmv": (_st, [_p, _p, _p, C.c_int, _p]),
    "dsm_spmv_accumulate": (_st, [_p, _p, _p, C.c_int, _p]),
    "dsm_spmv_noalloc": (_st, [_p, _p, _p, C.c_int, _p]),
    "dsm_spmv_kernel_time": (_st, [_p, _p, _p, C.c_int, C.POINTER(C.c_double), _p]),
    "dsm_set_variant": (_st, [_p, C.c_int32]),
    "dsm_get_variant": (_st, [_p, C.POINTER(C.c_int32)]),
    "dsm_select_opts_default": (None, [C.POINTER(SelectOpts)]),
    "dsm_select": (_st, [_p, C.c_uint32, C.POINTER(SelectOpts), C.POINTER(SelectReport), _p]),
    "dsm_select_cache_clear": (_st, [_p]),
    "dsm_time_spmv": (_st, [_p, _p, _p, C.c_int, C.c_int32, C.c_int32, C.POINTER(C.c_double), _p]),
    "dsm_cg_opts_default": (None, [C.POINTER(CgOpts)]),
    "dsm_cg_solve": (_st, [_p, _p, _p, C.POINTER(CgOpts), C.POINTER(CgResult), _p]),
    "dsm_cg_solve_batched": (_st, [C.c_int32, C.POINTER(_p), C.POINTER(_p), C.POINTER(_p), C.POINTER(CgOpts),
                                   C.POINTER(CgResult), _p]),
    "dsm_server_opts_default": (None, [C.POINTER(ServerOpts)]),
    "dsm_server_create": (_st, [_p, C.POINTER(ServerOpts), C.POINTER(_p)]),
    "dsm_server_submit": (_st, [_p, _p, _p, _p, C.POINTER(CgOpts), C.POINTER(C.c_uint64)]),
    "dsm_server_poll": (_st, [_p, C.c_uint64, C.POINTER(CgResult), C.POINTER(Timestamps)]),
    "dsm_server_wait": (_st, [_p, C.c_uint64, C.POINTER(CgResult), C.POINTER(Timestamps)]),
    "dsm_server_now": (C.c_double, [_p]),
    "dsm_server_get_stats": (_st, [_p, C.POINTER(ServerStats)]),
    "dsm_server_destroy": (_st, [_p]),
    "dsm_stream_probe": (_st, [C.c_int32, _p, _p, C.c_int64, _p]),
    "dsm_gather_probe": (_st, [_p, C.c_int64, _p, C.c_int64, _p, _p]),
    "dsm_mg_create": (_st, [_p, C.c_int32, C.POINTER(_p), C.POINTER(_p), C.POINTER(_p), _p, C.POINTER(_p)]),
    "dsm_mg_destroy": (_st, [_p]),
    "dsm_mg_symgs": (_st, [_p, C.c_int32, _p, _p, _p]),
    "dsm_mg_apply": (_st, [_p, _p, _p, _p]),
    "dsm_pcg_mg_solve": (_st, [_p, _p, _p, C.POINTER(CgOpts), C.POINTER(CgResult), _p]),
}

PROBE_READ, PROBE_COPY, PROBE_WRITE, PROBE_PARTIALS = 0, 1, 2, 4096

_lib = None


def load(path=None):
    """Loads libdsm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libdsm.so not found at {path}: build it with paper_2209_06478_amd/build.py "
                           "(there is no CPU fallback)")
    # torch first: its wheel carries its own HIP runtime under the same
    # soname (libamdhip64.so.7) as the system one libdsm was linked against,
    # and the first one loaded serves the process.  Device memory and
    # streams come from torch, so libdsm must run on torch's runtime; loaded
    # the other way round, torch's runtime finds no GPU.
    import torch  # noqa: F401
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
