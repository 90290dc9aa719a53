"""ctypes declarations of libjavelin.so (the C ABI in include/javelin.h).

Argument marshalling only: no step of the method runs here.  Loading fails
loudly when the library has not been built.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjavelin.so")

OK = 0
STATUS = {0: "ILU_OK", 1: "ILU_ERR_ARG", 2: "ILU_ERR_CSR", 3: "ILU_ERR_NOMEM", 4: "ILU_ERR_HIP",
          5: "ILU_ERR_ZERO_PIVOT", 6: "ILU_ERR_NONFINITE", 7: "ILU_ERR_NOCONV", 8: "ILU_ERR_BREAKDOWN",
          9: "ILU_ERR_STATE", 10: "ILU_ERR_UNSUPPORTED", 11: "ILU_ERR_TIMEOUT"}
ERR_ARG, ERR_CSR, ERR_NOMEM, ERR_HIP, ERR_ZERO_PIVOT, ERR_NONFINITE = 1, 2, 3, 4, 5, 6
ERR_NOCONV, ERR_BREAKDOWN, ERR_STATE, ERR_UNSUPPORTED, ERR_TIMEOUT = 7, 8, 9, 10, 11
PATTERN_LOWER_SYM, PATTERN_LOWER_A, PATTERN_UPPER_A = 0, 1, 2
PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2
PERMUTED_SPACE = 1
SCHED_AUTO, SCHED_LEVEL, SCHED_SYNCFREE, SCHED_TILED = 0, 1, 2, 3
CAST_F32, CAST_BF16, FACTOR_MODIFIED = 1, 2, 0x100
ORDER_NATURAL, ORDER_RCM = 0, 1
STAGE_FACTOR, STAGE_FORWARD, STAGE_BACKWARD, STAGE_SPMV, STAGE_FACTOR_CALL, STAGE_APPLY_CALL = 0, 1, 2, 3, 4, 5
STAGE_COUNT = 6
STAGES = ["factor", "forward", "backward", "spmv", "factor_call", "apply_call"]

# exported symbols that include/javelin.h declares
SYMBOLS = [
    "ilu_analyze", "ilu_analyze_batched", "ilu_levels_device", "ilu_permute_device", "ilu_transpose_device", "ilu_batch_offsets", "ilu_get_info", "ilu_copy_schedule", "ilu_copy_tiles",
    "ilu_copy_tail",
    "ilu_copy_factor_tail",
    "ilu_factor", "ilu_factor_values", "ilu_copy_factor", "ilu_copy_factor_prec", "ilu_apply", "ilu_get_status",
    "ilu_apply_noalloc", "ilu_apply_ex",
    "ilu_apply_adjoint", "ilu_apply_graph_create", "ilu_graph_launch", "ilu_graph_destroy", "ilu_spmv", "ilu_set_values", "ilu_solve_pcg", "ilu_solve_gmres",
    "ilu_set_schedule", "ilu_get_schedule", "ilu_set_tuning", "ilu_get_tuning", "ilu_tune", "ilu_profile_enable", "ilu_profile_read", "ilu_calibrate",
    "ilu_destroy", "ilu_version",
    "ilu_status_str", "ilu_last_error",
]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p)]


class AnalyzeOpts(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("pattern", C.c_int32), ("host_only", C.c_int32),
                ("tile_rows", C.c_int32), ("ordering", C.c_int32), ("tail_min_rows", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_levels", C.c_int32), ("n_ulevels", C.c_int32),
                ("max_row_lu", C.c_int32), ("nnz_a", C.c_int64), ("nnz_lu", C.c_int64),
                ("nnz_b", C.c_int64), ("level_min", C.c_int32), ("level_max", C.c_int32),
                ("level_median", C.c_double), ("batch_count", C.c_int32), ("n_tiles", C.c_int32),
                ("n_utiles", C.c_int32), ("tile_rows", C.c_int32), ("max_tile", C.c_int32),
                ("tail_rows", C.c_int32), ("tail_urows", C.c_int32), ("reserved", C.c_int32 * 1)]


class FactorInfo(C.Structure):
    _fields_ = [("bad_row", C.c_int32), ("bad_row_original", C.c_int32), ("bad_matrix", C.c_int32),
                ("reserved", C.c_int32), ("n_dropped", C.c_int64)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double),
                ("true_relres", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libjavelin.so and declares every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1812_06160_amd.build` "
                           "(or __graft_entry__.build()) first")
    L = C.CDLL(path)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    H = vp
    sig = {
        "ilu_analyze": [C.POINTER(Csr), C.POINTER(AnalyzeOpts), C.POINTER(H)],
        "ilu_analyze_batched": [i32, C.POINTER(Csr), C.POINTER(AnalyzeOpts), C.POINTER(H)],
        "ilu_batch_offsets": [H, vp, vp],
        "ilu_levels_device": [i32, i64, vp, vp, i32, vp, vp, vp, C.POINTER(i32), vp],
        "ilu_permute_device": [i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp],
        "ilu_transpose_device": [i32, i64, vp, vp, vp, vp, vp, vp, vp],
        "ilu_get_info": [H, C.POINTER(Info)],
        "ilu_copy_schedule": [H] + [vp] * 11,
        "ilu_copy_tiles": [H, i32, vp, vp, vp],
        "ilu_copy_tail": [H, i32, vp, vp, vp],
        "ilu_copy_factor_tail": [H, vp, vp, vp, vp, vp, vp],
        "ilu_factor": [H, vp, i32, f64, i32, C.POINTER(FactorInfo), vp],
        "ilu_factor_values": [H, i32, C.POINTER(vp)],
        "ilu_copy_factor": [H, vp, vp],
        "ilu_copy_factor_prec": [H, i32, vp],
        "ilu_apply": [H, vp, vp, i32, i64, i32, i32, i32, vp],
        "ilu_get_status": [H, vp],
        "ilu_apply_noalloc": [H, vp, vp, i32, i64, i32, i32, i32, vp],
        "ilu_apply_ex": [H, vp, vp, vp, vp, i32, i64, i32, vp],
        "ilu_apply_adjoint": [H, vp, vp, vp, vp, vp, vp, i32, i64, vp],
        "ilu_apply_graph_create": [H, vp, vp, i32, i64, i32, i32, i32, C.POINTER(vp)],
        "ilu_graph_launch": [vp, vp],
        "ilu_graph_destroy": [vp],
        "ilu_spmv": [H, f64, vp, f64, vp, i32, i64, i32, vp],
        "ilu_set_values": [H, vp, vp],
        "ilu_solve_pcg": [H, vp, vp, f64, i32, i32, i32, C.POINTER(SolveInfo), vp],
        "ilu_solve_gmres": [H, vp, vp, f64, i32, i32, i32, i32, C.POINTER(SolveInfo), vp],
        "ilu_set_schedule": [H, i32, i32, i32, i32],
        "ilu_get_schedule": [H, vp, vp, vp, vp],
        "ilu_set_tuning": [H, C.c_char_p, i64],
        "ilu_get_tuning": [H, C.c_char_p, C.POINTER(i64)],
        "ilu_tune": [H, vp, i32, vp, i32, vp, vp],
        "ilu_profile_enable": [H, i32, i32],
        "ilu_profile_read": [H, vp, vp],
        "ilu_calibrate": [i64, vp, i32],
        "ilu_destroy": [H],
        "ilu_version": [],
        "ilu_status_str": [i32],
        "ilu_last_error": [C.c_char_p, i32],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_char_p if name in ("ilu_version", "ilu_status_str") else C.c_int32
    _lib = L
    return L


class IluError(RuntimeError):
    def __init__(self, code, where=""):
        msg = ""
        if _lib is not None:
            buf = C.create_string_buffer(512)
            _lib.ilu_last_error(buf, 512)
            msg = buf.value.decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


def check(code, where=""):
    if code != OK:
        raise IluError(code, where)
    return code
