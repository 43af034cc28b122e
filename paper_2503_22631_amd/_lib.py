"""ctypes declarations of libfab's C ABI (include/fab.h).  Argument marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfab.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fab.h")

c_int32, c_int64, c_uint64, c_double, c_size_t, c_void_p = (
    ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p)

STATUS = {
    0: "FAB_OK", 1: "FAB_OK_BREAKDOWN", 2: "FAB_W_NOT_CONVERGED", 3: "FAB_W_QUADRATURE",
    -1: "FAB_E_INVALID", -2: "FAB_E_UNSUPPORTED", -3: "FAB_E_HIP", -4: "FAB_E_NONFINITE",
    -5: "FAB_E_DIVERGED", -6: "FAB_E_WORKSPACE",
}
EXPORTS = ["fab_create", "fab_destroy", "fab_csr_create", "fab_op_destroy", "fab_op_transpose",
           "fab_op_index_bytes", "fab_op_store_policy", "fab_op_copy_arrays", "fab_workspace_size", "fab_workspace_size_batched", "fab_solve",
           "fab_solve_batched", "fab_workspace_size_ragged", "fab_solve_ragged", "fab_spmv", "fab_sketch_apply", "fab_sketch_apply_noalloc",
           "fab_sketch_table", "fab_cycle_debug", "fab_dot", "fab_batch_group", "fab_divergence_limit", "fab_timing_enable", "fab_timing_read",
           "fab_status_string", "fab_last_error"]


class fab_params(ctypes.Structure):
    _fields_ = [("m", c_int32), ("k", c_int32), ("d", c_int32), ("zeta", c_int32), ("seed", c_uint64),
                ("tol", c_double), ("max_cycles", c_int32), ("method", c_int32), ("n_quad", c_int32),
                ("spec_lo", c_double), ("spec_hi", c_double)]


class fab_info(ctypes.Structure):
    _fields_ = [("status", c_int32), ("cycles", c_int32), ("matvecs", c_int32), ("group", c_int32),
                ("est_rel_update", c_double), ("quad_rule_error", c_double),
                ("kappa_T", c_double), ("err_est", c_double)]


class FabError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = ""
        if status == -3:
            try:
                detail = " [" + load().fab_last_error().decode() + "]"
            except Exception:
                pass
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status_string(status)}){detail}")


_lib = None


def load():
    """Load libfab.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_22631_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "fab_create": ([P(c_void_p), c_void_p], c_int32),
        "fab_destroy": ([c_void_p], c_int32),
        "fab_csr_create": ([c_void_p, c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_int32, P(c_void_p)], c_int32),
        "fab_op_destroy": ([c_void_p], c_int32),
        "fab_op_transpose": ([c_void_p, c_void_p, P(c_void_p)], c_int32),
        "fab_op_index_bytes": ([c_void_p, P(c_int32)], c_int32),
        "fab_op_store_policy": ([c_void_p, c_int32, P(c_int32)], c_int32),
        "fab_op_copy_arrays": ([c_void_p, c_void_p, c_void_p, c_void_p, c_void_p], c_int32),
        "fab_dot": ([c_void_p, c_int64, c_void_p, c_void_p, c_void_p], c_int32),
        "fab_workspace_size": ([c_void_p, P(fab_params), c_int32, P(c_size_t)], c_int32),
        "fab_solve": ([c_void_p, c_void_p, c_int32, P(c_double), c_int32, c_void_p, c_void_p, P(fab_params),
                       c_void_p, c_size_t, P(fab_info)], c_int32),
        "fab_workspace_size_ragged": ([c_int32, P(c_void_p), P(fab_params), c_int32, P(c_size_t)], c_int32),
        "fab_solve_ragged": ([c_void_p, c_int32, P(c_void_p), c_int32, P(c_double), c_int32, P(c_void_p),
                              P(c_void_p), P(fab_params), c_void_p, c_size_t, P(fab_info)], c_int32),
        "fab_workspace_size_batched": ([c_void_p, P(fab_params), c_int32, c_int32, P(c_size_t)], c_int32),
        "fab_solve_batched": ([c_void_p, c_void_p, c_int32, P(c_double), c_int32, c_int32, c_void_p, c_int64,
                               c_void_p, c_int64, P(fab_params), c_void_p, c_size_t, P(fab_info)], c_int32),
        "fab_spmv": ([c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t], c_int32),
        "fab_sketch_apply": ([c_void_p, c_int64, c_int32, c_int32, c_uint64, c_int32, c_void_p, c_void_p,
                              c_void_p, c_size_t], c_int32),
        "fab_sketch_apply_noalloc": ([c_void_p, c_int64, c_int32, c_int32, c_uint64, c_int32, c_void_p, c_void_p],
                                     c_int32),
        "fab_sketch_table": ([c_void_p, c_int64, c_int64, c_int32, c_int32, c_uint64, c_void_p, c_void_p], c_int32),
        "fab_cycle_debug": ([c_void_p, c_void_p, c_void_p, P(fab_params), c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, P(c_double), c_void_p, c_size_t], c_int32),
        "fab_batch_group": ([c_void_p, c_int32], c_int32),
        "fab_divergence_limit": ([c_void_p, c_double], c_int32),
        "fab_timing_enable": ([c_void_p, c_int32], c_int32),
        "fab_timing_read": ([c_void_p, P(c_double), P(c_int64), P(c_double), P(c_int64), P(c_double), P(c_int64)],
                            c_int32),
        "fab_status_string": ([c_int32], ctypes.c_char_p),
        "fab_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def status_string(s: int) -> str:
    try:
        return load().fab_status_string(s).decode()
    except ImportError:
        return STATUS.get(s, str(s))


def check(status: int, where: str, ok=(0, 1, 2, 3)) -> int:
    if status not in ok:
        raise FabError(status, where)
    return status
