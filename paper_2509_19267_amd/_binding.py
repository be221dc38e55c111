"""ctypes binding of librgdbek.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch supplies device memory
(tensors on a HIP device) and the stream.  Loading fails loudly when the
library has not been built: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "librgdbek.so")

# status codes (include/rgdbek.h)
OK, ERR_INVALID_ARG, ERR_NUMERIC, ERR_NOT_CONVERGED, ERR_OUT_OF_MEMORY, \
    ERR_DEVICE, ERR_UNSUPPORTED = range(7)
DENSE_ROW_MAJOR, CSR = 0, 1
F64, F32 = 0, 1
STOP_NONE, STOP_ERR_REF, STOP_RSE, STOP_RES_EXT = 0, 1, 2, 3
PREC_FP64, PREC_MIXED_F32 = 0, 1
SOLVER_AUTO, SOLVER_CHOL, SOLVER_CG = 0, 1, 2
FLAG_GRAPH, FLAG_GRAM_AAT, FLAG_CG_SPLIT, FLAG_SPARSE_CG, FLAG_PROFILE, \
    FLAG_SPARSE_FULL = 1, 2, 4, 8, 16, 32
PROF_REGIONS = ["col_residual", "col_draw", "col_solve", "col_update",
                "row_residual", "row_draw", "row_solve", "row_update",
                "stop", "refine"]
SELECT_RANDOM, SELECT_GREEDY, SELECT_BLOCK_LAW, SELECT_IID = 0, 1, 2, 3

STOP_NAMES = {"none": STOP_NONE, "err_ref": STOP_ERR_REF, "rse": STOP_RSE,
              "res_ext": STOP_RES_EXT}
PREC_NAMES = {"fp64": PREC_FP64, "mixed_f32": PREC_MIXED_F32}


class Matrix(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("layout", ctypes.c_int32),
                ("value_type", ctypes.c_int32), ("values", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("k_col", ctypes.c_int64), ("k_row", ctypes.c_int64),
                ("eta", ctypes.c_double), ("tol", ctypes.c_double),
                ("stop", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_iter", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("inner_max", ctypes.c_int32), ("graph_iters", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("solver", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("weight_floor", ctypes.c_double),
                ("tile_rows", ctypes.c_int32), ("select_mode", ctypes.c_int32),
                ("pass_drop", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64),
                ("outer_iterations", ctypes.c_int64),
                ("final_metric", ctypes.c_double),
                ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
SIGNATURES = {
    "rgdbek_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "rgdbek_create": (ctypes.c_int, [ctypes.POINTER(Matrix),
                                     ctypes.POINTER(Params), _vp,
                                     ctypes.POINTER(_vp)]),
    "rgdbek_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(Info)]),
    "rgdbek_solve_resume": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int64,
                                           _vp, ctypes.POINTER(Info)]),
    "rgdbek_get_z": (ctypes.c_int, [_vp, _vp]),
    "rgdbek_solve_adjoint": (ctypes.c_int, [_vp, _vp, _vp,
                                            ctypes.POINTER(Info)]),
    "rgdbek_grad_pattern": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "rgdbek_select": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32, _vp,
                                     ctypes.POINTER(ctypes.c_int64), _vp]),
    "rgdbek_select_noalloc": (ctypes.c_int, [_vp, ctypes.c_int64,
                                             ctypes.c_int64, ctypes.c_double,
                                             ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.c_uint32,
                                             ctypes.c_uint32, _vp,
                                             ctypes.POINTER(ctypes.c_int64),
                                             _vp]),
    "rgdbek_select_block_law": (ctypes.c_int, [_vp, ctypes.c_int64,
                                               ctypes.c_int64, ctypes.c_double,
                                               ctypes.c_uint64, ctypes.c_uint64,
                                               ctypes.c_uint64, ctypes.c_uint32,
                                               ctypes.c_uint32, _vp,
                                               ctypes.POINTER(ctypes.c_int64),
                                               _vp]),
    "rgdbek_select_iid": (ctypes.c_int, [_vp, ctypes.c_int64,
                                               ctypes.c_int64, ctypes.c_double,
                                               ctypes.c_uint64, ctypes.c_uint64,
                                               ctypes.c_uint64, ctypes.c_uint32,
                                               ctypes.c_uint32, _vp,
                                               ctypes.POINTER(ctypes.c_int64),
                                               _vp]),
    "rgdbek_select_threshold": (ctypes.c_int, [_vp, ctypes.c_int64,
                                               ctypes.c_double, ctypes.c_int64,
                                               _vp, ctypes.POINTER(ctypes.c_int64),
                                               _vp]),
    "rgdbek_apply": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "rgdbek_create_batched": (ctypes.c_int, [ctypes.POINTER(Matrix),
                                             ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(Params), _vp,
                                             ctypes.POINTER(_vp)]),
    "rgdbek_create_multirhs": (ctypes.c_int, [ctypes.POINTER(Matrix),
                                              ctypes.c_int64,
                                              ctypes.POINTER(Params), _vp,
                                              ctypes.POINTER(_vp)]),
    "rgdbek_batch_info": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int32)]),
    "rgdbek_profile_read": (ctypes.c_int, [_vp, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "rgdbek_destroy": (ctypes.c_int, [_vp]),
    "rgdbek_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rgdbek_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


def load():
    """Load librgdbek.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built: run paper_2509_19267_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class RgdbekError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__(f"[{status}] {message}")


def check(status, handle=None, allow=()):
    if status == OK or status in allow:
        return status
    lib = load()
    msg = lib.rgdbek_last_error(handle)
    msg = msg.decode() if msg else ""
    what = lib.rgdbek_status_string(status).decode()
    raise RgdbekError(status, f"{what}: {msg}")
