"""ctypes declarations of the C ABI in include/to.h.

Loading fails loudly when the built library is missing: there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtopo_mi355x.so")

TO_OK, TO_E_INVALID, TO_E_OOM, TO_E_HIP, TO_E_NOCONV, TO_E_NONFINITE, TO_E_SINGULAR, TO_E_BUSY = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "TO_OK", -1: "TO_E_INVALID", -2: "TO_E_OOM", -3: "TO_E_HIP",
                -4: "TO_E_NOCONV", -5: "TO_E_NONFINITE", -6: "TO_E_SINGULAR", -7: "TO_E_BUSY"}
BC_CANTILEVER, BC_MBB, BC_CUSTOM, BC_CANTILEVER_CORNERS, BC_MBB_STRIP = 0, 1, 2, 3, 4
PREC_FP64, PREC_FP32_REFINE, PREC_FP32_REFINE_BF16 = 0, 1, 2
FILTER_DENS, FILTER_DENS_T, FILTER_SENS = 0, 1, 2


class ToProblem(ctypes.Structure):
    _fields_ = [
        ("nelx", ctypes.c_int32), ("nely", ctypes.c_int32), ("nelz", ctypes.c_int32),
        ("h", ctypes.c_double), ("E0", ctypes.c_double), ("Emin", ctypes.c_double),
        ("nu", ctypes.c_double), ("penal", ctypes.c_double),
        ("bc", ctypes.c_int32),
        ("fixed_mask", ctypes.POINTER(ctypes.c_uint8)),
        ("load", ctypes.POINTER(ctypes.c_double)),
        ("load_total", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("rtol", ctypes.c_double),
        ("max_iters", ctypes.c_int32),
    ]


class ToSolveInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("ms", ctypes.c_double)]


class ToOcInfo(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("change", ctypes.c_double),
                ("volume", ctypes.c_double), ("bisections", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ToSimpParams(ctypes.Structure):
    _fields_ = [("vf", ctypes.c_double), ("rmin", ctypes.c_double), ("move", ctypes.c_double),
                ("eta", ctypes.c_double), ("change_tol", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("init_uniform", ctypes.c_int32)]


class ToSimpInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("c", ctypes.c_double), ("change", ctypes.c_double), ("volume", ctypes.c_double),
                ("ms", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_D = ctypes.c_double
_SIGS = {
    "to_workspace_size": (ctypes.c_int, [ctypes.POINTER(ToProblem), ctypes.POINTER(ctypes.c_size_t)]),
    "to_create": (ctypes.c_int, [ctypes.POINTER(ToProblem), _P, ctypes.c_size_t, _P,
                                 ctypes.POINTER(_P)]),
    "to_destroy": (None, [_P]),
    "to_last_error": (ctypes.c_char_p, [_P]),
    "to_solve": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(ToSolveInfo)]),
    "to_compliance_sensitivity": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_D), _P]),
    "to_filter": (ctypes.c_int, [_P, _D, ctypes.c_int32, _P, _P, _P]),
    "to_density_to_sdf": (ctypes.c_int, [_P, _P, _D, _P, _P, _P]),
    "to_density_to_sdf_noalloc": (ctypes.c_int, [_P, _P, _D, _P, _P, _P]),
    "to_volume_fraction": (ctypes.c_int, [_P, _P, _P]),
    "to_oc_update": (ctypes.c_int, [_P, _P, _P, _D, _D, _D, _P, ctypes.POINTER(ToOcInfo)]),
    "to_simp": (ctypes.c_int, [_P, ctypes.POINTER(ToSimpParams), _P, _P, _P, _P,
                               ctypes.POINTER(ToSimpInfo)]),
    "to_ls_advect": (ctypes.c_int, [_P, _P, _P, _D, ctypes.c_int32, ctypes.POINTER(_D)]),
    "to_ls_reinit": (ctypes.c_int, [_P, _P, _D, _D, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_D)]),
    "to_shape_rhs": (ctypes.c_int, [_P, _P, _P, _D, _D, _D, _P]),
    "to_hilbert_extend": (ctypes.c_int, [_P, _D, _P, _P, _D, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_D)]),
    "to_matvec": (ctypes.c_int, [_P, _P, _P, _P]),
    "to_matvec_f32": (ctypes.c_int, [_P, _P, _P, _P]),
    "to_last_energy_sum": (_D, [_P]),
    "to_last_triangle_count": (ctypes.c_int32, [_P]),
    "to_profile": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(_D),
                                  ctypes.POINTER(ctypes.c_int64)]),
    "to_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "to_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(ToProblem), _P, _P, ctypes.c_uint64]),
    "to_server_poll": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "to_server_wait_idle": (ctypes.c_int, [_P, _D]),
    "to_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "to_server_last_error": (ctypes.c_char_p, [_P]),
    "to_server_destroy": (None, [_P]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run __graft_entry__.build() "
                               "(or python paper_2605_04735_amd/build.py) first" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
