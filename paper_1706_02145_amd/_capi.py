"""ctypes declarations of the C ABI in include/celes.h (argument marshalling
only; all computation happens in libceles_amd.so)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CELES_LIB", os.path.join(HERE, "libceles_amd.so"))

CELES_OK = 0
ERRORS = {
    -1: "CELES_E_ARG", -2: "CELES_E_OVERLAP", -3: "CELES_E_LUT_RANGE", -4: "CELES_E_NONFINITE",
    -5: "CELES_E_NOCONV", -6: "CELES_E_BREAKDOWN", -7: "CELES_E_OOM", -8: "CELES_E_DEVICE",
    -9: "CELES_E_UNSUPPORTED", -10: "CELES_E_STATE",
}
CELES_FP64, CELES_MIXED = 0, 1
CELES_HANKEL_LUT, CELES_HANKEL_DIRECT = 0, 1
CELES_SOLVER_GMRES, CELES_SOLVER_BICGSTAB = 0, 1
CELES_CUBOID_AUTO = -1.0
CELES_TRANSLATION_DIRECT, CELES_TRANSLATION_ROTATE = 0, 1


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("hankel", C.c_int), ("lut_dr", C.c_double), ("tol", C.c_double),
                ("inner_tol", C.c_double), ("restart", C.c_int), ("maxiter", C.c_int),
                ("max_refinements", C.c_int), ("cuboid_edge", C.c_double), ("device", C.c_int),
                ("verbose", C.c_int), ("solver", C.c_int), ("target_Nj", C.c_double),
                ("mem_cap_bytes", C.c_double), ("autotune", C.c_int), ("translation", C.c_int),
                ("deterministic", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("refinements", C.c_int), ("matvecs", C.c_int),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("matvec_seconds", C.c_double),
                ("x0_used", C.c_int), ("x0_residual", C.c_double)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_vp = C.c_void_p
_h = C.c_void_p

SIGNATURES = {
    "celes_default_options": (None, [C.POINTER(Options)]),
    "celes_version": (C.c_int, []),
    "celes_last_error": (C.c_char_p, [_h]),
    "celes_create": (C.c_int, [C.POINTER(_h), C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int,
                               C.POINTER(Options)]),
    "celes_destroy": (None, [_h]),
    "celes_set_solve_options": (C.c_int, [_h, C.POINTER(Options)]),
    "celes_set_plane_waves": (C.c_int, [_h, C.c_int, _dp, _dp, _ip, _dp]),
    "celes_set_gaussian_beam": (C.c_int, [_h, C.c_double, _dp, C.c_double, C.c_double, C.c_double, C.c_int]),
    "celes_get_incident": (C.c_int, [_h, _dp]),
    "celes_num_rhs": (C.c_int, [_h]),
    "celes_build_preconditioner": (C.c_int, [_h, C.c_double]),
    "celes_plan_preconditioner": (C.c_int, [C.c_int64, _dp, C.c_int, C.c_double, C.c_double, _dp,
                                            C.POINTER(C.c_int64), _dp, C.POINTER(C.c_int64)]),
    "celes_preconditioner_info": (C.c_int, [_h, _dp, C.POINTER(C.c_int64), _dp]),
    "celes_solve": (C.c_int, [_h, _dp, _dp, C.POINTER(SolveInfo)]),
    "celes_apply_preconditioner": (C.c_int, [_h, C.c_int, C.c_int, _vp, _vp, _vp]),
    "celes_s11": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, _dp, C.c_int, _dp]),
    "celes_subsystem_guess": (C.c_int, [_h, C.c_int64, C.POINTER(C.c_int64), C.c_double, _dp, C.POINTER(SolveInfo)]),
    "celes_apply_W": (C.c_int, [_h, C.c_int, C.c_int, _vp, _vp, _vp]),
    "celes_apply_M": (C.c_int, [_h, C.c_int, C.c_int, _vp, _vp, _vp]),
    "celes_apply_W_noalloc": (C.c_int, [_h, C.c_int, C.c_int, _vp, _vp, _vp]),
    "celes_cross_sections": (C.c_int, [_h, _dp, _dp, _dp]),
    "celes_far_field": (C.c_int, [_h, C.c_int64, _dp, _dp, _dp]),
    "celes_near_field": (C.c_int, [_h, C.c_int64, _dp, C.c_int, _dp]),
    "celes_mie_coefficients": (C.c_int, [C.c_int, C.c_double, C.c_double, C.c_double, _dp]),
    "celes_lut_info": (C.c_int, [_h, _dp, _dp, C.POINTER(C.c_int64)]),
    "celes_kernel_timing": (C.c_int, [_h, C.c_int, _dp, C.POINTER(C.c_int)]),
    "celes_power_flux": (C.c_int, [_h, C.c_int, C.c_int, _dp]),
    "celes_dims": (C.c_int, [_h, C.POINTER(C.c_int64), _ip, _ip]),
    "celes_translation_tables": (C.c_int, [C.c_int, _dp, _dp]),
    "celes_get_solution": (C.c_int, [_h, _dp]),
    "celes_batch_create": (C.c_int, [C.POINTER(_h), C.c_int, C.POINTER(_h), C.POINTER(Options)]),
    "celes_batch_destroy": (None, [_h]),
    "celes_batch_num_systems": (C.c_int, [_h]),
    "celes_batch_last_error": (C.c_char_p, [_h]),
    "celes_batch_apply_M": (C.c_int, [_h, C.c_int, _vp, _vp, _vp]),
    "celes_batch_autotune": (C.c_int, [_h, C.c_int, _dp, _ip, _ip]),
    "celes_batch_solve": (C.c_int, [_h, C.POINTER(SolveInfo), C.POINTER(SolveInfo)]),
    "celes_nn_create": (C.c_int, [C.POINTER(_h), C.c_int, C.c_uint64]),
    "celes_nn_destroy": (None, [_h]),
    "celes_nn_last_error": (C.c_char_p, [_h]),
    "celes_nn_dims": (C.c_int, [_h, _ip, _ip, _ip, _ip, _ip, C.POINTER(C.c_int64)]),
    "celes_nn_get_params": (C.c_int, [_h, C.POINTER(C.c_float)]),
    "celes_nn_set_params": (C.c_int, [_h, C.POINTER(C.c_float)]),
    "celes_nn_features": (C.c_int, [_h, _h, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "celes_nn_loss_grad": (C.c_int, [_h, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float), _dp,
                                     C.POINTER(C.c_float)]),
    "celes_nn_forward": (C.c_int, [_h, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "celes_nn_add_training_problem": (C.c_int, [_h, _h]),
    "celes_nn_train": (C.c_int, [_h, C.c_int, C.c_int, C.c_double, C.c_uint64, _dp]),
    "celes_nn_predict": (C.c_int, [_h, _h, _dp]),
}

_lib = None


def lib():
    """Load libceles_amd.so (raises if it has not been built: there is no
    fallback implementation)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_1706_02145_amd.build`")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib
