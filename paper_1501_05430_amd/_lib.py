"""ctypes declarations of liblbm.so (include/lbm.h). Argument marshalling only."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_E_INVALID, LBM_E_WORKSPACE, LBM_E_HIP, LBM_E_UNSTABLE, LBM_E_STATE, LBM_E_UNSUPPORTED = range(7)
LBM_F64, LBM_F32, LBM_F32_SHIFTED, LBM_F32_SHIFTED_MIXED = 0, 1, 2, 3
PRECISIONS = {"f64": LBM_F64, "f32": LBM_F32, "f32_shifted": LBM_F32_SHIFTED, "f32_shifted_mixed": LBM_F32_SHIFTED_MIXED}


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32), ("wet_iters", C.c_int32),
        ("check_every", C.c_int32), ("strip_rows", C.c_int32), ("enable_adjoint", C.c_int32),
        ("step_variant", C.c_int32), ("boundary", C.c_int32), ("eos", C.c_int32),
        ("tau", C.c_double), ("G", C.c_double), ("A", C.c_double),
        ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double), ("T_over_Tc", C.c_double),
        ("rho0_shift", C.c_double), ("rho_fp64_below", C.c_double), ("body_force", C.c_double * 2),
        ("pw_theta", C.c_double * 3), ("pw_rho", C.c_double * 2),
        ("mrt_rates", C.c_double * 3), ("kappa", C.c_double),
        ("G_w", C.c_double * 2),
    ]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("checks", C.c_int64), ("nonfinite", C.c_int64), ("psi_clamps", C.c_int64),
                ("ghost_clamps", C.c_int64), ("steps", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("two_step", C.c_int32), ("waves", C.c_int32), ("prefetch", C.c_int32), ("waves2", C.c_int32)]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "lbm_workspace_bytes": (C.c_size_t, [C.POINTER(Params), C.c_int32]),
    "lbm_create": (C.c_int, [C.POINTER(Params), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "lbm_destroy": (C.c_int, [C.c_void_p]),
    "lbm_eos_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_init_droplet": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_double,
                                   C.c_double]),
    "lbm_apply_wetting": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64]),
    "lbm_measure_contact_angle": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_double)]),
    "lbm_mass": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_get_diag": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Diag)]),
    "lbm_get_rho": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "lbm_get_populations": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "lbm_set_populations": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "lbm_state_bytes": (C.c_size_t, [C.c_void_p, C.c_int32]),
    "lbm_get_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lbm_set_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lbm_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "lbm_adjoint_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "lbm_adjoint_step_f32": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "lbm_coexistence": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_step_timed": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)]),
    "lbm_adjoint_seed_rho": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_adjoint_seed_rho_f32": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "lbm_measure_contact_angle_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                                    C.POINTER(C.c_int32), C.c_void_p, C.POINTER(C.c_double)]),
    "lbm_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_last_error": (C.c_char_p, []),
}


def load():
    """Load liblbm.so (built in-tree by __graft_entry__.build()). torch is imported first so the HIP runtime
    it carries is the one the library binds to."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds libamdhip64 before the library is loaded)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code):
    if code != LBM_OK:
        raise LbmError(code, load().lbm_last_error().decode())
