"""ctypes binding of libppq.so (include/ppq.h): argument marshalling only.

Every entry point keeps the C name.  There is no fallback: if the library is
missing or cannot be loaded, importing a function raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppq.so")

PPQ_OK = 0
STATUS = {0: "PPQ_OK", -1: "PPQ_E_ARG", -2: "PPQ_E_STATE", -3: "PPQ_E_OOM", -4: "PPQ_E_CAPACITY",
          -5: "PPQ_E_HIP", -6: "PPQ_E_NUMERIC", -7: "PPQ_E_UNSUPPORTED"}
PPQ_FP64, PPQ_FP32 = 0, 1
PPQ_FAC_POWER, PPQ_FAC_MORSE, PPQ_FAC_TABLE, PPQ_FAC_MORSE_DA = 0, 1, 2, 3
PPQ_FAC_DENSE_REAL, PPQ_FAC_DENSE_COMPLEX = 4, 5
OBS_FIELDS = ("t", "norm2", "energy", "acf_re", "acf_im", "n_active", "n_above", "krylov_used", "substeps")
OBS_N = 9
PHASES = ("hpsi", "krylov", "adapt", "tables", "obs")  # ppq_timings order

# every exported symbol and its (restype, argtypes)
_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "ppq_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp, ctypes.c_int]),
    "ppq_destroy": (None, [_vp]),
    "ppq_last_error": (ctypes.c_char_p, [_vp]),
    "ppq_set_grid": (ctypes.c_int, [_vp, ctypes.c_int, _i32p, _dp, _dp, ctypes.c_double]),
    "ppq_get_grid": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "ppq_set_lattice": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ppq_add_potential_term": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int, _i32p, _i32p, _dp, _dp]),
    "ppq_add_term": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _i32p, _i32p, _dp, _dp]),
    "ppq_reserve": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "ppq_init_gaussian": (ctypes.c_int, [_vp, _dp, _dp, _dp, ctypes.c_double, _i64p]),
    "ppq_set_state": (ctypes.c_int, [_vp, ctypes.c_int64, _u64p, _dp]),
    "ppq_active_count": (ctypes.c_int, [_vp, _i64p]),
    "ppq_get_state": (ctypes.c_int, [_vp, ctypes.c_int64, _i64p, _u64p, _dp]),
    "ppq_apply_h": (ctypes.c_int, [_vp, _vp, _vp]),
    "ppq_step": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int]),
    "ppq_prune": (ctypes.c_int, [_vp, ctypes.c_double, _i64p, _i64p]),
    "ppq_set_reference": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "ppq_clear_potential": (ctypes.c_int, [_vp]),
    "ppq_set_factor": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "ppq_set_stencil": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ppq_set_weylets": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ppq_set_fgh": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ppq_set_state_device": (ctypes.c_int, [_vp, ctypes.c_int64, _vp, _vp]),
    "ppq_get_state_device": (ctypes.c_int, [_vp, ctypes.c_int64, _i64p, _vp, _vp]),
    "ppq_set_relative_exclusion": (ctypes.c_int, [_vp, ctypes.c_double]),
    "ppq_set_krylov_tolerance": (ctypes.c_int, [_vp, ctypes.c_double]),
    "ppq_set_step_control": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ppq_propagate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp]),
    "ppq_observables": (ctypes.c_int, [_vp, ctypes.c_double, _dp]),
    "ppq_expect_q": (ctypes.c_int, [_vp, _dp]),
    "ppq_expect_q_noalloc": (ctypes.c_int, [_vp, _dp]),
    "ppq_acf_doubled": (ctypes.c_int, [_vp, _dp]),
    "ppq_set_potential_term": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, _dp]),
    "ppq_add_potential_derivative": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _i32p, _i32p,
                                                    _dp, _dp]),
    "ppq_adjoint_record": (ctypes.c_int, [_vp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_int, _dp]),
    "ppq_adjoint_frozen": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "ppq_adjoint_gradient": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "ppq_time_apply": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "ppq_fiber_counts": (ctypes.c_int, [_vp, _i64p]),
    "ppq_enable_timings": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ppq_timings": (ctypes.c_int, [_vp, _dp]),
}

_LIB = None


def load():
    """Loads libppq.so (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "or python -m paper_1606_04004_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


class PPQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(ctx, code):
    if code != PPQ_OK:
        msg = load().ppq_last_error(ctx).decode(errors="replace") if ctx else ""
        raise PPQError(code, msg)
    return code
