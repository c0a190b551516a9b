"""ctypes binding of libcola (argument marshalling only).

Every function here forwards to the C ABI declared in include/cola.h; all
computation happens in the HIP kernels of libcola.so.  The library must have
been built (``python -m paper_1507_05329_amd.build``); loading fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcola.so")

COLA_OK = 0
COLA_EINVAL = -1
COLA_ENOMEM = -2
COLA_ESTATE = -3
COLA_EUNSUPPORTED = -4
COLA_EHIP = -5
COLA_ENONFINITE = -6
COLA_F_CHECK_FINITE = 1
COLA_F_STAGE_TIMERS = 2
COLA_F_D2_ODE = 4
PASS_PLAIN, PASS_GREEN, PASS_GRAD = 0, 1, 2
STAGES = ["sort", "deposit", "fft_z", "fft_y", "fft_x_green", "ifft_y", "ifft_z", "kick_drift",
          "ifft_y_grad", "velocity"]


class cola_params(C.Structure):
    _fields_ = [("np", C.c_int32), ("nmesh", C.c_int32), ("box", C.c_double),
                ("omega_m", C.c_double), ("n_lpt", C.c_double), ("a_init", C.c_double),
                ("flags", C.c_int32), ("reserved", C.c_int32)]


# name -> (restype, argtypes)
_P = C.c_void_p
_D = C.c_double
_I = C.c_int32
_DP = C.POINTER(C.c_double)
_SIGS = {
    "cola_params_default": (None, [C.POINTER(cola_params), _I, _I, _D]),
    "cola_workspace_query": (C.c_int, [C.POINTER(cola_params), C.POINTER(C.c_size_t)]),
    "cola_create": (C.c_int, [C.POINTER(cola_params), _P, C.c_size_t, _P, C.POINTER(_P)]),
    "cola_destroy": (C.c_int, [_P]),
    "cola_init_2lpt_from_noise": (C.c_int, [_P, _P, _DP, _DP, _I]),
    "cola_init_2lpt": (C.c_int, [_P, C.c_uint64, _DP, _DP, _I, _D, _I]),
    "cola_noise": (C.c_int, [_P, C.c_uint64, _P]),
    "cola_step": (C.c_int, [_P, _D, _D]),
    "cola_density": (C.c_int, [_P, _P]),
    "cola_pk": (C.c_int, [_P, _I, _DP, _I, _DP, _DP, C.POINTER(C.c_int64)]),
    "cola_pk_jing": (C.c_int, [_P, _I, _DP, _I, _DP, _DP, C.POINTER(C.c_int64)]),
    "cola_force": (C.c_int, [_P, _P]),
    "cola_pm_gradient": (C.c_int, [_P, _D, _P, _P, _P, _P]),
    "cola_velocity": (C.c_int, [_P, _P, _P, C.c_int32]),
    "cola_density_of": (C.c_int, [_P, _P, _P]),
    "cola_density_noalloc": (C.c_int, [_P, _I, _I, _P, _P]),
    "cola_snapshot": (C.c_int, [_P, C.c_double, C.c_double, _P, _P, _P, C.c_int32]),
    "cola_fof_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "cola_fof": (C.c_int, [_P, C.c_double, _P, _P, C.c_size_t]),
    "cola_fof_halos_workspace_bytes": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_size_t)]),
    "cola_fof_halos": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.POINTER(C.c_int32), _P, _P, _P, _P, _P,
                                 C.c_size_t]),
    "cola_pk_velocity": (C.c_int, [_P, C.c_int32, _DP, C.c_int32, _DP, _DP, _DP, _DP, C.POINTER(C.c_int64)]),
    "cola_pk_of": (C.c_int, [_P, _P, C.c_int32, _DP, C.c_int32, _DP, _DP, C.POINTER(C.c_int64)]),
    "cola_get_state": (C.c_int, [_P, _P, _P, _P, _P, _DP, _DP]),
    "cola_set_state": (C.c_int, [_P, _P, _P, _P, _P, _D, _D]),
    "cola_fft3d": (C.c_int, [_P, _I, _P, _I]),
    "cola_step_scalars": (C.c_int, [C.POINTER(cola_params), _D, _D, _D, _DP]),
    "cola_stage_times": (C.c_int, [_P, _DP, C.POINTER(C.c_int64)]),
    "cola_step_adjoint": (C.c_int, [_P, _D, _D, _D, _P, _P, _P, _P, _P]),
    "cola_density_adjoint": (C.c_int, [_P, _P, _P, _P]),
    "cola_pk_adjoint": (C.c_int, [_P, _P, _I, _DP, _I, _DP, _P]),
    "cola_init_2lpt_adjoint": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "cola_force_slot_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "cola_step_keep": (C.c_int, [_P, _D, _D, _P]),
    "cola_step_adjoint_kept": (C.c_int, [_P, _D, _D, _D, _P, _P, _P, _P, _P, _P]),
    "cola_synchronize": (C.c_int, [_P]),
    "cola_fft_set_schedule": (C.c_int, [_I, _I, _I]),
    "cola_fft_get_schedule": (C.c_int, [_I, _I, C.POINTER(C.c_int32)]),
    "cola_autotune": (C.c_int, [_P, _I, C.POINTER(C.c_int32), _DP]),
    "cola_batch_workspace_query": (C.c_int, [C.POINTER(cola_params), _I, C.POINTER(C.c_size_t)]),
    "cola_batch_create": (C.c_int, [C.POINTER(cola_params), _I, _P, C.c_size_t, _P, C.POINTER(_P)]),
    "cola_batch_destroy": (C.c_int, [_P]),
    "cola_batch_size": (_I, [_P]),
    "cola_batch_ngroups": (_I, [_P]),
    "cola_batch_mock": (_P, [_P, _I]),
    "cola_batch_set_graph": (C.c_int, [_P, _I]),
    "cola_batch_set_chunk_bytes": (C.c_int, [_P, C.c_size_t]),
    "cola_batch_step": (C.c_int, [_P, _D, _D]),
    "cola_batch_synchronize": (C.c_int, [_P]),
    "cola_batch_last_error": (C.c_char_p, [_P]),
    "cola_strerror": (C.c_char_p, [C.c_int]),
    "cola_last_error": (C.c_char_p, [_P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libcola.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcola.so not built at {path}; run python -m paper_1507_05329_amd.build")
    try:
        import torch  # noqa: F401  (HIP runtime shared with torch)
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


class ColaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def check(code, ctx=None, what="", batch=None):
    if code != COLA_OK:
        lib = load()
        if batch:
            detail = lib.cola_batch_last_error(batch).decode()
        else:
            detail = lib.cola_last_error(ctx).decode() if ctx else ""
        raise ColaError(code, f"{what}: {lib.cola_strerror(code).decode()} {detail}".strip())
    return code


def dptr(arr):
    """Pointer to a contiguous float64 numpy array."""
    return arr.ctypes.data_as(_DP)
