"""ctypes loader for libomm.so: declares the prototype of every C-ABI entry point."""

from __future__ import annotations

import ctypes as ct
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libomm.so"

_c_double_p = ct.POINTER(ct.c_double)
_c_int_p = ct.POINTER(ct.c_int)
_c_i64_p = ct.POINTER(ct.c_int64)
_vp = ct.c_void_p

# name -> (restype, argtypes); pointers to FP64 data are passed as void* (host or device address).
PROTOTYPES = {
    "omm_create": (ct.c_int, [ct.c_int64, ct.c_int64, ct.POINTER(_vp)]),
    "omm_destroy": (ct.c_int, [_vp]),
    "omm_set_precision": (ct.c_int, [_vp, ct.c_int, ct.c_int]),
    "omm_set_mixed_tol": (ct.c_int, [_vp, ct.c_double]),
    "omm_set_resync": (ct.c_int, [_vp, ct.c_int]),
    "omm_set_flavour": (ct.c_int, [_vp, ct.c_int]),
    "omm_set_sparse": (ct.c_int, [_vp, ct.c_int]),
    "omm_create_complex": (ct.c_int, [ct.c_int64, ct.c_int64, ct.POINTER(_vp)]),
    "omm_set_HS_complex": (ct.c_int, [_vp, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                      _c_double_p, _c_double_p]),
    "omm_minimize_complex": (ct.c_int, [_vp, _c_double_p, _c_double_p, ct.c_double, ct.c_double,
                                        ct.c_double, ct.c_int]),
    "omm_density_complex": (ct.c_int, [_vp, _c_double_p, _c_double_p]),
    "omm_batch_create_complex": (ct.c_int, [ct.c_int, _c_i64_p, _c_i64_p, ct.POINTER(_vp)]),
    "omm_batch_set_HS_complex": (ct.c_int, [_vp, ct.c_int, _c_double_p, _c_double_p,
                                            _c_double_p, _c_double_p, _c_double_p, _c_double_p]),
    "omm_batch_minimize_complex": (ct.c_int, [_vp, ct.POINTER(_vp), ct.POINTER(_vp), _c_double_p,
                                              _c_double_p, ct.c_double, ct.c_int]),
    "omm_sparse_density": (ct.c_int, [_vp, _c_double_p]),
    "omm_checkpoints": (ct.c_int, [_vp, _c_int_p, _c_double_p, ct.c_int, _c_int_p]),
    "omm_set_stream": (ct.c_int, [_vp, _vp]),
    "omm_set_HS": (ct.c_int, [_vp, _vp, _vp, _vp]),
    "omm_set_HS_device": (ct.c_int, [_vp, _vp, _vp, _vp]),
    "omm_minimize": (ct.c_int, [_vp, _vp, ct.c_double, ct.c_double, ct.c_double, ct.c_int]),
    "omm_minimize_device": (ct.c_int, [_vp, _vp, ct.c_double, ct.c_double, ct.c_double, ct.c_int]),
    "omm_iterate": (ct.c_int, [_vp, ct.c_int, ct.c_double]),
    "omm_set_profiling": (ct.c_int, [_vp, ct.c_int]),
    "omm_stage_times": (ct.c_int, [_vp, _c_double_p, ct.c_int, _c_int_p]),
    "omm_energy": (ct.c_int, [_vp, _c_double_p]),
    "omm_density": (ct.c_int, [_vp, _vp]),
    "omm_density_device": (ct.c_int, [_vp, _vp]),
    "omm_edm": (ct.c_int, [_vp, _vp]),
    "omm_edm_device": (ct.c_int, [_vp, _vp]),
    "omm_backward_device": (ct.c_int, [_vp, ct.c_double, _vp, _vp]),
    "omm_backward_device_noalloc": (ct.c_int, [_vp, ct.c_double, _vp, _vp]),
    "omm_get_C": (ct.c_int, [_vp, _vp]),
    "omm_get_subspace": (ct.c_int, [_vp, _vp, _vp]),
    "omm_get_preconditioner": (ct.c_int, [_vp, _vp]),
    "omm_stats": (ct.c_int, [_vp, _c_int_p, _c_double_p]),
    "omm_phase_stats": (ct.c_int, [_vp, _c_int_p, _c_int_p]),
    "omm_energy_trace": (ct.c_int, [_vp, _c_double_p, ct.c_int, _c_int_p]),
    "omm_last_error": (ct.c_char_p, [_vp]),
    "omm_batch_create": (ct.c_int, [ct.c_int, _c_i64_p, _c_i64_p, ct.POINTER(_vp)]),
    "omm_batch_destroy": (ct.c_int, [_vp]),
    "omm_batch_set_HS": (ct.c_int, [_vp, ct.c_int, _vp, _vp, _vp]),
    "omm_batch_set_HS_device": (ct.c_int, [_vp, ct.c_int, _vp, _vp, _vp]),
    "omm_batch_minimize": (ct.c_int, [_vp, ct.POINTER(_vp), _c_double_p, _c_double_p,
                                      ct.c_double, ct.c_int]),
    "omm_batch_energy": (ct.c_int, [_vp, _c_double_p]),
    "omm_batch_iterations": (ct.c_int, [_vp, _c_int_p]),
    "omm_batch_get_C": (ct.c_int, [_vp, ct.c_int, _vp]),
    "omm_batch_last_error": (ct.c_char_p, [_vp]),
    "omm_batch_set_precision": (ct.c_int, [_vp, ct.c_int, ct.c_int]),
    "omm_batch_set_mixed_tol": (ct.c_int, [_vp, ct.c_double]),
    "omm_batch_phase_iterations": (ct.c_int, [_vp, _c_int_p, _c_int_p]),
}

_lib = None


def lib() -> ct.CDLL:
    """The loaded library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(
                f"{LIB_PATH} is not built: run `python -m paper_1312_1549_amd.build` "
                "(the OMM path runs only in its HIP kernels)")
        L = ct.CDLL(str(LIB_PATH))
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
