"""ctypes loader for libslista.so (the C ABI declared in include/slista.h).

torch is imported first on purpose: torch ships its own HIP runtime
(libamdhip64.so.7), and loading it before libslista makes the library bind
to that same runtime (same SONAME), so device pointers and streams coming
from torch are valid inside the library.

There is no fallback: if the library is missing or fails to load, this
module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL load, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslista.so")

# Every symbol include/slista.h declares, with its C signature.
_c_int, _c_float, _c_double, _vp = ctypes.c_int, ctypes.c_float, ctypes.c_double, ctypes.c_void_p
_size_t = ctypes.c_size_t
SIGNATURES = {
    "slista_abi_version": (_c_int, []),
    "slista_status_string": (ctypes.c_char_p, [_c_int]),
    "slista_last_error": (ctypes.c_char_p, []),
    "slista_dict_create": (_c_int, [_vp, _c_int, _c_int, _vp, ctypes.POINTER(_vp)]),
    "slista_dict_destroy": (_c_int, [_vp]),
    "slista_dict_dims": (_c_int, [_vp, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)]),
    "slista_dict_gram": (_c_int, [_vp, _vp, _vp]),
    "slista_dict_lipschitz": (_c_int, [_vp, _c_int, _c_double, ctypes.POINTER(_c_double),
                                       ctypes.POINTER(_c_int), _vp]),
    "slista_workspace_size": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_size_t)]),
    "slista_forward": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _c_int, _c_int, _vp, _vp, _c_int, _vp,
                                _c_int, _vp, _size_t, _vp]),
    "slista_objective": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _vp, _vp]),
    "slista_forward_scratch": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _c_int, _c_int, _vp, _vp, _c_int, _vp,
                                        _vp]),
    "slista_backward": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _c_int, _c_int, _vp, _vp, _vp, _c_int,
                                 _vp, _size_t, _vp]),
    "slista_forward_backward": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _c_int, _c_int, _vp, _vp, _vp,
                                         _vp, _c_int, _vp, _size_t, _vp]),
    "slista_set_option": (_c_int, [_c_int, _c_int]),
    "slista_autotune": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _c_int, _c_int, _c_int, _vp, _vp, _vp, _size_t, _vp,
                                 ctypes.POINTER(_c_int), ctypes.POINTER(_c_double)]),
    "slista_batch_autotune": (_c_int, [_vp, _vp, ctypes.POINTER(_c_int)]),
    "slista_ckpt_for_budget": (_c_int, [_vp, _c_int, _c_int, _c_int, _size_t, ctypes.POINTER(_c_int),
                                        ctypes.POINTER(_size_t)]),
    "slista_oista_workspace_size": (_c_int, [_vp, _c_int, _c_int, _c_int, ctypes.POINTER(_size_t)]),
    "slista_oista": (_c_int, [_vp, _vp, _c_int, _c_float, _c_double, _c_int, _c_int, _c_int, _c_double, _vp, _vp,
                              _vp, _vp, _vp, _size_t, _vp]),
    "slista_fista_workspace_size": (_c_int, [_vp, _c_int, _c_int, _c_int, ctypes.POINTER(_size_t)]),
    "slista_fista": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _c_int, _c_int, _vp, _vp, _vp, _vp, _size_t, _vp]),
    "slista_train_workspace_size": (_c_int, [_vp, _c_int, _c_int, _c_int, ctypes.POINTER(_size_t)]),
    "slista_train": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _c_int, _c_int, _c_int, _c_double, _c_int, _vp,
                              ctypes.POINTER(_c_double), ctypes.POINTER(_c_int), ctypes.POINTER(_c_double), _vp,
                              _size_t, _vp]),
    "slista_lista_workspace_size": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_size_t)]),
    "slista_lista_forward": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _vp, _vp, _c_int, _c_int, _vp, _vp, _vp,
                                      _c_int, _vp, _size_t, _vp]),
    "slista_lista_backward": (_c_int, [_vp, _c_int, _c_float, _vp, _vp, _c_int, _c_int, _vp, _vp, _vp, _vp, _vp,
                                       _vp, _size_t, _vp]),
    "slista_lista_forward_backward": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _vp, _vp, _c_int, _c_int, _vp, _vp,
                                               _vp, _vp, _vp, _vp, _vp, _size_t, _vp]),
    "slista_tune_save": (_c_int, [ctypes.c_char_p]),
    "slista_tune_load": (_c_int, [ctypes.c_char_p]),
    "slista_batch_create": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_vp)]),
    "slista_batch_workspace_size": (_c_int, [_vp, ctypes.POINTER(_size_t)]),
    "slista_batch_bind": (_c_int, [_vp, _vp, _size_t, _vp]),
    "slista_batch_run": (_c_int, [_vp, _vp]),
    "slista_batch_capture": (_c_int, [_vp, _vp]),
    "slista_batch_replay": (_c_int, [_vp, _vp]),
    "slista_batch_destroy": (_c_int, [_vp]),
    "slista_kkt": (_c_int, [_vp, _vp, _c_int, _c_float, _vp, _vp, _vp, _vp]),
    "slista_forward_f64_workspace_size": (_c_int, [_vp, _c_int, ctypes.POINTER(_size_t)]),
    "slista_forward_f64": (_c_int, [_vp, _vp, _c_int, _c_double, _vp, _c_int, _vp, _vp, _c_int, _vp, _vp,
                                    _size_t, _vp]),
    "slista_lambda_max_workspace_size": (_c_int, [_vp, _c_int, ctypes.POINTER(_size_t)]),
    "slista_lambda_max": (_c_int, [_vp, _vp, _c_int, _vp, _vp, _vp, _size_t, _vp]),
    "slista_batched_workspace_size": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_size_t)]),
    "slista_batched_fwd_bwd": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, _vp, _size_t, _vp, _c_int]),
    "slista_batched_release": (_c_int, []),
    "slista_profile_begin": (_c_int, []),
    "slista_profile_end": (_c_int, [ctypes.POINTER(_c_int), ctypes.POINTER(_c_double), ctypes.POINTER(_c_int)]),
}

PROFILE_KINDS = ["correlation", "forward_layer", "objective", "backward_seed", "backward_layer", "elementwise"]

class Problem(ctypes.Structure):
    """C layout of slista_problem."""
    _fields_ = [("dict", ctypes.c_void_p), ("X", ctypes.c_void_p), ("N", ctypes.c_int), ("lam", ctypes.c_float),
                ("alpha", ctypes.c_void_p), ("Z", ctypes.c_void_p), ("F", ctypes.c_void_p),
                ("loss", ctypes.c_void_p), ("dalpha", ctypes.c_void_p)]


STATUS = {0: "SLISTA_OK", -1: "SLISTA_EINVAL", -2: "SLISTA_ENOMEM", -3: "SLISTA_EHIP",
          -4: "SLISTA_ENOTSUP", -5: "SLISTA_ENOTCONV", -6: "SLISTA_ENONFINITE"}


class SlistaError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (loaded once). Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1905_11071_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def check(status: int) -> None:
    if status != 0:
        raise SlistaError(status, lib().slista_last_error().decode(errors="replace"))
