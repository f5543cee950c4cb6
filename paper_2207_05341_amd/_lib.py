"""ctypes loader for libqst.so, the gfx950 likelihood-path library.

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqst.so")

QST_OK, QST_ERR_INVALID_ARG, QST_ERR_UNSUPPORTED, QST_ERR_WORKSPACE, QST_ERR_HIP = range(5)
QST_F64, QST_F32, QST_BF16GEMM, QST_F32X6 = 0, 1, 2, 3
QST_OP_STATE_MAP, QST_OP_POVM_PROBS, QST_OP_NLL, QST_OP_NLL_BACKWARD = 0, 1, 2, 3
QST_OP_LIKELIHOOD, QST_OP_GRAD_PRODUCT, QST_OP_FIDELITY, QST_OP_FNN, QST_OP_ABS_MAP = 4, 5, 6, 7, 8
QST_OP_LIKELIHOOD_GRAD = 9
QST_FIDELITY_MAX_RANK = 32
QST_MAX_QUBITS = 13
QST_PREMAP_HERMITIAN, QST_PREMAP_LOWER = 1, 2
QST_STATIC_SCRATCH_BYTES = 16 << 20

#: Every symbol include/qst.h declares, with (restype, argtypes).
_vp, _i64, _sz, _int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t, ctypes.c_int
SIGNATURES = {
    "qst_state_map": (_int, [_int, _int, _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp]),
    "qst_povm_probs": (_int, [_int, _int, _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    "qst_nll": (_int, [_int, _int, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qst_nll_backward": (_int, [_int, _int, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    "qst_likelihood": (_int, [_int, _int, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    "qst_likelihood_fc": (_int, [_int, _int, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz,
                                 _vp]),
    "qst_likelihood_noalloc": (_int, [_int, _int, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    "qst_workspace_bytes_general": (_sz, [_int, _int, _int, _int]),
    "qst_povm_probs_general": (_int, [_int, _int, _vp, _i64, _int, _vp, _vp, _vp, _sz, _vp]),
    "qst_likelihood_general": (_int, [_int, _int, _vp, _i64, _int, _int, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                       _sz, _vp]),
    "qst_grad_product": (_int, [_int, _int, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    "qst_likelihood_grad": (_int, [_int, _int, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    "qst_state_premap": (_int, [_int, _int, _int, _vp, _i64, _vp, _i64, _vp]),
    "qst_abs_map": (_int, [_int, _int, ctypes.c_double, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qst_abs_map_async": (_int, [_int, _int, ctypes.c_double, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _int, _vp, _vp,
                                  _sz, _vp]),
    "qst_fidelity_general_async": (_int, [_int, _int, _vp, _i64, _vp, _i64, _vp, _int, _vp, _vp, _sz, _vp]),
    "qst_abs_map_backward": (_int, [_int, _int, ctypes.c_double, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
    "qst_fnn_forward": (_int, [_int, _int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _sz, _vp]),
    "qst_fnn_backward": (_int, [_int, _int, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qst_rprop_step": (_int, [_i64, _int, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, _vp]),
    "qst_fidelity_lowrank": (_int, [_int, _int, _vp, _i64, _vp, _i64, _int, _vp, _vp, _sz, _vp]),
    "qst_fidelity_classical": (_int, [_int, _int, _vp, _vp, _vp, _vp, _sz, _vp]),
    "qst_fidelity_general": (_int, [_int, _int, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    "qst_workspace_bytes": (_sz, [_int, _int, _int]),
    "qst_status_string": (ctypes.c_char_p, [_int]),
    "qst_last_error": (ctypes.c_char_p, []),
    "qst_version": (ctypes.c_char_p, []),
    "qst_profile_enable": (_int, [_int, ctypes.c_char_p]),
    "qst_profile_report": (_sz, [ctypes.c_char_p, _sz, _int]),
    "qst_batch_plan_create": (_int, [_vp, _int, _int, _vp, ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "qst_batch_offsets": (_int, [_vp, _vp, _vp]),
    "qst_batch_run": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _int, _vp]),
    "qst_batch_info": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double)]),
    "qst_batch_shape": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int)]),
    "qst_batch_plan_destroy": (None, [_vp]),
}

_lib = None


class QstError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {status_string(status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2207_05341_amd.build` "
                "(or __graft_entry__.build()) first.  There is no non-HIP fallback.")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status: int) -> str:
    return lib().qst_status_string(status).decode()


def check(status: int, where: str) -> None:
    if status != QST_OK:
        raise QstError(status, where, lib().qst_last_error().decode())


def workspace_bytes(n: int, prec: int, op: int) -> int:
    return int(lib().qst_workspace_bytes(n, prec, op))


def profile_enable(on: bool, only: str | None = None) -> None:
    """Time every library kernel scope, or only the scope named `only`."""
    check(lib().qst_profile_enable(1 if on else 0, only.encode() if only else None), "qst_profile_enable")


def profile_report(reset: bool = True) -> dict[str, tuple[int, float]]:
    """{kernel name: (calls, total ms)} since the last reset (waits for the
    recorded events)."""
    need = int(lib().qst_profile_report(None, 0, 0))
    buf = ctypes.create_string_buffer(need + 1024)
    lib().qst_profile_report(buf, len(buf), 1 if reset else 0)
    out = {}
    for line in buf.value.decode().splitlines():
        name, calls, ms = line.split()
        out[name] = (int(calls), float(ms))
    return out
