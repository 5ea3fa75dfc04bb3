"""ctypes binding of libqva.so (the C ABI declared in include/qva.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Importing this module loads the in-tree library and
fails loudly when it has not been built.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqva.so")

QVA_OK = 0
QVA_ERR_ARG = -1
QVA_ERR_SIZE = -2
QVA_ERR_ALIGN = -3
QVA_ERR_WORKSPACE = -4
QVA_ERR_HIP = -5
QVA_ERR_UNSUPPORTED = -6
QVA_ERR_SCRATCH = -7

QVA_MIX_X = 0
QVA_MIX_CIRCULANT = 1
QVA_MIX_XY = 2
QVA_LAMBDA_ARRAY = 0
QVA_LAMBDA_RING = 1
QVA_LAMBDA_COMPLETE = 2
QVA_MAX_QUBITS = 33
QVA_MAX_TERMS = 1024
QVA_MAX_XY_PAIRS = 256
QVA_EVOLVE_SKIP_FINAL_STATE = 1
QVA_STATIC_SCRATCH_BYTES = 16 << 20


class QvaProblem(ctypes.Structure):
    _fields_ = [
        ("mixer", ctypes.c_int),
        ("n_qubits", ctypes.c_int),
        ("q", ctypes.c_void_p),
        ("lam", ctypes.c_void_p),
        ("lambda_kind", ctypes.c_int),
        ("n_states", ctypes.c_int64),
        ("terms", ctypes.c_void_p),
        ("n_terms", ctypes.c_int),
        ("xy_pairs", ctypes.c_void_p),
        ("n_xy_pairs", ctypes.c_int),
        ("q_tiles", ctypes.c_void_p),
        ("q_tiles_key", ctypes.c_uint64),
    ]


class QvaPassInfo(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("group_first", ctypes.c_int),
        ("group_bits", ctypes.c_int),
        ("col_bits", ctypes.c_int),
        ("mix_layer", ctypes.c_int),
        ("mix_layer2", ctypes.c_int),
        ("phase_layer", ctypes.c_int),
        ("bytes", ctypes.c_double),
    ]


PASS_KINDS = {0: "whole", 1: "first", 2: "middle", 3: "boundary", 4: "last", 5: "last_store",
              6: "init", 7: "expect", 8: "reduce", 9: "fft_first", 10: "fft_dif", 11: "fft_lowdiag",
              12: "fft_dit", 13: "fft_boundary", 14: "fft_last", 15: "fft_last_store",
              16: "lambda_prep", 17: "grad_whole", 18: "grad_turn", 19: "grad_mid",
              20: "grad_bound", 21: "grad_final", 22: "grad_dif", 23: "grad_dit",
              24: "grad_lowdiag", 25: "grad_reduce", 26: "cpl_first", 27: "cpl_layer",
              28: "cpl_last", 29: "cpl_last_store", 30: "cpl_sum", 31: "grad_cpl_turn",
              32: "grad_cpl_back", 33: "grad_cpl_sum", 34: "blu_chirp", 35: "blu_tile",
              36: "blu_first", 37: "blu_mul", 38: "blu_lambda", 39: "blu_phase", 40: "blu_last",
              41: "blu_last_store", 42: "xy", 43: "xy_last", 44: "xy_turn", 45: "grad_xy",
              46: "grad_blu_turn", 47: "grad_blu_lambda", 48: "grad_blu_phase", 49: "grad_blu_final",
              50: "grad_zslot", 51: "twiddle_prep", 52: "mr_tables", 53: "mr_first", 54: "mr_dif",
              55: "mr_dit", 56: "mr_lowdiag", 57: "mr_boundary", 58: "mr_last", 59: "mr_last_store",
              60: "mr_small", 61: "grad_mr_turn", 62: "grad_mr_dif", 63: "grad_mr_dit",
              64: "grad_mr_lowdiag", 65: "grad_mr_bound", 66: "grad_mr_final", 67: "grad_mr_small"}


class QvaBatchItem(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_int),
        ("p", ctypes.c_int),
        ("q", ctypes.c_void_p),
        ("gammas", ctypes.c_void_p),
        ("ts", ctypes.c_void_p),
        ("psi", ctypes.c_void_p),
        ("chi", ctypes.c_void_p),
        ("out_f", ctypes.c_void_p),
        ("dgammas", ctypes.c_void_p),
        ("dts", ctypes.c_void_p),
    ]


QVA_BATCH_ALIGN_START = 0
QVA_BATCH_ALIGN_END = 1
QVA_BATCH_ALIGN_SPREAD = 2
QVA_BATCH_MAX_DEPTH = 64
QVA_BATCH_MAX_LANES = 8


class QvaError(RuntimeError):
    def __init__(self, fn: str, status: int, text: str):
        super().__init__(f"{fn}: {text} (status {status})")
        self.status = status


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_I = ctypes.c_int
_SZ = ctypes.c_size_t
_PROB = ctypes.POINTER(QvaProblem)

# name -> (restype, argtypes); one entry per function declared in include/qva.h
SIGNATURES = {
    "qva_status_string": (ctypes.c_char_p, [_I]),
    "qva_version": (ctypes.c_char_p, []),
    "qva_set_group_split": (_I, [_I, ctypes.POINTER(ctypes.c_int), _I]),
    "qva_get_group_split": (_I, [_I, ctypes.POINTER(ctypes.c_int), _I]),
    "qva_parity_ring_pairs": (_I, [ctypes.POINTER(ctypes.c_int), _I, ctypes.POINTER(ctypes.c_int), _I]),
    "qva_init_uniform": (_I, [_P, _I64, _P]),
    "qva_phase": (_I, [_P, _P, _I64, _D, _P]),
    "qva_mix_x": (_I, [_P, _I, _D, _P]),
    "qva_mix_circulant": (_I, [_P, _P, _I, _I64, _D, _P, _SZ, _P]),
    "qva_mix_circulant_workspace_bytes": (_SZ, [_I64]),
    "qva_workspace_bytes": (_SZ, [_PROB, _I, _I]),
    "qva_q_tiles_bytes": (_SZ, [_PROB]),
    "qva_q_tiles": (_I, [_PROB, _P, _SZ, ctypes.POINTER(ctypes.c_uint64), _P]),
    "qva_expectation_workspace_bytes": (_SZ, [_I64]),
    "qva_expectation": (_I, [_P, _P, _I64, _P, _P, _P, _SZ, _P]),
    "qva_evolve": (_I, [_PROB, _P, _P, _I, _P, _P, _P, _I, _P, _SZ, _P]),
    "qva_evolve_noalloc": (_I, [_PROB, _P, _P, _I, _P, _P, _P, _I, _P]),
    "qva_grad": (_I, [_PROB, _P, _P, _I, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "qva_plan": (_I, [_PROB, _I, _I, _I, ctypes.POINTER(QvaPassInfo), _I]),
    "qva_evolve_timed": (_I, [_PROB, _P, _P, _I, _P, _P, _P, _I, _P, _SZ,
                              ctypes.POINTER(ctypes.c_void_p), _I, _P]),
    "qva_grad_timed": (_I, [_PROB, _P, _P, _I, _P, _P, _P, _P, _P, _P, _SZ,
                            ctypes.POINTER(ctypes.c_void_p), _I, _P]),
    "qva_batch_create": (_I, [ctypes.POINTER(QvaBatchItem), _I, _I, ctypes.POINTER(ctypes.c_void_p)]),
    "qva_batch_create_lanes": (_I, [ctypes.POINTER(QvaBatchItem), _I, _I, _I, ctypes.POINTER(ctypes.c_void_p)]),
    "qva_batch_workspace_bytes": (_SZ, [_P]),
    "qva_batch_upload": (_I, [_P, _P, _SZ, _P]),
    "qva_batch_grad": (_I, [_P, _P, _SZ, _P]),
    "qva_batch_sgd": (_I, [_P, _D, _P, _SZ, _P]),
    "qva_batch_grad_timed": (_I, [_P, _P, _SZ, ctypes.POINTER(ctypes.c_void_p), _I, _P]),
    "qva_batch_launch_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "qva_batch_rounds": (_I, [_P]),
    "qva_batch_launches": (_I, [_P]),
    "qva_batch_tiles": (_I64, [_P]),
    "qva_batch_destroy": (_I, [_P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libqva.so; raise if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_2110_03963_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(fn: str, status: int) -> None:
    if status != QVA_OK:
        text = load().qva_status_string(status).decode()
        raise QvaError(fn, status, text)
