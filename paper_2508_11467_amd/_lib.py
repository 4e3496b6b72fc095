"""ctypes declarations of libbdc.so (the C ABI in include/bdc.h)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdc.so")

BDC_OK = 0
BDC_ERR_INVALID_HANDLE = -1001
BDC_ERR_NO_DEVICE = -1002
BDC_ERR_NOMEM = -1003
BDC_ERR_HIP = -1004
BDC_ERR_NONFINITE = -1005
BDC_ERR_UNSUPPORTED = -1006
BDC_ERR_NO_MODEL = -1007
BDC_ERR_TOO_LARGE = -1008
BDC_START_PLAIN = 0
BDC_START_LEARNED = 1
BDC_GEMM_FP64 = 0
BDC_GEMM_OZAKI = 1
BDC_GEMM_CRT = 2
MLP_FEATURES = 19
MLP_PARAMS = 19 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1

c_int = ctypes.c_int
c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
c_char_p = ctypes.c_char_p


class Options(ctypes.Structure):
    _fields_ = [
        ("leaf_size", c_int),
        ("max_secular_iters", c_int),
        ("max_leaf_sweeps", c_int),
        ("workspace_cap_bytes", ctypes.c_size_t),
        ("timing", c_int),
        ("use_graph", c_int),
        ("start", c_int),
        ("gemm", c_int),
        ("ozaki_slices", c_int),
        ("ozaki_min_n", c_int),
        ("crt_moduli", c_int),
        ("learned_min_n", c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("merges", c_i64),
        ("roots", c_i64),
        ("secular_evals", c_i64),
        ("deflated_small_z", c_i64),
        ("deflated_zero_d", c_i64),
        ("deflated_close", c_i64),
        ("rotations", c_i64),
        ("update_flops", c_dbl),
        ("root_N", c_i64),
        ("levels", c_i64),
        ("secular_terms", c_i64),
        ("leaf_flops", c_dbl),
        ("gather_bytes", c_dbl),
        ("final_read_elems", c_i64),
        ("split_merges", c_i64),
        ("split_flops", c_dbl),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [
        ("small_n", c_int),
        ("flat", c_int),
        ("grid64", c_int),
        ("grid128", c_int),
        ("sec_small_n", c_int),
        ("leaf_size", c_int),
        ("tile128", c_int),
        ("streams", c_int),
        ("ms", ctypes.c_float),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes)
SIGNATURES = {
    "bdc_default_options": (None, [ctypes.POINTER(Options)]),
    "bdc_create": (c_int, [ctypes.POINTER(c_vp), c_int, ctypes.POINTER(Options)]),
    "bdc_destroy": (c_int, [c_vp]),
    "bdc_svd": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "bdc_svd_batched": (c_int, [c_vp, c_i64, ctypes.POINTER(c_i64), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "bdc_get_info": (c_int, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(Stats)]),
    "bdc_get_timing": (c_int, [c_vp, c_int, ctypes.POINTER(c_char_p), ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64)]),
    "bdc_clear_timing": (c_int, [c_vp]),
    "bdc_step_leaf": (c_int, [c_vp, c_int, c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "bdc_step_deflate": (c_int, [c_vp, c_int, c_int, c_vp, c_vp, c_vp, c_dbl, c_dbl, c_vp, c_vp, c_vp,
                                 c_vp, c_vp, c_vp, c_vp, c_vp]),
    "bdc_step_secular": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "bdc_step_vectors": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "bdc_step_gemm": (c_int, [c_vp, c_int, c_int, c_int, c_vp, c_int, c_vp, c_int, c_vp, c_int, c_vp]),
    "bdc_step_secular_start": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "bdc_step_features": (c_int, [c_vp, c_int, c_vp, c_vp, c_vp, c_vp]),
    "bdc_mlp_set": (c_int, [c_vp, c_vp, c_i64]),
    "bdc_mlp_get": (c_int, [c_vp, c_vp, c_i64]),
    "bdc_mlp_forward": (c_int, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "bdc_mlp_grad": (c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "bdc_mlp_train": (c_int, [c_vp, c_vp, c_vp, c_vp, c_i64, c_i64, ctypes.c_float, c_vp, c_vp]),
    "bdc_set_harvest": (c_int, [c_vp, c_vp, c_vp, c_vp, c_i64, c_vp]),
    "bdc_step_gemm_ozaki": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_vp, c_int, c_vp, c_int, c_vp, c_int, c_vp]),
    "bdc_step_gemm_crt": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_vp, c_int, c_vp, c_int, c_vp, c_int, c_vp]),
    "bdc_apply_reflectors": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_int, c_vp, c_i64, c_i64, c_vp, c_vp, c_int,
                                     c_int, c_vp]),
    "bdc_apply_reflectors_noalloc": (c_int, [c_vp, c_int, c_int, c_int, c_int, c_int, c_vp, c_i64, c_i64, c_vp,
                                             c_vp, c_int, c_int, c_vp]),
    "bdc_geqrf": (c_int, [c_vp, c_int, c_int, c_vp, c_int, c_vp, c_int, c_vp]),
    "bdc_gebrd": (c_int, [c_vp, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_vp, c_vp, c_int, c_vp]),
    "bdc_orgqr": (c_int, [c_vp, c_int, c_int, c_int, c_vp, c_int, c_vp, c_vp, c_int, c_int, c_vp]),
    "bdc_get_tuning": (c_int, [c_vp, ctypes.POINTER(Tuning)]),
    "bdc_set_tuning": (c_int, [c_vp, ctypes.POINTER(Tuning)]),
    "bdc_autotune": (c_int, [c_vp, c_i64, ctypes.POINTER(c_i64), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_int,
                             ctypes.POINTER(Tuning)]),
    "bdc_status_string": (c_char_p, [c_int]),
}

_LIB = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libbdc.so; raises when it has not been built."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run __graft_entry__.build() "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib


def status_string(code: int) -> str:
    return load().bdc_status_string(code).decode()


class BdcError(RuntimeError):
    def __init__(self, func: str, code: int):
        self.code = code
        super().__init__(f"{func} failed: {code} ({status_string(code)})")


def check(func: str, code: int) -> int:
    if code != BDC_OK:
        raise BdcError(func, code)
    return code
