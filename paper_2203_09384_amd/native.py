"""ctypes declarations of the C ABI in include/mifft.h (no logic here).

The library is loaded from this package directory.  There is no fallback:
if ``libmifft.so`` is missing the import of any compute entry point raises.
torch is imported first so the library binds to the HIP runtime torch has
already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmifft.so")

FFT_C32, FFT_C16, FFT_CBF16, FFT_R32 = 0, 1, 2, 3
STATUS = {
    0: "FFT_OK", 1: "FFT_EINVAL_N", 2: "FFT_EINVAL_BATCH", 3: "FFT_EINVAL_SIGN",
    4: "FFT_EINVAL_DTYPE", 5: "FFT_ENULL", 6: "FFT_EOVERLAP", 7: "FFT_EINVAL_OFFSETS",
    8: "FFT_EHIP", 9: "FFT_ENOMEM", 10: "FFT_EINVAL_CONFIG", 11: "FFT_EALIGN", 12: "FFT_EDEVICE",
    13: "FFT_ECAPTURE",
}
FFT_ECAPTURE = 13
EXPORTS = [
    "fft_plan_create", "fft_plan_create_config", "fft_plan_create_ragged",
    "fft_plan_create_ragged_config", "fft_execute", "fft_execute_adjoint",
    "fft_execute_scaled", "fft_plan_destroy", "fft_plan_describe", "fft_plan_query",
    "fft_plan_twiddles", "fft_last_error", "fft_last_error_string", "fft_version",
    "fft_execute_loss_grad", "fft_plan_create_nd", "fft_c32_variants",
    "fft_execute_static_scratch",
]
STATIC_SCRATCH_BYTES = 64 << 20  # MIFFT_STATIC_SCRATCH_BYTES


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("batch", ctypes.c_int64), ("sign", ctypes.c_int),
        ("dtype", ctypes.c_int), ("scale", ctypes.c_float), ("ept", ctypes.c_int),
        ("wg", ctypes.c_int), ("transforms_per_wg", ctypes.c_int), ("grid", ctypes.c_int64),
        ("npasses", ctypes.c_int), ("radices", ctypes.c_int * 8), ("lds_bytes", ctypes.c_int),
        ("kind", ctypes.c_int), ("tiles", ctypes.c_int64), ("variant", ctypes.c_int),
        ("ept_by_log2n", ctypes.c_int * 12), ("rank", ctypes.c_int), ("dims", ctypes.c_int64 * 3),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("radices", "ept_by_log2n", "dims")}
        d["radices"] = list(self.radices)[: self.npasses]
        d["ept_by_log2n"] = list(self.ept_by_log2n)
        d["dims"] = list(self.dims)[: self.rank]
        return d


class MifftError(RuntimeError):
    def __init__(self, code: int, message: str):
        self.code = code
        self.status = STATUS.get(code, str(code))
        super().__init__(f"{self.status}: {message}")


_lib = None


def lib():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (share torch's HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(or python -m paper_2203_09384_amd.build)")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _declare(L):
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.fft_plan_create.argtypes = [i64, i64, i32, i32]
    L.fft_plan_create.restype = vp
    L.fft_plan_create_config.argtypes = [i64, i64, i32, i32, i32, i32, i32]
    L.fft_plan_create_config.restype = vp
    L.fft_plan_create_nd.argtypes = [i32, ctypes.POINTER(i64), i64, i32, i32]
    L.fft_plan_create_nd.restype = vp
    L.fft_plan_create_ragged.argtypes = [i64, ctypes.POINTER(i64), i32, i32]
    L.fft_plan_create_ragged.restype = vp
    L.fft_plan_create_ragged_config.argtypes = [i64, ctypes.POINTER(i64), i32, i32,
                                                ctypes.POINTER(i32), i32, i32]
    L.fft_plan_create_ragged_config.restype = vp
    L.fft_execute.argtypes = [vp, vp, vp, vp]
    L.fft_execute.restype = i32
    L.fft_execute_static_scratch.argtypes = [vp, vp, vp, vp]
    L.fft_execute_static_scratch.restype = i32
    L.fft_execute_adjoint.argtypes = [vp, vp, vp, vp]
    L.fft_execute_adjoint.restype = i32
    L.fft_execute_scaled.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fft_execute_scaled.restype = i32
    L.fft_execute_loss_grad.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fft_execute_loss_grad.restype = i32
    L.fft_plan_destroy.argtypes = [vp]
    L.fft_plan_destroy.restype = None
    L.fft_plan_describe.argtypes = [vp, ctypes.POINTER(PlanDesc)]
    L.fft_plan_describe.restype = i32
    L.fft_plan_query.argtypes = [i64, i64, i32, i32, ctypes.POINTER(PlanDesc)]
    L.fft_plan_query.restype = i32
    L.fft_plan_twiddles.argtypes = [vp]
    L.fft_plan_twiddles.restype = vp
    L.fft_last_error.argtypes = []
    L.fft_last_error.restype = i32
    L.fft_last_error_string.argtypes = []
    L.fft_last_error_string.restype = ctypes.c_char_p
    L.fft_c32_variants.argtypes = [i64, ctypes.POINTER(i32), i32]
    L.fft_c32_variants.restype = i32
    L.fft_version.argtypes = []
    L.fft_version.restype = ctypes.c_char_p
    return L


def check(rc: int):
    if rc != 0:
        raise MifftError(rc, lib().fft_last_error_string().decode())


def check_plan(handle):
    if not handle:
        L = lib()
        raise MifftError(L.fft_last_error(), L.fft_last_error_string().decode())
    return handle
