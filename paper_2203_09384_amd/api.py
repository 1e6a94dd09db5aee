"""Python binding of the mifft C ABI: plans, execute calls and the
differentiable FFT.  Argument marshalling only -- every transform runs in
the HIP kernels of libmifft.so; torch provides device memory and streams.
"""
from __future__ import annotations

import ctypes
import threading

import torch

from . import native
from .native import FFT_C16, FFT_C32, FFT_CBF16, FFT_R32, MifftError, check, check_plan, lib

DTYPES = {"c32": FFT_C32, "c16": FFT_C16, "cbf16": FFT_CBF16, "r32": FFT_R32}
_HALF_TORCH = {FFT_C16: torch.float16, FFT_CBF16: torch.bfloat16}


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def query(n: int, batch: int = 1, sign: int = -1, dtype: str = "c32") -> dict:
    """Host-only planning (no device needed): what a plan would launch."""
    d = native.PlanDesc()
    check(lib().fft_plan_query(n, batch, sign, DTYPES[dtype], ctypes.byref(d)))
    return d.as_dict()


def c32_variants(n: int) -> list:
    """Host-only: the compiled FP32 variants (ept, wg, variant) for length n."""
    L = lib()
    count = L.fft_c32_variants(n, None, 0)
    if count < 0:
        check(L.fft_last_error())
    buf = (ctypes.c_int * (3 * count))()
    L.fft_c32_variants(n, buf, count)
    return [tuple(buf[3 * i: 3 * i + 3]) for i in range(count)]


class Plan:
    """fft_plan_create(n, batch, sign, dtype) and its execute calls.

    sign -1 is the forward transform of the paper's Eq. (dft); +1 the
    inverse of Eq. (idft) with its 1/n.  For dtype 'c32' tensors are
    torch.complex64 of shape (..., n) with batch = numel / n; for 'c16' /
    'cbf16' they are float16 / bfloat16 of shape (..., n, 2).  For 'r32'
    (real input) the real side is float32 (..., n) and the spectrum side
    complex64 (..., n/2 + 1): sign -1 maps real -> spectrum, +1 back.
    """

    def __init__(self, n: int, batch: int, sign: int = -1, dtype: str = "c32",
                 ept: int | None = None, wg: int | None = None, variant: int = 0):
        L = lib()
        self.n, self.batch, self.sign, self.dtype = int(n), int(batch), int(sign), DTYPES[dtype]
        if ept is not None or wg is not None:
            h = L.fft_plan_create_config(self.n, self.batch, self.sign, self.dtype,
                                         int(ept or 0), int(wg or 0), int(variant))
        else:
            h = L.fft_plan_create(self.n, self.batch, self.sign, self.dtype)
        self._h = check_plan(h)

    # -- marshalling -------------------------------------------------------
    def _check_tensor(self, x, what, side=None):
        if not x.is_cuda:
            raise ValueError(f"{what} must be a GPU tensor")
        if not x.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if self.dtype == FFT_R32:
            want, count = ((torch.float32, self.n * self.batch) if side == "real"
                           else (torch.complex64, (self.n // 2 + 1) * self.batch))
            if x.dtype != want:
                raise ValueError(f"{what} must be {want}, got {x.dtype}")
            if x.numel() != count:
                raise ValueError(f"{what} has {x.numel()} elements, plan needs {count}")
        elif self.dtype == FFT_C32:
            if x.dtype != torch.complex64:
                raise ValueError(f"{what} must be complex64, got {x.dtype}")
            if x.numel() != self.n * self.batch:
                raise ValueError(f"{what} has {x.numel()} elements, plan needs {self.n}*{self.batch}")
        else:
            if x.dtype != _HALF_TORCH[self.dtype]:
                raise ValueError(f"{what} must be {_HALF_TORCH[self.dtype]}, got {x.dtype}")
            if x.numel() != 2 * self.n * self.batch:
                raise ValueError(f"{what} has {x.numel()} values, plan needs 2*{self.n}*{self.batch}")

    def _sides(self, to_spectrum: bool):
        return ("real", "spectrum") if to_spectrum else ("spectrum", "real")

    def _new_like_side(self, x, side):
        lead = x.shape[:-1]
        if side == "real":
            return torch.empty(lead + (self.n,), dtype=torch.float32, device=x.device)
        return torch.empty(lead + (self.n // 2 + 1,), dtype=torch.complex64, device=x.device)

    def _run(self, fn, x, out, stream, to_spectrum):
        if self.dtype == FFT_R32:
            sin, sout = self._sides(to_spectrum)
            self._check_tensor(x, "input", sin)
            if out is None:
                out = self._new_like_side(x, sout)
            self._check_tensor(out, "output", sout)
        else:
            self._check_tensor(x, "input")
            if out is None:
                out = torch.empty_like(x)
            self._check_tensor(out, "output")
        check(fn(self._h, _ptr(x), _ptr(out), _stream_handle(stream)))
        return out

    def execute(self, x, out=None, stream=None):
        """out = plan(x); allocates `out` (torch caching allocator) if not given."""
        return self._run(lib().fft_execute, x, out, stream, self.sign < 0)

    def adjoint(self, g, out=None, stream=None):
        """out = plan^H(g): conjugate sign, same scale (real-input plans: the
        adjoint under Re<a, b>, from the spectrum side for sign -1)."""
        return self._run(lib().fft_execute_adjoint, g, out, stream, self.sign > 0)

    def execute_scaled(self, x, in_exp=None, out=None, out_exp=None, stream=None):
        """Block floating point (FP16/BF16 plans): value = stored * 2^exp[b]."""
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        if out_exp is None:
            out_exp = torch.empty(self.batch, dtype=torch.int32, device=x.device)
        for e, nm in ((in_exp, "in_exp"), (out_exp, "out_exp")):
            if e is not None and (e.dtype != torch.int32 or e.numel() != self.batch
                                  or not e.is_cuda or not e.is_contiguous()):
                raise ValueError(f"{nm} must be a contiguous int32 GPU tensor of {self.batch} values")
        check(lib().fft_execute_scaled(self._h, _ptr(x),
                                       _ptr(in_exp) if in_exp is not None else None,
                                       _ptr(out), _ptr(out_exp), _stream_handle(stream)))
        return out, out_exp

    def loss_grad(self, x, w, grad=None, loss=None, stream=None):
        """Fused loss[b] = sum_k w |(A x_b)_k|^2 and grad = A^H (2 w A x) (FP32 plans)."""
        self._check_tensor(x, "input")
        if w.dtype != torch.float32 or not w.is_cuda or not w.is_contiguous() or w.numel() != x.numel():
            raise ValueError("w must be a contiguous float32 GPU tensor shaped like x")
        if grad is None:
            grad = torch.empty_like(x)
        self._check_tensor(grad, "grad")
        if loss is None:
            loss = torch.empty(self.batch, dtype=torch.float32, device=x.device)
        if loss.dtype != torch.float32 or loss.numel() != self.batch or not loss.is_contiguous():
            raise ValueError(f"loss must be a contiguous float32 tensor of {self.batch} values")
        check(lib().fft_execute_loss_grad(self._h, _ptr(x), _ptr(w), _ptr(grad), _ptr(loss),
                                          _stream_handle(stream)))
        return loss, grad

    def describe(self) -> dict:
        d = native.PlanDesc()
        check(lib().fft_plan_describe(self._h, ctypes.byref(d)))
        return d.as_dict()

    def twiddles(self):
        """A copy of the plan's FP32 twiddle table, exp(-2 pi i m / 2048) for
        m < 2048, as a complex64 GPU tensor."""
        p = lib().fft_plan_twiddles(self._h)
        view = torch.as_tensor(_DeviceArray(p, (2048, 2), "<f4"), device="cuda")
        return torch.view_as_complex(view.clone())

    def close(self):
        if getattr(self, "_h", None):
            lib().fft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Exposes a raw device pointer through __cuda_array_interface__."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2, "strides": None}


class RaggedPlan:
    """fft_plan_create_ragged(count, offsets, sign, dtype): mixed lengths,
    packed back to back, one launch per execute."""

    def __init__(self, offsets, sign: int = -1, dtype: str = "c32",
                 ept_by_log2n=None, wg: int = 0, ctas_per_cu: int = 0):
        import numpy as np
        L = lib()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.offsets = off
        self.count = len(off) - 1
        self.total = int(off[-1])
        self.sign = int(sign)
        self.dtype = DTYPES[dtype]
        op = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        if ept_by_log2n is not None or wg or ctas_per_cu:
            arr = None
            if ept_by_log2n is not None:
                arr = (ctypes.c_int * 12)(*[int(v) for v in ept_by_log2n])
            h = L.fft_plan_create_ragged_config(self.count, op, self.sign, self.dtype, arr,
                                                int(wg), int(ctas_per_cu))
        else:
            h = L.fft_plan_create_ragged(self.count, op, self.sign, self.dtype)
        self._h = check_plan(h)

    def _check_tensor(self, x, what):
        if not x.is_cuda or not x.is_contiguous() or x.dtype != torch.complex64:
            raise ValueError(f"{what} must be a contiguous complex64 GPU tensor")
        if x.numel() != self.total:
            raise ValueError(f"{what} has {x.numel()} elements, plan needs {self.total}")

    def execute(self, x, out=None, stream=None):
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        check(lib().fft_execute(self._h, _ptr(x), _ptr(out), _stream_handle(stream)))
        return out

    def adjoint(self, g, out=None, stream=None):
        self._check_tensor(g, "input")
        if out is None:
            out = torch.empty_like(g)
        self._check_tensor(out, "output")
        check(lib().fft_execute_adjoint(self._h, _ptr(g), _ptr(out), _stream_handle(stream)))
        return out

    def describe(self) -> dict:
        d = native.PlanDesc()
        check(lib().fft_plan_describe(self._h, ctypes.byref(d)))
        return d.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().fft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ plan cache
_cache: dict = {}
_cache_lock = threading.Lock()


def _refuse_under_capture(what):
    """Plan creation allocates device memory and waits for its tables, which
    a stream capture cannot contain: raise before touching the device (the
    capture stays intact) rather than let the capture be invalidated."""
    if torch.cuda.is_current_stream_capturing():
        raise MifftError(native.FFT_ECAPTURE, f"{what}: no cached plan for this shape, and plans cannot be "
                                              "created during stream capture; run the call once before capturing")


def get_plan(n: int, batch: int, sign: int, dtype: str = "c32", device=None) -> Plan:
    dev = torch.cuda.current_device() if device is None else device
    key = (dev, n, batch, sign, dtype)
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            _refuse_under_capture(f"plan n={n} batch={batch} sign={sign} {dtype}")
            with torch.cuda.device(dev):
                p = Plan(n, batch, sign, dtype)
            _cache[key] = p
        return p


def fft(x, sign: int = -1):
    """Transform over the last dimension of a complex64 GPU tensor (new tensor)."""
    x = x.contiguous()
    n = x.shape[-1]
    return get_plan(n, x.numel() // n, sign, "c32", x.device.index).execute(x)


def ifft(X):
    return fft(X, sign=+1)


class FFTFn(torch.autograd.Function):
    """Differentiable batched FFT.  Forward: the plan's transform.  Backward:
    its adjoint (conjugate sign, same scale) applied to the incoming
    gradient, which for PyTorch's complex convention (grad = dL/dRe + i
    dL/dIm) is exactly the gradient of any real loss.  No tensors are saved:
    the map is linear."""

    @staticmethod
    def forward(ctx, x, sign: int = -1):
        x = x.contiguous()
        n = x.shape[-1]
        plan = get_plan(n, x.numel() // n, sign, "c32", x.device.index)
        ctx.plan = plan
        return plan.execute(x)

    @staticmethod
    def backward(ctx, grad_out):
        g = grad_out.contiguous()
        if g.dtype != torch.complex64:
            g = g.to(torch.complex64)
        return ctx.plan.adjoint(g), None


def fft_differentiable(x, sign: int = -1):
    return FFTFn.apply(x, sign)


FUSED_LOSS_MAX_N = 2048  # the fused loss-gradient kernel's lengths


class WeightedPowerLossFn(torch.autograd.Function):
    """L = sum_b sum_k w |(A x_b)_k|^2 in one fused kernel that also produces
    dL/dx = A^H (2 w A x) (PyTorch's complex convention); backward scales the
    saved gradient by the incoming scalar.  w is treated as a constant.
    Lengths 2..2048 (the fused kernel's range); for longer transforms
    compose fft_differentiable with the loss in torch."""

    @staticmethod
    def forward(ctx, x, w, sign: int = -1):
        x = x.contiguous()
        w = w.contiguous()
        n = x.shape[-1]
        if n > FUSED_LOSS_MAX_N:
            raise ValueError(f"the fused loss kernel covers n <= {FUSED_LOSS_MAX_N} (got n={n}); "
                             "use fft_differentiable and the loss in torch")
        plan = get_plan(n, x.numel() // n, sign, "c32", x.device.index)
        loss, grad = plan.loss_grad(x, w)
        ctx.save_for_backward(grad)
        return loss.sum()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g.to(grad.real.dtype), None, None


def weighted_power_loss(x, w, sign: int = -1):
    return WeightedPowerLossFn.apply(x, w, sign)


# ------------------------------------------------------------------ real input
def rfft(x):
    """Bins 0..n/2 of the forward transform of a real float32 GPU tensor
    (last dimension n) as a new complex64 tensor (..., n/2 + 1)."""
    x = x.contiguous()
    n = x.shape[-1]
    return get_plan(n, x.numel() // n, -1, "r32", x.device.index).execute(x)


def irfft(X, n: int | None = None):
    """Inverse of rfft: n reals (default 2 * (bins - 1)) from n/2 + 1 bins,
    with the 1/n of Eq. (idft); imaginary parts of bins 0 and n/2 ignored."""
    X = X.contiguous()
    n = 2 * (X.shape[-1] - 1) if n is None else int(n)
    if X.shape[-1] != n // 2 + 1:
        raise ValueError(f"{X.shape[-1]} bins given, n={n} needs {n // 2 + 1}")
    return get_plan(n, X.numel() // (n // 2 + 1), +1, "r32", X.device.index).execute(X)


class RFFTFn(torch.autograd.Function):
    """Differentiable rfft; backward is the plan's adjoint, x.grad =
    Re sum_k g_k w^{-jk} over the n/2 + 1 bins."""

    @staticmethod
    def forward(ctx, x):
        x = x.contiguous()
        n = x.shape[-1]
        ctx.plan = get_plan(n, x.numel() // n, -1, "r32", x.device.index)
        return ctx.plan.execute(x)

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        if g.dtype != torch.complex64:
            g = g.to(torch.complex64)
        return ctx.plan.adjoint(g)


class IRFFTFn(torch.autograd.Function):
    """Differentiable irfft; backward is the plan's adjoint (an R2C with
    the 1/n and the interior bins doubled)."""

    @staticmethod
    def forward(ctx, X, n: int):
        X = X.contiguous()
        ctx.plan = get_plan(n, X.numel() // (n // 2 + 1), +1, "r32", X.device.index)
        return ctx.plan.execute(X)

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        if g.dtype != torch.float32:
            g = g.to(torch.float32)
        return ctx.plan.adjoint(g), None


def rfft_differentiable(x):
    return RFFTFn.apply(x)


def irfft_differentiable(X, n: int | None = None):
    n = 2 * (X.shape[-1] - 1) if n is None else int(n)
    return IRFFTFn.apply(X, n)


# ------------------------------------------------------------------ multidimensional
class PlanND(Plan):
    """fft_plan_create_nd(rank, dims, batch, sign, FFT_C32): `batch` arrays
    of shape `dims` (row-major), transformed over all their axes."""

    def __init__(self, dims, batch: int, sign: int = -1):
        import numpy as np
        L = lib()
        self.dims = tuple(int(d) for d in dims)
        self.n = int(np.prod(self.dims))
        self.batch, self.sign, self.dtype = int(batch), int(sign), FFT_C32
        arr = (ctypes.c_int64 * len(self.dims))(*self.dims)
        self._h = check_plan(L.fft_plan_create_nd(len(self.dims), arr, self.batch, self.sign, FFT_C32))


def _nd_plan(shape, batch, sign, device):
    dev = torch.cuda.current_device() if device is None else device
    key = (dev, "nd", tuple(shape), batch, sign)
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            _refuse_under_capture(f"plan dims={tuple(shape)} batch={batch} sign={sign}")
            with torch.cuda.device(dev):
                p = PlanND(shape, batch, sign)
            _cache[key] = p
        return p


def fftn(x, ndim: int | None = None, sign: int = -1):
    """Transform over the last `ndim` dimensions (default all, at most 3) of
    a complex64 GPU tensor; new tensor."""
    x = x.contiguous()
    ndim = x.dim() if ndim is None else int(ndim)
    shape = tuple(x.shape[x.dim() - ndim:])
    n = 1
    for d in shape:
        n *= d
    return _nd_plan(shape, x.numel() // n, sign, x.device.index).execute(x)


def ifftn(X, ndim: int | None = None):
    return fftn(X, ndim, sign=+1)


def fft2(x):
    return fftn(x, 2)


def ifft2(X):
    return fftn(X, 2, sign=+1)


class FFTNFn(torch.autograd.Function):
    """Differentiable multidimensional FFT; backward is the plan's adjoint."""

    @staticmethod
    def forward(ctx, x, ndim: int, sign: int = -1):
        x = x.contiguous()
        shape = tuple(x.shape[x.dim() - ndim:])
        n = 1
        for d in shape:
            n *= d
        ctx.plan = _nd_plan(shape, x.numel() // n, sign, x.device.index)
        return ctx.plan.execute(x)

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        if g.dtype != torch.complex64:
            g = g.to(torch.complex64)
        return ctx.plan.adjoint(g), None, None


def fftn_differentiable(x, ndim: int, sign: int = -1):
    return FFTNFn.apply(x, ndim, sign)
