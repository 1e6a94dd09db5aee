"""FP64 CPU oracle for batched 1D C2C DFTs (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package imports nothing from it: the two share no code, headers,
tables or helpers.  Inputs reach both from the seeded generators in
``paper_2203_09384_amd.synth``, which hold none of the method's arithmetic.

Every function here is a thin ctypes wrapper over ``fft_oracle.c``, the
recursive radix-2 decimation-in-time FFT of the paper's Eq. (radix2) in
double precision (section "Fast Fourier Transform", Cooley-Tukey
subsection), plus the compositions the hot path needs:

* ``fft(x, sign, scale)``   y = scale * sum_n x_n exp(sign 2 pi i k n / N)
* ``forward``               Eq. (dft): sign -1, scale 1
* ``inverse``               Eq. (idft): sign +1, scale 1/N
* ``adjoint``               adjoint of the (sign, scale) map: (-sign, scale)
* ``fft_ragged``            the same per segment of a packed, offset-indexed
                            batch of mixed power-of-two lengths
* ``loss_grad``             L = sum w |F x|^2 and its PyTorch-convention
                            gradient F^H (2 w * F x)
* ``rfft`` / ``irfft``      real input: the first N/2 + 1 bins of Eq. (dft)
                            of x + 0i; its inverse, Eq. (idft) of the
                            Hermitian extension of N/2 + 1 bins, real part
* ``rfft_adjoint`` / ``irfft_adjoint``  the adjoints of those two real-linear
                            maps (the gradients PyTorch takes through them)
* ``fftn``                  multidimensional transform over the trailing
                            axes: the kernel exp(sign 2 pi i sum_a k_a n_a / N_a)
                            factors into one per axis, so it is the 1D
                            transform applied along each axis in turn

Readings of the paper that these functions take (the inverse carries 1/N,
the adjoint keeps the plan's scale, inputs and outputs in natural order)
are listed in the design notes of the repository.
"""
from __future__ import annotations

import ctypes
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load(path: str = LIB_PATH):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_fft.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oracle_fft.restype = ctypes.c_int
    lib.oracle_fft_ragged.argtypes = [dp, dp, i64p, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oracle_fft_ragged.restype = ctypes.c_int
    lib.oracle_mutant_id.restype = ctypes.c_int
    return lib


def lib():
    """Load liboracle.so, building it with gcc if it is not there yet."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _load(LIB_PATH)
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


class Oracle:
    """The oracle bound to one shared library (the real one, or a mutant
    built by the test-suite with a planted mistake)."""

    def __init__(self, handle=None):
        self._h = handle

    @property
    def h(self):
        return self._h if self._h is not None else lib()

    def fft(self, x, sign: int = -1, scale: float = 1.0, threads: int | None = None):
        """Batched transform over the last axis: scale * DFT with exponent sign."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
        n = x.shape[-1]
        batch = x.size // n if n else 0
        out = np.empty_like(x)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self.h.oracle_fft(x.ctypes.data_as(dp), out.ctypes.data_as(dp), n, batch,
                               int(sign), float(scale), int(threads or default_threads()))
        if rc != 0:
            raise ValueError(f"oracle_fft rejected n={n}, sign={sign}")
        return out

    def forward(self, x, threads=None):
        """Eq. (dft): X_k = sum_n x_n w_N^{kn}."""
        return self.fft(x, -1, 1.0, threads)

    def inverse(self, X, threads=None):
        """Eq. (idft): x_k = (1/N) sum_n X_n w_N^{-kn}."""
        n = np.shape(X)[-1]
        return self.fft(X, +1, 1.0 / n, threads)

    def adjoint(self, g, sign: int = -1, scale: float = 1.0, threads=None):
        """Adjoint of the map x -> scale * DFT_sign(x): the conjugate-sign
        transform at the same (real) scale."""
        return self.fft(g, -sign, scale, threads)

    def fft_ragged(self, x, offsets, sign: int = -1, inverse_scale: bool = False,
                   threads=None):
        """Each segment [offsets[b], offsets[b+1]) transformed on its own;
        inverse_scale multiplies each segment by 1/its length."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(-1))
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        out = np.zeros_like(x)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self.h.oracle_fft_ragged(
            x.ctypes.data_as(dp), out.ctypes.data_as(dp),
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(off) - 1,
            int(sign), 1 if inverse_scale else 0, 1.0, int(threads or default_threads()))
        if rc != 0:
            raise ValueError("oracle_fft_ragged rejected its offsets")
        return out

    def loss_grad(self, x, w, threads=None):
        """L = sum w |F x|^2 with F the forward DFT, and the gradient in
        PyTorch's convention for complex inputs (dL/dRe x + i dL/dIm x),
        which is F^H (2 w * F x)."""
        y = self.forward(x, threads)
        w = np.asarray(w, dtype=np.float64)
        loss = float(np.sum(w * (y.real ** 2 + y.imag ** 2)))
        grad = self.adjoint(2.0 * w * y, sign=-1, scale=1.0, threads=threads)
        return loss, grad

    # -------------------------------------------------------- real input
    # A real sequence is a complex one with zero imaginary parts (the paper
    # allows real- or complex-valued input to Eq. (dft)); its spectrum is
    # Hermitian, X_{N-k} = conj(X_k), so bins 0..N/2 determine it.

    def rfft(self, x, threads=None):
        """X_k = sum_n x_n w_N^{kn} for real x and k = 0..N/2."""
        x = np.asarray(x, dtype=np.float64)
        n = x.shape[-1]
        return self.forward(x.astype(np.complex128), threads)[..., : n // 2 + 1]

    @staticmethod
    def hermitian_extension(X, n: int):
        """The length-n spectrum whose bins 0..n/2 are X (Im of bins 0 and
        n/2 dropped: a real sequence has them real) and whose bins
        n/2+1..n-1 are conj(X_{n-k})."""
        X = np.asarray(X, dtype=np.complex128)
        m = n // 2
        if X.shape[-1] != m + 1:
            raise ValueError(f"{X.shape[-1]} bins given, n={n} needs {m + 1}")
        full = np.empty(X.shape[:-1] + (n,), np.complex128)
        full[..., : m + 1] = X
        full[..., 0] = X[..., 0].real
        full[..., m] = X[..., m].real
        full[..., m + 1:] = np.conj(X[..., 1:m][..., ::-1])
        return full

    def irfft(self, X, n: int, threads=None):
        """x_j = (1/n) sum_k Xfull_k w_n^{-jk} (Eq. (idft)) over the
        Hermitian extension Xfull of X; the result is real."""
        return self.inverse(self.hermitian_extension(X, n), threads).real

    def rfft_adjoint(self, g, n: int, threads=None):
        """Adjoint of x -> rfft(x) from real n-vectors to complex
        (n/2+1)-vectors under Re<a, b>: x_j = Re sum_{k<=n/2} g_k w_n^{-jk}."""
        g = np.asarray(g, dtype=np.complex128)
        padded = np.zeros(g.shape[:-1] + (n,), np.complex128)
        padded[..., : n // 2 + 1] = g
        return self.fft(padded, +1, 1.0, threads).real

    def irfft_adjoint(self, v, threads=None):
        """Adjoint of X -> irfft(X, n), composed from the adjoints of its
        three steps: real part (embed v as complex), the inverse DFT
        (adjoint: sign -1, scale 1/n) and the Hermitian extension (adjoint:
        Y_k + conj(Y_{n-k}) for 0 < k < n/2, Re Y_k at k = 0 and n/2)."""
        v = np.asarray(v, dtype=np.float64)
        n = v.shape[-1]
        m = n // 2
        Y = self.adjoint(v.astype(np.complex128), +1, 1.0 / n, threads)
        out = np.empty(v.shape[:-1] + (m + 1,), np.complex128)
        out[..., 1:m] = Y[..., 1:m] + np.conj(Y[..., n - 1:m:-1])
        out[..., 0] = Y[..., 0].real
        out[..., m] = Y[..., m].real
        return out

    # -------------------------------------------------------- multidimensional
    def fftn(self, x, ndim: int, sign: int = -1, scale: float = 1.0, threads=None):
        """X[k] = scale * sum_n x[n] prod_a exp(sign 2 pi i k_a n_a / N_a) over
        the last `ndim` axes of x (the leading axes are the batch)."""
        y = np.asarray(x, dtype=np.complex128)
        for ax in range(y.ndim - ndim, y.ndim):
            moved = np.moveaxis(y, ax, -1)
            y = np.moveaxis(self.fft(moved, sign, 1.0, threads), -1, ax)
        return y * scale

    def mutant_id(self) -> int:
        return int(self.h.oracle_mutant_id())


_default = Oracle()
fft = _default.fft
forward = _default.forward
inverse = _default.inverse
adjoint = _default.adjoint
fft_ragged = _default.fft_ragged
loss_grad = _default.loss_grad
rfft = _default.rfft
irfft = _default.irfft
rfft_adjoint = _default.rfft_adjoint
irfft_adjoint = _default.irfft_adjoint
hermitian_extension = Oracle.hermitian_extension
fftn = _default.fftn
