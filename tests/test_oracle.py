"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself or retypes its recursion:
each pin is an independent statement (the direct O(N^2) sum of Eq. (dft),
closed forms, hand-worked values, invariants, an independent FP64 library).
``test_pins_catch_planted_mistakes`` builds the oracle with one planted
mistake at a time and checks that at least one pin fails for every one.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_2203_09384_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
POW2_SMALL = [2, 4, 8, 16, 32, 64]
POW2_ALL = [1 << L for L in range(1, 12)]


def relerr(y, ref):
    y = np.asarray(y, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300))


def direct_dft(x, sign):
    """Eq. (dft) / Eq. (idft) without the 1/N: N terms per output, the
    exponent k*n reduced modulo N in exact integers before the angle."""
    n = x.shape[-1]
    kn = np.outer(np.arange(n), np.arange(n)) % n
    W = np.exp(sign * 2j * np.pi * kn / n)
    return x @ W.T


# ---------------------------------------------------------------- pin bodies

def pin_brute_force(orc):
    for n in POW2_SMALL:
        x = synth.uniform_complex(7, (3, n), key=(n,), dtype=np.complex128)
        assert relerr(orc.forward(x), direct_dft(x, -1)) < 1e-13, n
        assert relerr(orc.inverse(x), direct_dft(x, +1) / n) < 1e-13, n


def pin_small_closed_forms(orc):
    a, b, c, d = 0.3 - 0.7j, -1.1 + 0.2j, 0.5 + 0.9j, -0.4 - 0.25j
    X2 = orc.forward(np.array([a, b]))
    assert np.allclose(X2, [a + b, a - b], rtol=0, atol=1e-15)
    X4 = orc.forward(np.array([a, b, c, d]))
    want = [a + b + c + d, a - 1j * b - c + 1j * d, a - b + c - d, a + 1j * b - c - 1j * d]
    assert np.allclose(X4, want, rtol=0, atol=1e-15)


def pin_impulse_tone_constant(orc):
    for n in (8, 256, 2048):
        k = np.arange(n)
        for n0 in (0, 1, n // 3, n - 1):
            x = np.zeros(n, np.complex128)
            x[n0] = 1.0
            want = np.exp(-2j * np.pi * ((k * n0) % n) / n)
            assert np.max(np.abs(orc.forward(x) - want)) < 1e-13 * np.sqrt(n)
        for k0 in (0, 1, n // 2 - 1, n - 1):
            tone = np.exp(2j * np.pi * ((k0 * k) % n) / n)
            want = np.zeros(n, np.complex128)
            want[k0] = n
            assert np.max(np.abs(orc.forward(tone) - want)) < 1e-10
        const = np.full(n, 0.75 - 0.5j)
        want = np.zeros(n, np.complex128)
        want[0] = n * (0.75 - 0.5j)
        assert np.max(np.abs(orc.forward(const) - want)) < 1e-10


def pin_ramp_closed_form(orc):
    """The paper's f(x) = x workload: X_0 = N(N-1)/2, X_k = -N/2 + i (N/2) cot(pi k / N)."""
    for n in POW2_ALL:
        x = np.arange(n, dtype=np.float64).astype(np.complex128)
        k = np.arange(1, n)
        want = np.empty(n, np.complex128)
        want[0] = n * (n - 1) / 2
        want[1:] = -n / 2 + 1j * (n / 2) / np.tan(np.pi * k / n)
        assert relerr(orc.forward(x), want) < 1e-13, n


def pin_golden_ramps(orc):
    for name, n in (("ramp_n4.txt", 4), ("ramp_n8.txt", 8)):
        tab = np.loadtxt(os.path.join(GOLDEN, name), comments="#")
        want = tab[:, 1] + 1j * tab[:, 2]
        got = orc.forward(np.arange(n, dtype=np.float64).astype(np.complex128))
        assert np.max(np.abs(got - want)) < 1e-13, name
        # inverse of the printed spectrum gives the ramp back (Eq. (idft))
        assert np.max(np.abs(orc.inverse(want) - np.arange(n))) < 1e-13, name


def pin_linearity_parseval_roundtrip(orc):
    for n in (2, 32, 2048):
        x = synth.uniform_complex(11, (4, n), key=(n, 0), dtype=np.complex128)
        y = synth.uniform_complex(11, (4, n), key=(n, 1), dtype=np.complex128)
        a, b = 0.7 - 1.3j, -2.0 + 0.1j
        assert relerr(orc.forward(a * x + b * y), a * orc.forward(x) + b * orc.forward(y)) < 1e-13
        X = orc.forward(x)
        lhs = np.sum(np.abs(X) ** 2, axis=-1)
        rhs = n * np.sum(np.abs(x) ** 2, axis=-1)
        assert np.max(np.abs(lhs - rhs) / rhs) < 1e-13
        assert relerr(orc.inverse(X), x) < 1e-14


def pin_shift_theorem(orc):
    for n in (16, 1024):
        x = synth.uniform_complex(13, (2, n), key=(n,), dtype=np.complex128)
        k = np.arange(n)
        for s in (1, 5, n - 3):
            lhs = orc.forward(np.roll(x, s, axis=-1))
            rhs = orc.forward(x) * np.exp(-2j * np.pi * ((k * s) % n) / n)
            assert relerr(lhs, rhs) < 1e-13


def pin_numpy_library(orc):
    """numpy.fft (pocketfft, FP64) is an FFT written independently of this one."""
    for n in POW2_ALL:
        x = synth.uniform_complex(17, (5, n), key=(n,), dtype=np.complex128)
        assert relerr(orc.forward(x), np.fft.fft(x, axis=-1)) < 1e-13, n
        assert relerr(orc.inverse(x), np.fft.ifft(x, axis=-1)) < 1e-13, n


def pin_adjoint_identity(orc):
    """<A x, y> = <x, A^H y> for the forward map and the inverse map."""
    for n in (4, 128, 2048):
        x = synth.uniform_complex(19, (3, n), key=(n, 0), dtype=np.complex128)
        y = synth.uniform_complex(19, (3, n), key=(n, 1), dtype=np.complex128)
        for sign, scale in ((-1, 1.0), (+1, 1.0 / n)):
            Ax = orc.fft(x, sign, scale)
            AHy = orc.adjoint(y, sign, scale)
            lhs = np.vdot(y, Ax)
            rhs = np.vdot(AHy, x)
            assert abs(lhs - rhs) < 1e-12 * abs(lhs), (n, sign)


def pin_loss_gradient_fd(orc):
    """Central finite differences are exact for the quadratic loss sum w |Fx|^2
    (up to rounding), for any step, so they pin the gradient convention."""
    n, batch, h = 16, 4, 1e-2
    x = synth.uniform_complex(23, (batch, n), dtype=np.complex128)
    w = synth.uniform_weights(23, (batch, n), key=(1,), dtype=np.float64)

    def loss(z):
        return float(np.sum(w * np.abs(direct_dft(z, -1)) ** 2))

    _, g = orc.loss_grad(x, w)
    fd = np.zeros_like(x)
    for b in range(batch):
        for i in range(n):
            for part, unit in ((0, 1.0), (1, 1j)):
                e = np.zeros_like(x)
                e[b, i] = unit * h
                d = (loss(x + e) - loss(x - e)) / (2 * h)
                if part == 0:
                    fd[b, i] += d
                else:
                    fd[b, i] += 1j * d
    assert relerr(g, fd) < 1e-11


def pin_ragged(orc):
    lengths = synth.ragged_lengths(29, 40, 1, 11)
    off = synth.offsets_from_lengths(lengths)
    x = synth.uniform_complex(29, (int(off[-1]),), key=(1,), dtype=np.complex128)
    for inv in (False, True):
        y = orc.fft_ragged(x, off, +1 if inv else -1, inverse_scale=inv)
        for b in range(len(lengths)):
            seg = slice(off[b], off[b + 1])
            ref = np.fft.ifft(x[seg]) if inv else np.fft.fft(x[seg])
            assert relerr(y[seg], ref) < 1e-13


PINS = [pin_brute_force, pin_small_closed_forms, pin_impulse_tone_constant,
        pin_ramp_closed_form, pin_golden_ramps, pin_linearity_parseval_roundtrip,
        pin_shift_theorem, pin_numpy_library, pin_adjoint_identity,
        pin_loss_gradient_fd, pin_ragged]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    pin(Oracle())


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((2, 12), np.complex128))
    with pytest.raises(ValueError):
        oracle.fft_ragged(np.zeros(10, np.complex128), [0, 4, 10])


def test_threads_do_not_change_results():
    x = synth.uniform_complex(31, (37, 512), dtype=np.complex128)
    a = oracle.forward(x, threads=1)
    b = oracle.forward(x, threads=7)
    assert np.array_equal(a, b)


MUTANTS = list(range(1, 8))


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    from oracle import build as obuild
    d = tmp_path_factory.mktemp("mutants")
    libs = {}
    for m in MUTANTS:
        libs[m] = obuild.build(out=str(d / f"liboracle_m{m}.so"), mutant=m)
    return libs


@pytest.mark.parametrize("mutant", MUTANTS)
def test_pins_catch_planted_mistakes(mutant, mutant_libs):
    orc = Oracle(oracle._load(mutant_libs[mutant]))
    assert orc.mutant_id() == mutant
    caught = []
    for pin in PINS:
        try:
            pin(orc)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {mutant} passed every pin"


# ---------------------------------------------------------------- real input
# rfft / irfft and their adjoints are compositions over the complex oracle
# (Eq. (dft) of x + 0i, Hermitian extension, Eq. (idft)).  They get pins of
# their own, and planted mistakes in those compositions must fail one.

REAL_N = [2, 4, 8, 16, 64, 2048]


def _real_direct_forward(x):
    """Eq. (dft) for real x, bins 0..N/2 only, as an explicit O(N^2) sum."""
    n = x.shape[-1]
    kn = np.outer(np.arange(n // 2 + 1), np.arange(n)) % n
    return x @ np.exp(-2j * np.pi * kn / n).T


def _real_direct_inverse(X, n):
    """The textbook real inverse: x_j = (1/N)[Re X_0 + Re X_{N/2} (-1)^j
    + 2 sum_{0<k<N/2} Re(X_k e^{2 pi i jk/N})], as an explicit sum."""
    m = n // 2
    j = np.arange(n)
    out = X[..., :1].real + X[..., m:m + 1].real * ((-1.0) ** j)
    if m > 1:
        kj = np.outer(np.arange(1, m), j) % n
        out = out + 2.0 * (X[..., 1:m] @ np.exp(2j * np.pi * kj / n)).real
    return out / n


def rpin_brute_force(orc):
    for n in REAL_N[:5]:
        x = synth.uniform_complex(47, (3, n), key=(n,), dtype=np.complex128).real.copy()
        assert relerr(orc.rfft(x), _real_direct_forward(x)) < 1e-13, n
        X = synth.uniform_complex(47, (3, n // 2 + 1), key=(n, 1), dtype=np.complex128)
        assert relerr(orc.irfft(X, n), _real_direct_inverse(X, n)) < 1e-13, n


def rpin_numpy_library(orc):
    for n in REAL_N:
        x = synth.uniform_complex(53, (4, n), key=(n,), dtype=np.complex128).real.copy()
        assert relerr(orc.rfft(x), np.fft.rfft(x, axis=-1)) < 1e-13, n
        # edge bins with nonzero imaginary parts: numpy ignores them too
        X = synth.uniform_complex(53, (4, n // 2 + 1), key=(n, 1), dtype=np.complex128)
        assert relerr(orc.irfft(X, n), np.fft.irfft(X, n, axis=-1)) < 1e-13, n


def rpin_ramp_closed_form(orc):
    """The paper's f(x) = x is real: X_0 = N(N-1)/2, X_k = -N/2 + i (N/2) cot(pi k/N)."""
    for n in POW2_ALL:
        k = np.arange(1, n // 2 + 1)
        want = np.empty(n // 2 + 1, np.complex128)
        want[0] = n * (n - 1) / 2
        want[1:] = -n / 2 + 1j * (n / 2) * np.cos(np.pi * k / n) / np.sin(np.pi * k / n)
        got = orc.rfft(np.arange(n, dtype=np.float64))
        assert relerr(got, want) < 1e-13, n
        assert np.max(np.abs(orc.irfft(want, n) - np.arange(n))) < 1e-10 * n, n


def rpin_adjoint_identities(orc):
    """Re<R x, g> = <x, R^H g> and <C X, v> = Re<X, C^H v> (real inner products)."""
    for n in REAL_N:
        x = synth.uniform_complex(59, (3, n), key=(n, 0), dtype=np.complex128).real.copy()
        g = synth.uniform_complex(59, (3, n // 2 + 1), key=(n, 1), dtype=np.complex128)
        lhs = np.sum((orc.rfft(x) * np.conj(g)).real)
        rhs = np.sum(x * orc.rfft_adjoint(g, n))
        assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0), n
        X = synth.uniform_complex(59, (3, n // 2 + 1), key=(n, 2), dtype=np.complex128)
        v = synth.uniform_complex(59, (3, n), key=(n, 3), dtype=np.complex128).real.copy()
        lhs = np.sum(orc.irfft(X, n) * v)
        rhs = np.sum((X * np.conj(orc.irfft_adjoint(v))).real)
        assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1e-3), n


def rpin_gradient_fd(orc):
    """Finite differences of quadratic losses through rfft and irfft (exact up
    to rounding for any step) pin the adjoints in PyTorch's convention."""
    n, h = 16, 1e-2
    x = synth.uniform_complex(61, (2, n), dtype=np.complex128).real.copy()
    w = synth.uniform_weights(61, (2, n // 2 + 1), key=(1,), dtype=np.float64)
    g = orc.rfft_adjoint(2.0 * w * _real_direct_forward(x), n)
    fd = np.zeros_like(x)
    for b in range(2):
        for i in range(n):
            e = np.zeros_like(x)
            e[b, i] = h
            fd[b, i] = (np.sum(w * np.abs(_real_direct_forward(x + e)) ** 2)
                        - np.sum(w * np.abs(_real_direct_forward(x - e)) ** 2)) / (2 * h)
    assert relerr(g, fd) < 1e-11
    X = synth.uniform_complex(61, (2, n // 2 + 1), key=(2,), dtype=np.complex128)
    u = synth.uniform_weights(61, (2, n), key=(3,), dtype=np.float64)
    gX = orc.irfft_adjoint(2.0 * u * _real_direct_inverse(X, n))
    fdX = np.zeros_like(X)
    for b in range(2):
        for i in range(n // 2 + 1):
            for unit in (1.0, 1j):
                e = np.zeros_like(X)
                e[b, i] = unit * h
                d = (np.sum(u * _real_direct_inverse(X + e, n) ** 2)
                     - np.sum(u * _real_direct_inverse(X - e, n) ** 2)) / (2 * h)
                fdX[b, i] += unit * d
    assert relerr(gX, fdX) < 1e-11


REAL_PINS = [rpin_brute_force, rpin_numpy_library, rpin_ramp_closed_form,
             rpin_adjoint_identities, rpin_gradient_fd]


@pytest.mark.parametrize("pin", REAL_PINS, ids=lambda p: p.__name__)
def test_real_oracle_pin(pin):
    pin(Oracle())


class _ExtNoConj(Oracle):
    @staticmethod
    def hermitian_extension(X, n):
        full = Oracle.hermitian_extension(X, n)
        m = n // 2
        full[..., m + 1:] = X[..., 1:m][..., ::-1]
        return full


class _ExtMirrorOffByOne(Oracle):
    @staticmethod
    def hermitian_extension(X, n):
        full = Oracle.hermitian_extension(X, n)
        m = n // 2
        full[..., m + 1:] = np.conj(X[..., 2:m + 1][..., ::-1])
        return full


class _ExtNoReversal(Oracle):
    @staticmethod
    def hermitian_extension(X, n):
        full = Oracle.hermitian_extension(X, n)
        m = n // 2
        full[..., m + 1:] = np.conj(X[..., 1:m])
        return full


class _RfftAdjointWrongSign(Oracle):
    def rfft_adjoint(self, g, n, threads=None):
        padded = np.zeros(np.shape(g)[:-1] + (n,), np.complex128)
        padded[..., : n // 2 + 1] = g
        return self.fft(padded, -1, 1.0, threads).real


class _IrfftAdjointOneSided(Oracle):
    def irfft_adjoint(self, v, threads=None):
        out = Oracle.irfft_adjoint(self, v, threads)
        n = np.shape(v)[-1]
        Y = self.adjoint(np.asarray(v, np.complex128), +1, 1.0 / n, threads)
        out[..., 1:n // 2] = Y[..., 1:n // 2]
        return out


class _IrfftAdjointNoScale(Oracle):
    def irfft_adjoint(self, v, threads=None):
        return Oracle.irfft_adjoint(self, v, threads) * np.shape(v)[-1]


class _RfftDropsNyquist(Oracle):
    def rfft(self, x, threads=None):
        X = Oracle.rfft(self, x, threads)
        X[..., -1] = 0
        return X


REAL_MUTANTS = [_ExtNoConj, _ExtMirrorOffByOne, _ExtNoReversal, _RfftAdjointWrongSign,
                _IrfftAdjointOneSided, _IrfftAdjointNoScale, _RfftDropsNyquist]


@pytest.mark.parametrize("mutant", REAL_MUTANTS, ids=lambda m: m.__name__)
def test_real_pins_catch_planted_mistakes(mutant):
    orc = mutant()
    caught = []
    for pin in REAL_PINS:
        try:
            pin(orc)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"{mutant.__name__} passed every real-input pin"


# ---------------------------------------------------------------- multidimensional
def _direct_dft2(x, sign):
    """The 2D DFT as one explicit double sum over (n1, n2) for each (k1, k2),
    the exponents k_a n_a reduced modulo N_a in integers."""
    n1, n2 = x.shape[-2:]
    out = np.zeros(x.shape, np.complex128)
    a1 = np.arange(n1)
    a2 = np.arange(n2)
    for k1 in range(n1):
        for k2 in range(n2):
            ph = (np.outer((k1 * a1) % n1, np.ones(n2)) / n1 + np.outer(np.ones(n1), (k2 * a2) % n2) / n2)
            out[..., k1, k2] = np.sum(x * np.exp(sign * 2j * np.pi * ph), axis=(-2, -1))
    return out


def npin_brute_force(orc):
    for shape in ((2, 2), (4, 8), (8, 2), (16, 4)):
        x = synth.uniform_complex(67, (3,) + shape, key=shape, dtype=np.complex128)
        assert relerr(orc.fftn(x, 2), _direct_dft2(x, -1)) < 1e-13, shape
        n = shape[0] * shape[1]
        assert relerr(orc.fftn(x, 2, +1, 1.0 / n), _direct_dft2(x, +1) / n) < 1e-13, shape


def npin_numpy_library(orc):
    for shape in ((32, 64), (2, 1024), (8, 4, 16), (2, 2, 2)):
        x = synth.uniform_complex(71, (2,) + shape, key=shape, dtype=np.complex128)
        axes = tuple(range(1, 1 + len(shape)))
        assert relerr(orc.fftn(x, len(shape)), np.fft.fftn(x, axes=axes)) < 1e-13, shape
        n = int(np.prod(shape))
        assert relerr(orc.fftn(x, len(shape), +1, 1.0 / n), np.fft.ifftn(x, axes=axes)) < 1e-13, shape


def npin_separable_and_invariants(orc):
    """An outer product of 1D signals has the outer product of their 1D
    spectra; impulses give plane waves; Parseval; round trip."""
    for n1, n2 in ((8, 16), (64, 32)):
        u = synth.uniform_complex(73, (n1,), key=(n1, n2, 0), dtype=np.complex128)
        v = synth.uniform_complex(73, (n2,), key=(n1, n2, 1), dtype=np.complex128)
        want = np.outer(np.fft.fft(u), np.fft.fft(v))
        assert relerr(orc.fftn(np.outer(u, v), 2), want) < 1e-13
        x = np.zeros((n1, n2), np.complex128)
        x[3, 5] = 1.0
        k1, k2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
        plane = np.exp(-2j * np.pi * (((3 * k1) % n1) / n1 + ((5 * k2) % n2) / n2))
        assert np.max(np.abs(orc.fftn(x, 2) - plane)) < 1e-13
        y = synth.uniform_complex(73, (2, n1, n2), key=(n1, n2, 2), dtype=np.complex128)
        Y = orc.fftn(y, 2)
        assert np.max(np.abs(np.sum(np.abs(Y) ** 2, axis=(1, 2)) / (n1 * n2 * np.sum(np.abs(y) ** 2, axis=(1, 2))) - 1)) < 1e-13
        assert relerr(orc.fftn(Y, 2, +1, 1.0 / (n1 * n2)), y) < 1e-14


ND_PINS = [npin_brute_force, npin_numpy_library, npin_separable_and_invariants]


@pytest.mark.parametrize("pin", ND_PINS, ids=lambda p: p.__name__)
def test_nd_oracle_pin(pin):
    pin(Oracle())


class _NdSkipsFirstAxis(Oracle):
    def fftn(self, x, ndim, sign=-1, scale=1.0, threads=None):
        return Oracle.fftn(self, x, ndim - 1, sign, scale, threads)


class _NdSwapsSign(Oracle):
    def fftn(self, x, ndim, sign=-1, scale=1.0, threads=None):
        y = np.asarray(x, dtype=np.complex128)
        for i, ax in enumerate(range(y.ndim - ndim, y.ndim)):
            moved = np.moveaxis(y, ax, -1)
            y = np.moveaxis(self.fft(moved, sign if i else -sign, 1.0, threads), -1, ax)
        return y * scale


class _NdTransposesResult(Oracle):
    def fftn(self, x, ndim, sign=-1, scale=1.0, threads=None):
        y = Oracle.fftn(self, x, ndim, sign, scale, threads)
        return np.swapaxes(y, -1, -2).reshape(y.shape)


@pytest.mark.parametrize("mutant", [_NdSkipsFirstAxis, _NdSwapsSign, _NdTransposesResult],
                         ids=lambda m: m.__name__)
def test_nd_pins_catch_planted_mistakes(mutant):
    orc = mutant()
    caught = []
    for pin in ND_PINS:
        try:
            pin(orc)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"{mutant.__name__} passed every multidimensional pin"
