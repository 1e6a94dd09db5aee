"""CPU emulation of the FP16/BF16 pipeline's rounding, to predict its error
budget independently of the GPU kernel.

The emulated pipeline (N = 2048 = 8 * 16 * 16): stored half-precision input
scaled by a power of two to max component in [8, 16); radix-8 pass in FP32;
FP32 twiddles; two radix-16 passes whose operands (data and DFT matrix) are
rounded to the operand type (the kernel uses FP16 for both storage types;
BF16 operands split into hi + lo are modelled for comparison), with products
accumulated in FP32; output rounded to the storage type.  The reference is
numpy's FP64 FFT of the stored input (the method's own error), and the raw
FP64 draw is the second column.  Bar: 3e-3 relative L2 per transform.
"""
import numpy as np
import pytest

from paper_2203_09384_amd import synth

N = 2048


def bf16_round(x):
    """float32 -> nearest-even bfloat16, returned as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def q(x, kind):
    x = np.asarray(x, np.float32)
    if kind == "f16":
        return x.astype(np.float16).astype(np.float32)
    return bf16_round(x)


def quant_parts(x, kind, split):
    hi = q(x, kind)
    if not split:
        return [hi]
    return [hi, q(x - hi, kind)]


def emulate(xs, kind, split, op_kind=None):
    """xs: (batch, N) complex, already the stored input (as float64); kind
    is the storage type, op_kind the MFMA operand type (default: kind)."""
    op_kind = op_kind or kind
    out = np.empty_like(xs)
    n = np.arange(16)
    F = np.exp(-2j * np.pi * np.outer(n, n) / 16)
    Fr = quant_parts(F.real, op_kind, split)
    Fi = quant_parts(F.imag, op_kind, split)
    k8 = np.arange(8)
    F8 = np.exp(-2j * np.pi * np.outer(k8, k8) / 8)
    for b, x in enumerate(xs):
        mx = max(np.abs(x.real).max(), np.abs(x.imag).max())
        e = int(np.frexp(mx)[1]) if mx > 0 else 0
        v = (x * 2.0 ** (4 - e)).astype(np.complex64)
        # pass A: radix 8 over x[j + 256 r]
        a = v.reshape(8, 256)
        y = (F8.astype(np.complex64) @ a).astype(np.complex64)  # y[m, j]
        # Stockham layout after pass A: d = 8 j + m
        z = y.T.reshape(-1)
        # pass B input z[j + 128 r], twiddle w_128^{r (j mod 8)}
        for ns in (8, 128):
            zz = z.reshape(16, 128)  # [r, j]
            j = np.arange(128)
            r = np.arange(16)[:, None]
            tw = np.exp(-2j * np.pi * (r * (j % ns)) / (ns * 16)).astype(np.complex64)
            zz = (zz * tw).astype(np.complex64)
            Xr = quant_parts(zz.real, op_kind, split)
            Xi = quant_parts(zz.imag, op_kind, split)

            def prod(A, B):  # hi*hi + hi*lo + lo*hi, accumulated in fp64 then fp32
                s = A[0].astype(np.float64) @ B[0].astype(np.float64)
                if split:
                    s = s + A[0].astype(np.float64) @ B[1].astype(np.float64)
                    s = s + A[1].astype(np.float64) @ B[0].astype(np.float64)
                return s.astype(np.float32)
            Yr = prod(Fr, Xr) - prod(Fi, Xi)
            Yi = prod(Fi, Xr) + prod(Fr, Xi)
            Y = (Yr + 1j * Yi).astype(np.complex64)  # [m, j]
            nxt = np.empty(2048, np.complex64)
            jj = np.arange(128)
            for m in range(16):
                d = ((jj // ns) * ns * 16) + (jj % ns) + m * ns
                nxt[d] = Y[m]
            z = nxt
        yo = q(z.real, kind) + 1j * q(z.imag, kind)
        out[b] = yo.astype(np.complex128) * 2.0 ** (e - 4)
    return out


def rel(y, ref):
    return np.max(np.linalg.norm(y - ref, axis=-1) / np.linalg.norm(ref, axis=-1))


def inputs(cls, batch):
    if cls == "uniform":
        return synth.uniform_complex(synth.SEED_HALF, (batch, N), key=(0,), dtype=np.complex128)
    return synth.log_uniform_polar(synth.SEED_HALF, (batch, N), key=(1,))


def stored(x, kind):
    return (q(x.real, kind) + 1j * q(x.imag, kind)).astype(np.complex128)


@pytest.mark.parametrize("kind,limit", [("f16", 1e-3), ("bf16", 2.8e-3)])
@pytest.mark.parametrize("cls", ["uniform", "loguniform"])
def test_emulated_error_within_budget(kind, limit, cls):
    """The kernel as built: FP16 MFMA operands for both storage types."""
    x = inputs(cls, 8)
    xs = stored(x, kind)
    y = emulate(xs, kind, False, op_kind="f16")
    e_method = rel(y, np.fft.fft(xs, axis=-1))
    e_raw = rel(y, np.fft.fft(x, axis=-1))
    print(f"{kind} storage, f16 operands, {cls}: vs stored input {e_method:.2e}, vs raw draw {e_raw:.2e}")
    assert e_method <= limit


@pytest.mark.parametrize("cls", ["uniform", "loguniform"])
def test_bf16_storage_fp16_operands_match_split_bf16(cls):
    """For BF16 storage the output rounding sets the error: FP16 operands
    (one MFMA per product) are within 5% of BF16 operands split hi + lo
    (three MFMAs per product), and far below single BF16 operands."""
    x = inputs(cls, 8)
    xs = stored(x, "bf16")
    ref = np.fft.fft(xs, axis=-1)
    e_f16 = rel(emulate(xs, "bf16", False, op_kind="f16"), ref)
    e_split = rel(emulate(xs, "bf16", True), ref)
    e_single = rel(emulate(xs, "bf16", False), ref)
    print(f"bf16 {cls}: f16 operands {e_f16:.2e}, bf16 hi/lo {e_split:.2e}, bf16 single {e_single:.2e}")
    assert e_f16 <= 1.05 * e_split
    assert e_f16 < e_single


def test_emulator_is_an_fft_without_rounding():
    """With rounding switched off the emulated data flow is an exact DFT."""
    global q
    saved = q
    try:
        q = lambda x, kind: np.asarray(x, np.float32)  # noqa: E731
        x = inputs("uniform", 2)
        y = emulate(x, "f16", False)
        assert rel(y, np.fft.fft(x, axis=-1)) < 1e-6
    finally:
        q = saved
