"""Seeded random sweep over every plan kind against the FP64 oracle.

The systematic tests walk each length and variant at chosen batches; this
sweep draws (length, batch, sign, dtype) combinations from one seeded
generator, with batch 1 and odd batches that leave a partial last
workgroup, and runs the transform and its adjoint through the Python
binding.  Bars as elsewhere: FP32 relative L2 per transform <= 1e-5;
FP16/BF16 3e-3 at N = 2048, below it the rounding of the stored output
(2^-11 FP16, 2^-8 BF16) plus 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from gpu_util import need_gpu, per_transform_relerr, to_cpu, to_gpu

pytestmark = pytest.mark.gpu
SEED = 20221203
TOL32 = 1e-5
HALF_TOL = {"c16": 2.0 ** -11 + 1e-5, "cbf16": 2.0 ** -8 + 1e-5}
TORCH = {"c16": torch.float16, "cbf16": torch.bfloat16}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _cases(kind, count):
    g = np.random.default_rng([SEED, kind])
    out = []
    for i in range(count):
        if kind == 0:    # FP32 complex, single pass and four-step
            L = int(g.integers(1, 18))
        elif kind == 1:  # FP16 / BF16
            L = int(g.integers(1, 12))
        elif kind == 2:  # real input
            L = int(g.integers(1, 18))
        else:            # 2D
            L = (int(g.integers(1, 9)), int(g.integers(1, 9)))
        n_elems = (1 << L) if kind != 3 else (1 << (L[0] + L[1]))
        cap = max(1, min(300, (1 << 21) // n_elems))
        batch = 1 if i % 5 == 0 else int(g.integers(1, cap + 1))
        sign = -1 if g.integers(0, 2) == 0 else 1
        out.append((i, L, batch, sign))
    return out


@pytest.mark.parametrize("i,L,batch,sign", _cases(0, 24))
def test_c32_random(i, L, batch, sign):
    n = 1 << L
    x = synth.uniform_complex(SEED, (batch, n), key=(0, i))
    p = api.Plan(n, batch, sign)
    print(f"[case] c32 n={n} batch={batch} sign={sign} {p.describe()}", flush=True)
    xg = to_gpu(x)
    y = to_cpu(p.execute(xg))
    x64 = x.astype(np.complex128)
    ref = oracle.forward(x64) if sign < 0 else oracle.inverse(x64)
    assert per_transform_relerr(y, ref) <= TOL32
    # adjoint: opposite sign at the plan's scale
    a = to_cpu(p.adjoint(xg))
    assert per_transform_relerr(a, oracle.adjoint(x64, sign, 1.0 if sign < 0 else 1.0 / n)) <= TOL32


@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
@pytest.mark.parametrize("i,L,batch,sign", _cases(1, 10))
def test_half_random(dtype, i, L, batch, sign):
    n = 1 << L
    x = synth.uniform_complex(SEED, (batch, n), key=(1, i), dtype=np.complex128)
    xh = torch.from_numpy(np.stack([x.real, x.imag], -1).astype(np.float32)).to(TORCH[dtype]).cuda().contiguous()
    p = api.Plan(n, batch, sign, dtype=dtype)
    print(f"[case] {dtype} n={n} batch={batch} sign={sign} {p.describe()}", flush=True)
    yh, ex = p.execute_scaled(xh)
    torch.cuda.synchronize()
    a = yh.float().cpu().numpy().astype(np.float64)
    y = (a[..., 0] + 1j * a[..., 1]) * np.exp2(ex.cpu().numpy().astype(np.float64))[:, None]
    s = xh.float().cpu().numpy().astype(np.float64)
    stored = s[..., 0] + 1j * s[..., 1]
    ref = oracle.forward(stored) if sign < 0 else oracle.inverse(stored)
    tol = 3e-3 if n == 2048 else HALF_TOL[dtype]
    assert per_transform_relerr(y, ref) <= tol


@pytest.mark.parametrize("i,L,batch,sign", _cases(2, 16))
def test_real_random(i, L, batch, sign):
    n = 1 << L
    p = api.Plan(n, batch, sign, "r32")
    print(f"[case] r32 n={n} batch={batch} sign={sign} {p.describe()}", flush=True)
    if sign < 0:
        x = synth.uniform_real(SEED, (batch, n), key=(2, i))
        y = to_cpu(p.execute(to_gpu(x)))
        ref = oracle.rfft(x.astype(np.float64))
    else:
        X = synth.uniform_complex(SEED, (batch, n // 2 + 1), key=(2, i))
        y = to_cpu(p.execute(to_gpu(X)))
        ref = oracle.irfft(X.astype(np.complex128), n)
    assert per_transform_relerr(y, ref) <= TOL32


@pytest.mark.parametrize("i,L,batch,sign", _cases(3, 12))
def test_2d_random(i, L, batch, sign):
    shape = (1 << L[0], 1 << L[1])
    x = synth.uniform_complex(SEED, (batch,) + shape, key=(3, i))
    p = api.PlanND(shape, batch, sign)
    print(f"[case] 2d shape={shape} batch={batch} sign={sign} {p.describe()}", flush=True)
    y = to_cpu(p.execute(to_gpu(x)))
    scale = 1.0 if sign < 0 else 1.0 / (shape[0] * shape[1])
    ref = oracle.fftn(x.astype(np.complex128), 2, sign, scale)
    assert per_transform_relerr(y.reshape(batch, -1), ref.reshape(batch, -1)) <= TOL32
