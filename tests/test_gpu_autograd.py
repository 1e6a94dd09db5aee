"""Differentiable FFT: loss = sum(w * |FFT(x)|^2), backward through the
hand-written adjoint kernel.

Gradient convention (PyTorch, complex input): x.grad = dL/dRe x + i dL/dIm x
= F^H (2 w * F x).  Pins: FP64 central finite differences (exact for a
quadratic loss up to rounding) at N = 16, batch 4; the oracle's adjoint at
the full N = 2048, batch 16384 size on sampled transforms; the adjoint
identity <F x, y> = <x, F^H y>.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from gpu_util import need_gpu, per_transform_relerr, to_cpu, to_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def gpu_loss_grad(x_np, w_np):
    x = to_gpu(x_np).requires_grad_(True)
    w = to_gpu(w_np)
    y = api.fft_differentiable(x)
    loss = (w * (y.real ** 2 + y.imag ** 2)).sum()
    loss.backward()
    torch.cuda.synchronize()
    return float(loss), x.grad.cpu().numpy()


def test_gradient_vs_fp64_finite_differences():
    n, batch, h = 16, 4, 1e-2
    x = synth.uniform_complex(synth.SEED_AUTOGRAD, (batch, n))
    w = synth.uniform_weights(synth.SEED_AUTOGRAD, (batch, n), key=(1,))
    _, g = gpu_loss_grad(x, w)
    x64, w64 = x.astype(np.complex128), w.astype(np.float64)

    def loss(z):
        return float(np.sum(w64 * np.abs(oracle.forward(z)) ** 2))

    fd = np.zeros_like(x64)
    for b in range(batch):
        for i in range(n):
            for unit in (1.0, 1j):
                e = np.zeros_like(x64)
                e[b, i] = unit * h
                fd[b, i] += unit * (loss(x64 + e) - loss(x64 - e)) / (2 * h)
    assert per_transform_relerr(g, fd) <= TOL


def test_full_size_gradient_vs_oracle_adjoint():
    n, batch = 2048, 16384
    x = synth.uniform_complex(synth.SEED_AUTOGRAD, (batch, n))
    w = synth.uniform_weights(synth.SEED_AUTOGRAD, (batch, n), key=(1,))
    print(f"[case] autograd full n={n} batch={batch}", flush=True)
    loss, g = gpu_loss_grad(x, w)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([[0, batch - 1], rng.integers(0, batch, 62)]))
    _, g_ref = oracle.loss_grad(x[idx].astype(np.complex128), w[idx].astype(np.float64))
    assert per_transform_relerr(g[idx], g_ref) <= TOL
    # the loss itself, against the oracle on the whole batch in chunks
    ref_loss = 0.0
    for c in range(0, batch, 4096):
        ref_loss += oracle.loss_grad(x[c:c + 4096].astype(np.complex128),
                                     w[c:c + 4096].astype(np.float64))[0]
    assert abs(loss - ref_loss) / ref_loss < 1e-5


@pytest.mark.parametrize("n", [2, 16, 256, 2048])
@pytest.mark.parametrize("sign", [-1, 1])
def test_adjoint_identity(n, sign):
    batch = 64
    x = to_gpu(synth.uniform_complex(29, (batch, n), key=(n, 0)))
    y = to_gpu(synth.uniform_complex(29, (batch, n), key=(n, 1)))
    p = api.Plan(n, batch, sign)
    Ax = to_cpu(p.execute(x)).astype(np.complex128)
    AHy = to_cpu(p.adjoint(y)).astype(np.complex128)
    lhs = np.vdot(to_cpu(y).astype(np.complex128), Ax)
    rhs = np.vdot(AHy, to_cpu(x).astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("n", [16, 2048])
def test_adjoint_kernel_vs_oracle(n):
    batch = 97
    g = synth.uniform_complex(31, (batch, n))
    for sign in (-1, 1):
        p = api.Plan(n, batch, sign)
        got = to_cpu(p.adjoint(to_gpu(g)))
        scale = 1.0 if sign < 0 else 1.0 / n
        ref = oracle.adjoint(g.astype(np.complex128), sign, scale)
        assert per_transform_relerr(got, ref) <= TOL


def test_inverse_fft_differentiable():
    """Gradient through the inverse transform uses its adjoint (sign -1, 1/n)."""
    n, batch = 64, 8
    x = synth.uniform_complex(37, (batch, n))
    w = synth.uniform_weights(37, (batch, n), key=(1,))
    xg = to_gpu(x).requires_grad_(True)
    y = api.fft_differentiable(xg, +1)
    ((to_gpu(w) * (y.real ** 2 + y.imag ** 2)).sum()).backward()
    x64 = x.astype(np.complex128)
    yy = oracle.inverse(x64)
    ref = oracle.adjoint(2.0 * w * yy, sign=+1, scale=1.0 / n)
    assert per_transform_relerr(xg.grad.cpu().numpy(), ref) <= TOL
