"""Lengths 2^12 .. 2^20 (FP32, four-step: column and row passes) against the
FP64 oracle; bar: per-transform relative L2 <= 1e-5."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from gpu_util import need_gpu, per_transform_relerr, to_cpu, to_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5
LS = list(range(12, 21))


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("L", LS)
@pytest.mark.parametrize("sign", [-1, 1])
def test_large_parity(L, sign):
    n = 1 << L
    batch = max(2, (1 << 22) // n) + 1
    x = synth.uniform_complex(61, (batch, n), key=(L, sign + 1))
    p = api.Plan(n, batch, sign)
    print(f"[case] large n={n} batch={batch} sign={sign} {p.describe()}", flush=True)
    y = to_cpu(p.execute(to_gpu(x)))
    x64 = x.astype(np.complex128)
    ref = oracle.forward(x64) if sign < 0 else oracle.inverse(x64)
    assert per_transform_relerr(y, ref) <= TOL


@pytest.mark.parametrize("L", [12, 16, 20])
def test_large_adjoint_and_roundtrip(L):
    n = 1 << L
    batch = 3
    x = synth.uniform_complex(63, (batch, n), key=(L,))
    xg = to_gpu(x)
    p = api.Plan(n, batch, -1)
    adj = to_cpu(p.adjoint(xg))
    assert per_transform_relerr(adj, oracle.adjoint(x.astype(np.complex128), -1, 1.0)) <= TOL
    back = api.Plan(n, batch, +1).execute(p.execute(xg))
    assert per_transform_relerr(to_cpu(back), x) <= 2 * TOL


def test_large_ramp_closed_form():
    """The paper's f(x) = x at N = 2^16."""
    n = 1 << 16
    y = to_cpu(api.Plan(n, 1, -1).execute(to_gpu(synth.ramp(n, 1))))
    k = np.arange(1, n)
    want = np.empty(n, np.complex128)
    want[0] = n * (n - 1) / 2
    want[1:] = -n / 2 + 1j * (n / 2) / np.tan(np.pi * k / n)
    assert per_transform_relerr(y, want[None]) <= TOL


def test_large_full_size_sampled():
    """2^26 elements at N = 2^20 (64 transforms) and N = 2^16 (1024 transforms)."""
    for L in (16, 20):
        n = 1 << L
        batch = (1 << 26) // n
        x_np = synth.uniform_complex(65, (batch, n), key=(L,))
        y = api.Plan(n, batch, -1).execute(to_gpu(x_np))
        torch.cuda.synchronize()
        idx = np.unique(np.array([0, batch // 3, batch - 1]))
        ys = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        assert per_transform_relerr(ys, oracle.forward(x_np[idx].astype(np.complex128))) <= TOL


@pytest.mark.parametrize("L", [12, 13, 14])
@pytest.mark.parametrize("sign", [-1, 1])
def test_forced_four_step(L, sign):
    """The four-step split (variant 9) at the lengths that default to the
    single-pass kernels."""
    n = 1 << L
    batch = 5
    x = synth.uniform_complex(67, (batch, n), key=(L, sign + 1))
    p = api.Plan(n, batch, sign, ept=2, wg=64, variant=9)
    assert p.describe()["variant"] == 9
    print(f"[case] forced four-step n={n} sign={sign}", flush=True)
    y = to_cpu(p.execute(to_gpu(x)))
    x64 = x.astype(np.complex128)
    ref = oracle.forward(x64) if sign < 0 else oracle.inverse(x64)
    assert per_transform_relerr(y, ref) <= TOL
