"""Real-input transforms (R2C / C2R) on the GPU against the FP64 oracle.

The oracle's rfft / irfft are Eq. (dft) of x + 0i restricted to bins
0..n/2 and Eq. (idft) of the Hermitian extension (pinned in the oracle's own
tests).  Bar: max over transforms of the relative L2 error <= 1e-5, as for
the complex FP32 path.  Every length 2..2^21 runs with its built-in
configuration at a batch that leaves a partial last workgroup (above 2^15:
the four-step half-length transform plus the split pass); every compiled
configuration of a few lengths runs too.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from paper_2203_09384_amd.native import MifftError
from gpu_util import need_gpu, per_transform_relerr, to_cpu, to_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5
LS = list(range(1, 22))


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def batch_for(n):
    """Several workgroups of transforms plus a ragged tail, bounded in size."""
    return max(3, min(3 * max(1, 4096 // n), 200)) + 1


def bins(seed, batch, n, key=()):
    """Spectrum-side inputs: n/2 + 1 complex bins, edge bins with nonzero
    imaginary parts (the inverse must ignore them)."""
    return synth.uniform_complex(seed, (batch, n // 2 + 1), key=key)


@pytest.mark.parametrize("L", LS)
def test_r2c_default(L):
    n = 1 << L
    batch = batch_for(n)
    x = synth.uniform_real(synth.SEED_REAL, (batch, n), key=(n,))
    p = api.Plan(n, batch, -1, "r32")
    print(f"[case] r2c n={n} batch={batch} {p.describe()}", flush=True)
    y = to_cpu(p.execute(to_gpu(x)))
    assert y.shape == (batch, n // 2 + 1)
    assert per_transform_relerr(y, oracle.rfft(x.astype(np.float64))) <= TOL


@pytest.mark.parametrize("L", LS)
def test_c2r_default(L):
    n = 1 << L
    batch = batch_for(n)
    X = bins(synth.SEED_REAL, batch, n, key=(n, 1))
    p = api.Plan(n, batch, +1, "r32")
    print(f"[case] c2r n={n} batch={batch} {p.describe()}", flush=True)
    y = to_cpu(p.execute(to_gpu(X)))
    assert y.shape == (batch, n)
    assert per_transform_relerr(y, oracle.irfft(X.astype(np.complex128), n)) <= TOL


@pytest.mark.parametrize("L", LS)
def test_adjoints(L):
    n = 1 << L
    batch = batch_for(n)
    g = bins(synth.SEED_REAL, batch, n, key=(n, 2))
    v = synth.uniform_real(synth.SEED_REAL, (batch, n), key=(n, 3))
    pf = api.Plan(n, batch, -1, "r32")
    pi = api.Plan(n, batch, +1, "r32")
    print(f"[case] real adjoints n={n} batch={batch}", flush=True)
    got = to_cpu(pf.adjoint(to_gpu(g)))
    assert per_transform_relerr(got, oracle.rfft_adjoint(g.astype(np.complex128), n)) <= TOL
    got = to_cpu(pi.adjoint(to_gpu(v)))
    assert per_transform_relerr(got, oracle.irfft_adjoint(v.astype(np.float64))) <= TOL


def real_configs(L):
    """The compiled menu of the real-input kernels for half length 2^(L-1)."""
    lm = L - 1
    out = []
    for e in range(1, 5):
        if e > lm:
            continue
        if e == lm:
            if lm <= 4:
                out += [(1 << e, wg, 0) for wg in (64, 128, 256)]
            continue
        if e < 2:
            continue
        tpt = (1 << lm) >> e
        wgs = [tpt] if lm > 11 else [w for w in (64, 128, 256) if tpt <= w]
        if lm > 11 and (e < 3 or tpt > 1024):
            continue
        for wg in wgs:
            kinds = [2, 3] + ([6, 7] if tpt <= 64 else [])
            out += [(1 << e, wg, k) for k in kinds]
    return out


def _lds_estimate(L, ept, wg):
    m = 1 << (L - 1)
    tpt = max(1, m // ept)
    return (wg // tpt) * m * 8


@pytest.mark.parametrize("L", [3, 5, 8, 11, 12, 14])
def test_every_config(L):
    n = 1 << L
    batch = batch_for(n)
    x = synth.uniform_real(synth.SEED_REAL, (batch, n), key=(n, 4))
    X = bins(synth.SEED_REAL, batch, n, key=(n, 5))
    ref_f = oracle.rfft(x.astype(np.float64))
    ref_i = oracle.irfft(X.astype(np.complex128), n)
    tried = 0
    for ept, wg, kind in real_configs(L):
        try:
            pf = api.Plan(n, batch, -1, "r32", ept=ept, wg=wg, variant=kind)
            pi = api.Plan(n, batch, +1, "r32", ept=ept, wg=wg, variant=kind)
        except MifftError as e:
            # only configurations over the LDS budget may be missing
            assert e.code == 10 and _lds_estimate(L, ept, wg) > 56 * 1024, (ept, wg, kind)
            continue
        print(f"[case] real config n={n} ept={ept} wg={wg} kind={kind}", flush=True)
        assert per_transform_relerr(to_cpu(pf.execute(to_gpu(x))), ref_f) <= TOL, (ept, wg, kind)
        assert per_transform_relerr(to_cpu(pi.execute(to_gpu(X))), ref_i) <= TOL, (ept, wg, kind)
        tried += 1
    assert tried > 0


def test_paper_ramp_closed_form():
    """The paper's f(x) = x is real: X_0 = N(N-1)/2, X_k = -N/2 + i (N/2) cot(pi k/N)."""
    for n in (8, 256, 2048, 1 << 15, 1 << 18):
        k = np.arange(1, n // 2 + 1)
        want = np.empty(n // 2 + 1, np.complex128)
        want[0] = n * (n - 1) / 2
        want[1:] = -n / 2 + 1j * (n / 2) * np.cos(np.pi * k / n) / np.sin(np.pi * k / n)
        x = np.arange(n, dtype=np.float32)[None]
        y = to_cpu(api.Plan(n, 1, -1, "r32").execute(to_gpu(x)))
        assert per_transform_relerr(y, want[None]) <= TOL, n


def test_full_size_sampled():
    """n = 2048, batch 2^16 (512 MiB of reals): sampled transforms against
    the oracle, and the round trip over the whole batch."""
    n, batch = 2048, 1 << 16
    x = synth.uniform_real(synth.SEED_REAL, (batch, n), key=(7,))
    xg = to_gpu(x)
    print(f"[case] real full size n={n} batch={batch}", flush=True)
    y = api.Plan(n, batch, -1, "r32").execute(xg)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, batch - 1], rng.integers(0, batch, 62)]))
    ys = to_cpu(y[torch.as_tensor(idx, device=y.device)])
    assert per_transform_relerr(ys, oracle.rfft(x[idx].astype(np.float64))) <= TOL
    back = api.Plan(n, batch, +1, "r32").execute(y)
    assert per_transform_relerr(to_cpu(back), x) <= 2 * TOL


def test_inverse_is_bitwise_adjoint_scaled():
    """The inverse (bin weights 1/n) and the adjoint of the forward plan
    (weights 1 at the edge bins, 1/2 inside) run the same C2R kernel: fed
    the same spectrum, with the interior bins doubled for the adjoint, the
    two results differ by exactly the power-of-two factor n."""
    n, batch = 512, 33
    X = bins(synth.SEED_REAL, batch, n, key=(8,))
    X[:, 0] = X[:, 0].real
    X[:, -1] = X[:, -1].real
    pi = api.Plan(n, batch, +1, "r32")
    pf = api.Plan(n, batch, -1, "r32")
    a = to_cpu(pi.execute(to_gpu(X)))
    Xw = X.copy()
    Xw[:, 1:-1] *= 2
    b = to_cpu(pf.adjoint(to_gpu(Xw)))
    assert np.array_equal(a * n, b)


def test_autograd_rfft_irfft():
    """Gradients through rfft and irfft against the oracle's adjoints and
    exact central differences (quadratic losses)."""
    n, batch = 64, 5
    x = synth.uniform_real(synth.SEED_REAL, (batch, n), key=(9,))
    w = synth.uniform_weights(synth.SEED_REAL, (batch, n // 2 + 1), key=(10,))
    xg = to_gpu(x).requires_grad_(True)
    Y = api.rfft_differentiable(xg)
    (to_gpu(w) * (Y.real ** 2 + Y.imag ** 2)).sum().backward()
    x64, w64 = x.astype(np.float64), w.astype(np.float64)
    ref = oracle.rfft_adjoint(2.0 * w64 * oracle.rfft(x64), n)
    assert per_transform_relerr(xg.grad.cpu().numpy(), ref) <= TOL
    X = bins(synth.SEED_REAL, batch, n, key=(11,))
    u = synth.uniform_weights(synth.SEED_REAL, (batch, n), key=(12,))
    Xg = to_gpu(X).requires_grad_(True)
    y = api.irfft_differentiable(Xg, n)
    (to_gpu(u) * y ** 2).sum().backward()
    X64 = X.astype(np.complex128)
    ref = oracle.irfft_adjoint(2.0 * u.astype(np.float64) * oracle.irfft(X64, n))
    assert per_transform_relerr(Xg.grad.cpu().numpy(), ref) <= TOL
    # central differences of the rfft loss in FP64 through the oracle
    h = 1e-2

    def loss(z):
        return float(np.sum(w64 * np.abs(oracle.rfft(z)) ** 2))

    fd = np.zeros_like(x64)
    for b in range(2):
        for i in range(n):
            e = np.zeros_like(x64)
            e[b, i] = h
            fd[b, i] = (loss(x64 + e) - loss(x64 - e)) / (2 * h)
    assert per_transform_relerr(xg.grad.cpu().numpy()[:2], fd[:2]) <= TOL


def test_functional_api_shapes():
    x = to_gpu(synth.uniform_real(synth.SEED_REAL, (2, 3, 128), key=(13,)))
    X = api.rfft(x)
    assert X.shape == (2, 3, 65) and X.dtype == torch.complex64
    y = api.irfft(X)
    assert y.shape == (2, 3, 128) and y.dtype == torch.float32
    assert per_transform_relerr(to_cpu(y), to_cpu(x)) <= 2 * TOL
    with pytest.raises(ValueError):
        api.irfft(X, 100)


def test_overlap_and_size_checks():
    n, batch = 256, 8
    p = api.Plan(n, batch, -1, "r32")
    buf = torch.empty(4 * n * batch, dtype=torch.float32, device="cuda")
    import ctypes
    from paper_2203_09384_amd.native import lib
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    base = buf.data_ptr()
    # spectrum side of 8 * 129 bins starting 4 KiB after the reals: overlaps
    rc = lib().fft_execute(p._h, ctypes.c_void_p(base), ctypes.c_void_p(base + 4096), s)
    assert rc == 6
    # disjoint
    rc = lib().fft_execute(p._h, ctypes.c_void_p(base), ctypes.c_void_p(base + 4 * n * batch), s)
    assert rc == 0
    with pytest.raises(ValueError):
        p.execute(torch.empty(batch, n, dtype=torch.complex64, device="cuda"))
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [16, 2048, 1 << 15])
def test_run_to_run_bitwise(n):
    """No atomics on data: repeated executes give identical bits."""
    batch = 37
    x = to_gpu(synth.uniform_real(synth.SEED_REAL, (batch, n), key=(n, 20)))
    pf, pi = api.Plan(n, batch, -1, "r32"), api.Plan(n, batch, +1, "r32")
    X0 = pf.execute(x)
    x0 = pi.execute(X0)
    for _ in range(3):
        assert torch.equal(pf.execute(x), X0)
        assert torch.equal(pi.execute(X0), x0)
