"""FP32 batched path on the GPU, checked element by element against the FP64 oracle.

Bar: max over transforms of the relative L2 error <= 1e-5 (single precision
C2C against the exact DFT).  Inputs are the seeded generators' values; the
oracle reads exactly the stored complex64 values.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from gpu_util import need_gpu, per_transform_relerr, to_cpu, to_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5
NS = [1 << L for L in range(1, 12)]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def run(plan, x_np):
    print(f"[case] n={plan.n} batch={plan.batch} sign={plan.sign} {plan.describe()}", flush=True)
    y = plan.execute(to_gpu(x_np))
    return to_cpu(y)


def oracle_ref(x, sign):
    x = x.astype(np.complex128)
    return oracle.forward(x) if sign < 0 else oracle.inverse(x)


def test_twiddle_table():
    p = api.Plan(2048, 1, -1)
    tw = p.twiddles().cpu().numpy()
    m = np.arange(2048)
    exact = np.exp(-2j * np.pi * m / 2048)
    # one rounding of the exact value to FP32 per component
    assert np.max(np.abs(tw.real - exact.real)) <= 2 ** -24
    assert np.max(np.abs(tw.imag - exact.imag)) <= 2 ** -24
    # quarter-period identity of Eq. (twiddle), bit for bit: w^{m+512} = -i w^m
    q = tw[:1536]
    r = tw[512:]
    assert np.array_equal(r.real, q.imag) and np.array_equal(r.imag, -q.real)
    assert tw[0] == 1 and tw[512] == -1j and tw[1024] == -1 and tw[1536] == 1j


def test_config1_n256_batch64():
    x = synth.uniform_complex(synth.SEED_PLAIN, (64, 256))
    y = run(api.Plan(256, 64, -1), x)
    assert per_transform_relerr(y, oracle_ref(x, -1)) <= TOL


def test_paper_ramp_closed_form():
    """The paper's f(x) = x workload against its closed-form spectrum."""
    for n in NS:
        x = synth.ramp(n, 3)
        y = run(api.Plan(n, 3, -1), x)
        k = np.arange(1, n)
        want = np.empty(n, np.complex128)
        want[0] = n * (n - 1) / 2
        want[1:] = -n / 2 + 1j * (n / 2) / np.tan(np.pi * k / n)
        assert per_transform_relerr(y, np.tile(want, (3, 1))) <= TOL, n


@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("n", NS)
def test_default_variant_parity(n, sign):
    p = api.Plan(n, 1, sign)
    tpw = p.describe()["transforms_per_wg"]
    batch = 3 * tpw + 1  # several workgroups and a partly filled last one
    x = synth.uniform_complex(synth.SEED_PLAIN, (batch, n), key=(n, sign + 1))
    y = run(api.Plan(n, batch, sign), x)
    assert per_transform_relerr(y, oracle_ref(x, sign)) <= TOL


def variants():
    """Every (n, ept, wg, variant) compiled into the library (host-only query)."""
    return [(n, *v) for n in NS for v in api.c32_variants(n)]


@pytest.mark.parametrize("n,ept,wg,var", variants())
def test_every_compiled_variant(n, ept, wg, var):
    """Every compiled kernel variant, both signs, several workgroups and a
    partly filled last group; persistent variants (3, 4, 7, 8) additionally with
    more groups than workgroups, so each workgroup loops and prefetches."""
    d = api.Plan(n, 1 << 24, -1, ept=ept, wg=wg, variant=var).describe()
    tpw = d["transforms_per_wg"]
    batches = [2 * tpw + 3 if tpw > 3 else 2 * tpw + 1]
    if var in (3, 4, 7, 8):
        batches.append(int(2.5 * d["grid"] * tpw) + (tpw // 2 if tpw > 1 else 0) + 1)
    for batch in batches:
        for sign in (-1, 1):
            x = synth.uniform_complex(synth.SEED_PLAIN, (batch, n), key=(n, ept, wg, var, sign + 1))
            y = run(api.Plan(n, batch, sign, ept=ept, wg=wg, variant=var), x)
            assert per_transform_relerr(y, oracle_ref(x, sign)) <= TOL, (n, ept, wg, var, sign, batch)


@pytest.mark.parametrize("n", NS)
def test_inverse_equals_scaled_adjoint_bitwise(n):
    """Inverse (sign +1, scale 1/n) and the forward plan's adjoint (sign +1,
    scale 1) run the same kernel; 1/n is a power of two, so the two results
    differ by exactly that factor."""
    batch = 37
    x = to_gpu(synth.uniform_complex(synth.SEED_PLAIN, (batch, n), key=(n, 99)))
    inv = api.Plan(n, batch, +1).execute(x)
    adj = api.Plan(n, batch, -1).adjoint(x)
    assert torch.equal(inv, adj * (1.0 / n))


@pytest.mark.parametrize("n", [2, 64, 2048])
def test_run_to_run_bitwise(n):
    batch = 1000
    x = to_gpu(synth.uniform_complex(synth.SEED_PLAIN, (batch, n), key=(n, 7)))
    p = api.Plan(n, batch, -1)
    a = p.execute(x)
    b = p.execute(x)
    assert torch.equal(a, b)


@pytest.mark.parametrize("n", NS)
def test_roundtrip(n):
    batch = 129
    x = to_gpu(synth.uniform_complex(synth.SEED_PLAIN, (batch, n), key=(n, 5)))
    y = api.Plan(n, batch, +1).execute(api.Plan(n, batch, -1).execute(x))
    assert per_transform_relerr(to_cpu(y), to_cpu(x)) <= 2 * TOL


@pytest.mark.parametrize("n", NS)
def test_full_size_sampled(n):
    """Full sweep size (2^26 complex elements, 512 MiB) in the benchmark's
    launch configuration: sampled transforms against the oracle, and
    Parseval on every transform."""
    batch = (1 << 26) // n
    x_np = synth.uniform_complex(synth.SEED_PLAIN, (batch, n), key=(n,))
    x = to_gpu(x_np)
    for sign in (-1, 1):
        plan = api.Plan(n, batch, sign)
        print(f"[case] full n={n} batch={batch} sign={sign} {plan.describe()}", flush=True)
        y = plan.execute(x)
        torch.cuda.synchronize()
        rng = np.random.default_rng(n)
        idx = np.unique(np.concatenate([[0, batch - 1], rng.integers(0, batch, 62)]))
        ys = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        assert per_transform_relerr(ys, oracle_ref(x_np[idx], sign)) <= TOL
        # Parseval per transform: sum |X|^2 = N^(1 if fwd else -1) sum |x|^2
        ex = (x.abs().double() ** 2).sum(-1)
        ey = (y.abs().double() ** 2).sum(-1)
        f = float(n) if sign < 0 else 1.0 / n
        assert float(((ey - f * ex).abs() / (f * ex)).max()) < 1e-5
        del y


def test_rejects_overlap_misalignment_null():
    n, batch = 256, 4
    p = api.Plan(n, batch, -1)
    buf = torch.zeros(2 * n * batch, dtype=torch.complex64, device="cuda")
    L = api.lib()
    import ctypes
    base = buf.data_ptr()
    s = ctypes.c_void_p(0)
    assert L.fft_execute(p._h, ctypes.c_void_p(base), ctypes.c_void_p(base + 8 * 16), s) == 6  # overlap
    # complex64 buffers need 8-byte (element) alignment; both calls are refused
    # before any launch
    assert L.fft_execute(p._h, ctypes.c_void_p(base + 4), ctypes.c_void_p(base + 8 * n * batch), s) == 11
    assert L.fft_execute(p._h, ctypes.c_void_p(base), ctypes.c_void_p(base + 8 * n * batch + 4), s) == 11
    assert L.fft_execute(p._h, None, ctypes.c_void_p(base), s) == 5
    assert L.fft_execute(None, ctypes.c_void_p(base), ctypes.c_void_p(base + 8 * n * batch), s) == 5
    # exactly adjacent buffers do not overlap
    assert L.fft_execute(p._h, ctypes.c_void_p(base), ctypes.c_void_p(base + 8 * n * batch), s) == 0
    torch.cuda.synchronize()
