"""FP16 / BF16 block-floating-point path (N = 2048, radix-16 passes on MFMA)
against the FP64 oracle.

The oracle transforms the stored half-precision input values (times
2^in_exp) in FP64; the GPU output is de-scaled (stored * 2^out_exp) in FP64.
Bar: per-transform relative L2 <= 3e-3 for each dtype and input class
(uniform[-1,1) re/im; log-uniform magnitude 1e-3..1e3 with uniform phase).
The error against the raw FP64 draw (which adds input quantisation) is
printed as a second figure.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
N = 2048
TOL = 3e-3
TORCH = {"c16": torch.float16, "cbf16": torch.bfloat16}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def draw(cls, batch, key=0):
    if cls == "uniform":
        return synth.uniform_complex(synth.SEED_HALF, (batch, N), key=(key, 0), dtype=np.complex128)
    return synth.log_uniform_polar(synth.SEED_HALF, (batch, N), key=(key, 1))


def to_half(x, dtype):
    t = torch.from_numpy(np.stack([x.real, x.imag], -1).astype(np.float32)).to(TORCH[dtype])
    return t.cuda().contiguous()


def from_half(t, exps=None):
    a = t.float().cpu().numpy().astype(np.float64)
    z = a[..., 0] + 1j * a[..., 1]
    if exps is not None:
        z = z * np.exp2(exps.cpu().numpy().astype(np.float64))[:, None]
    return z


def rel(y, ref):
    return float(np.max(np.linalg.norm(y - ref, axis=-1) / np.linalg.norm(ref, axis=-1)))


@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
@pytest.mark.parametrize("cls", ["uniform", "loguniform"])
@pytest.mark.parametrize("sign", [-1, 1])
def test_parity_small_batch(dtype, cls, sign):
    batch = 257
    x = draw(cls, batch)
    xh = to_half(x, dtype)
    p = api.Plan(N, batch, sign, dtype=dtype)
    print(f"[case] half {dtype} {cls} sign={sign} {p.describe()}", flush=True)
    yh, ex = p.execute_scaled(xh)
    torch.cuda.synchronize()
    y = from_half(yh, ex)
    xs = from_half(xh)
    ref = oracle.forward(xs) if sign < 0 else oracle.inverse(xs)
    ref_raw = oracle.forward(x) if sign < 0 else oracle.inverse(x)
    e, e_raw = rel(y, ref), rel(y, ref_raw)
    print(f"{dtype} {cls} sign={sign}: vs stored input {e:.3e}, vs raw draw {e_raw:.3e}")
    assert np.all(np.isfinite(y))
    assert e <= TOL


@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
@pytest.mark.parametrize("cls", ["uniform", "loguniform"])
def test_full_size_sampled(dtype, cls):
    """The reduced-precision workload of record: N=2048, batch 32768."""
    batch = 32768
    x = draw(cls, batch, key=1)
    xh = to_half(x, dtype)
    del x
    p = api.Plan(N, batch, -1, dtype=dtype)
    print(f"[case] half full {dtype} {cls}", flush=True)
    yh, ex = p.execute_scaled(xh)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(yh.float()).all())
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, batch - 1], rng.integers(0, batch, 62)]))
    it = torch.from_numpy(idx).cuda()
    y = from_half(yh[it], ex[it])
    xs = from_half(xh[it])
    e = rel(y, oracle.forward(xs))
    print(f"full {dtype} {cls}: sampled max rel L2 {e:.3e}")
    assert e <= TOL
    # exponents: the stored output's largest component lies in [2^-1, 2^15)
    mx = yh.float().abs().amax(dim=(1, 2))
    assert float(mx.max()) < 2.0 ** 15 and float(mx.min()) >= 0.5


def grid_limit(n, sign, dtype):
    """Workgroups a plan of length n < 2048 launches at most (the looping
    cap), and transforms per workgroup, from describe()."""
    assert n < N
    p = api.Plan(n, 1 << 22, sign, dtype=dtype)
    d = p.describe()
    p.close()
    return d["grid"], d["transforms_per_wg"]


def check_every_transform(yh, ex, xh, sign, n, tol, chunk_elems=1 << 22):
    """Every transform of a stored result against the oracle on the stored
    input, in chunks (FP64 on the host)."""
    batch = yh.shape[0]
    step = max(1, chunk_elems // n)
    worst = 0.0
    for a in range(0, batch, step):
        b = min(batch, a + step)
        y = from_half(yh[a:b], ex[a:b])
        xs = from_half(xh[a:b])
        ref = oracle.forward(xs) if sign < 0 else oracle.inverse(xs)
        worst = max(worst, rel(y, ref))
    assert worst <= tol, worst
    return worst


def run_length(sign, dtype, batch=1 << 16):
    """Consecutive transforms per workgroup at N = 2048 (describe())."""
    p = api.Plan(N, batch, sign, dtype=dtype)
    d = p.describe()
    p.close()
    return d["transforms_per_wg"]


@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
@pytest.mark.parametrize("cls", ["uniform", "loguniform"])
@pytest.mark.parametrize("sign", [-1, 1])
def test_runs_every_transform(dtype, cls, sign):
    """Workgroups take runs of consecutive transforms with the next two
    prefetched, alternating two buffers: a batch of many runs and a partial
    last run, so every workgroup runs both bodies of the loop and the last
    one ends early.  Every transform, forward and inverse, against the oracle."""
    t = run_length(sign, dtype)
    batch = 1025 * t + t - 1
    x = draw(cls, batch, key=7)
    xh = to_half(x, dtype)
    del x
    p = api.Plan(N, batch, sign, dtype=dtype)
    d = p.describe()
    print(f"[case] half runs {dtype} {cls} sign={sign} batch={batch} {d}", flush=True)
    assert t >= 2 and d["transforms_per_wg"] == t and d["grid"] == -(-batch // t)
    yh, ex = p.execute_scaled(xh)
    torch.cuda.synchronize()
    e = check_every_transform(yh, ex, xh, sign, N, TOL)
    print(f"runs {dtype} {cls} sign={sign}: max rel L2 over {batch} transforms {e:.3e}")


def edge_batch(dtype, batch, t):
    """Uniform transforms with special ones planted at both ends of the batch
    and around the first run boundaries (t transforms per workgroup).
    Returns the stored input and the kinds."""
    rng = np.random.default_rng(11)
    x = draw("uniform", batch, key=8)
    kinds = {}
    pos = [0, 1, t - 1, t, t + 1, 2 * t + 2, batch - 2, batch - 1]
    specials = ["zero", "big", "tiny", "bottom", "inf", "bottom", "zero", "big"]
    for b, kind in zip(pos, specials):
        kinds[b] = kind
        if kind == "zero":
            x[b] = 0
        elif kind == "big":  # near the top of FP16's range, the rest small
            x[b] = 1e-3 * (rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N))
            x[b, rng.integers(N)] = 6.0e4
        elif kind == "tiny":  # FP16 subnormal range
            x[b] = 2.0 ** -20 * (rng.uniform(1, 2, N) * rng.choice([-1, 1], N)
                                 + 1j * rng.uniform(1, 2, N) * rng.choice([-1, 1], N))
        elif kind == "bottom":  # the bottom of the storage format's range
            lo = -130 if dtype == "cbf16" else -24  # BF16 subnormals / the FP16 subnormal unit
            x[b] = 2.0 ** lo * (rng.integers(1, 8, N) + 1j * rng.integers(-7, 8, N))
        elif kind == "inf":
            x[b, rng.integers(N)] = np.inf
    return x, kinds


@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
@pytest.mark.parametrize("sign", [-1, 1])
def test_block_fp_edge_cases(dtype, sign):
    """Block-floating-point edge cases inside a batch of many workgroups'
    runs of transforms.  Documented results: an all-zero transform gives stored
    zeros (logical value 0); one with a component near FP16's maximum, one in
    FP16's subnormal range and one at the bottom of the storage format's
    range (BF16 subnormals) are each scaled into range and meet the 3e-3
    bar; a transform holding an inf gives non-finite values in that
    transform only.  Every other transform still meets the bar."""
    t = run_length(sign, dtype)
    batch = 64 * t + 5
    x, kinds = edge_batch(dtype, batch, t)
    xh = to_half(x, dtype)
    p = api.Plan(N, batch, sign, dtype=dtype)
    print(f"[case] half edge {dtype} sign={sign} batch={batch} kinds={kinds}", flush=True)
    yh, ex = p.execute_scaled(xh)
    torch.cuda.synchronize()
    y = from_half(yh, ex)
    xs = from_half(xh)
    with np.errstate(invalid="ignore", over="ignore"):
        ref = oracle.forward(xs) if sign < 0 else oracle.inverse(xs)
    for b in range(batch):
        kind = kinds.get(b, "uniform")
        if kind == "zero":
            assert not np.any(yh[b].float().cpu().numpy()), b
        elif kind == "inf":
            assert not np.all(np.isfinite(y[b])), b
        else:
            e = float(np.linalg.norm(y[b] - ref[b]) / np.linalg.norm(ref[b]))
            assert np.all(np.isfinite(y[b])) and e <= TOL, (b, kind, e)


@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
def test_input_exponent_is_exact(dtype):
    """Scaling the input by 2^k per transform changes only the exponent."""
    batch = 64
    xh = to_half(draw("uniform", batch, key=2), dtype)
    p = api.Plan(N, batch, -1, dtype=dtype)
    y0, e0 = p.execute_scaled(xh)
    k = torch.from_numpy(np.random.default_rng(0).integers(-20, 20, batch).astype(np.int32)).cuda()
    y1, e1 = p.execute_scaled(xh, in_exp=k)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    assert torch.equal(e1, e0 + k)


@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
def test_unit_scale_execute_and_determinism(dtype):
    batch = 32
    x = 1e-2 * draw("uniform", batch, key=3)
    xh = to_half(x, dtype)
    p = api.Plan(N, batch, -1, dtype=dtype)
    out = p.execute(xh)  # unit-scale output, no exponent array
    y, ex = p.execute_scaled(xh)
    y2, _ = p.execute_scaled(xh)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    ref = oracle.forward(from_half(xh))
    assert rel(from_half(out), ref) <= TOL


# ---------------------------------------------------------------- n = 2 .. 1024
# FP32 Stockham passes with 16-bit storage and block exponents.
SMALL = [1 << L for L in range(1, 11)]


def draw_n(cls, batch, n, key):
    if cls == "uniform":
        return synth.uniform_complex(synth.SEED_HALF, (batch, n), key=(n, key, 0), dtype=np.complex128)
    return synth.log_uniform_polar(synth.SEED_HALF, (batch, n), key=(n, key, 1))


# The error of these lengths is the rounding of the stored output: one
# value rounds with relative error at most 2^-11 (FP16) or 2^-8 (BF16, 8
# significant bits), and with few outputs per transform the per-transform
# L2 error need not average below that.  Bars: those bounds plus the FP32
# passes' ~1e-6.  (At N = 2048 the BF16 error averages to ~1.7e-3, under
# the 3e-3 bar of that workload.)
SMALL_TOL = {"c16": 2.0 ** -11 + 1e-5, "cbf16": 2.0 ** -8 + 1e-5}


@pytest.mark.parametrize("n", SMALL)
@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
@pytest.mark.parametrize("sign", [-1, 1])
def test_small_lengths_parity(n, dtype, sign):
    """Both input classes against the oracle on the stored input."""
    batch = 3 * max(1, 4096 // n) + 1
    p = api.Plan(n, batch, sign, dtype=dtype)
    print(f"[case] half small n={n} {dtype} sign={sign} {p.describe()}", flush=True)
    for cls in ("uniform", "loguniform"):
        xh = to_half(draw_n(cls, batch, n, 4), dtype)
        yh, ex = p.execute_scaled(xh)
        torch.cuda.synchronize()
        y = from_half(yh, ex)
        xs = from_half(xh)
        ref = oracle.forward(xs) if sign < 0 else oracle.inverse(xs)
        e = rel(y, ref)
        assert np.all(np.isfinite(y))
        assert e <= SMALL_TOL[dtype], (cls, e)
        # stored outputs use the format's range: largest component in
        # [2^14, 2^15] (scaled below 2^15, which rounding may reach)
        mx = yh.float().abs().amax(dim=(1, 2))
        assert float(mx.max()) <= 2.0 ** 15 and float(mx.min()) >= 2.0 ** 14


@pytest.mark.parametrize("n", [2, 64, 1024])
@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
def test_small_lengths_exponents_and_unit_scale(n, dtype):
    """An input exponent shifts only the output exponent; unit-scale output
    (no exponent array) is the logical value."""
    batch = 33
    xh = to_half(1e-2 * draw_n("uniform", batch, n, 5), dtype)
    p = api.Plan(n, batch, -1, dtype=dtype)
    y0, e0 = p.execute_scaled(xh)
    k = torch.from_numpy(np.random.default_rng(1).integers(-20, 20, batch).astype(np.int32)).cuda()
    y1, e1 = p.execute_scaled(xh, in_exp=k)
    out = p.execute(xh)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    assert torch.equal(e1, e0 + k)
    assert rel(from_half(out), oracle.forward(from_half(xh))) <= SMALL_TOL[dtype]


@pytest.mark.parametrize("n", [64, 2048])
@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
@pytest.mark.parametrize("sign", [-1, 1])
def test_half_adjoint(n, dtype, sign):
    """The adjoint of a half-precision plan: opposite sign, the plan's scale,
    unit-scale output."""
    batch = 19
    xh = to_half(1e-2 * draw_n("uniform", batch, n, 6), dtype)
    p = api.Plan(n, batch, sign, dtype=dtype)
    out = p.adjoint(xh)
    torch.cuda.synchronize()
    ref = oracle.adjoint(from_half(xh), sign, 1.0 if sign < 0 else 1.0 / n)
    bar = SMALL_TOL[dtype] if n < 2048 else TOL
    assert rel(from_half(out), ref) <= bar


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
def test_small_lengths_looping_grid(n, dtype):
    """Batches past the launch's grid cap (read from describe()) with a
    ragged last group, so workgroups loop over groups of transforms: every
    transform against the oracle, and the stored range of every transform."""
    cap, tpb = grid_limit(n, -1, dtype)
    batch = cap * tpb * 3 // 2 + 3
    gen = torch.Generator(device="cuda").manual_seed(2203 + n)
    x = (2 * torch.rand(batch, n, 2, device="cuda", generator=gen) - 1).to(TORCH[dtype])
    p = api.Plan(n, batch, -1, dtype=dtype)
    d = p.describe()
    print(f"[case] half looping grid n={n} {dtype} batch={batch} {d}", flush=True)
    assert d["grid"] == cap and cap * tpb < batch
    yh, ex = p.execute_scaled(x)
    torch.cuda.synchronize()
    mx = yh.float().abs().amax(dim=(1, 2))
    assert float(mx.max()) <= 2.0 ** 15 and float(mx.min()) >= 2.0 ** 14
    check_every_transform(yh, ex, x, -1, n, SMALL_TOL[dtype])
