"""Multidimensional FP32 transforms (2D / 3D) on the GPU against the FP64
oracle's fftn (pinned in the oracle's own tests).  Bar: max over arrays of
the relative L2 error <= 1e-5."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from gpu_util import need_gpu, to_cpu, to_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5
SEED_ND = 20220322

SHAPES = [(2, 2), (4, 8), (8, 2), (16, 2048), (2048, 16), (64, 64), (2, 4096), (4, 65536), (8, 4, 2), (2, 2, 2),
          (32, 64, 8), (16, 16, 16), (4, 2048, 4), (2048, 2, 2),
          # single-pass 2D (the array fits one workgroup's LDS)
          (128, 128), (64, 256), (256, 64), (16, 1024), (1024, 16), (2, 1024), (32, 32), (8, 512), (4, 4),
          # 3D: last two axes in one pass, or not
          (2, 128, 128), (4, 64, 64), (2, 256, 256), (8, 2, 1024),
          # 3D single pass (every axis >= 4, at most 16384 points)
          (4, 4, 4), (16, 32, 32), (32, 16, 8), (4, 256, 16), (64, 4, 4), (8, 8, 128)]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def per_array_relerr(y, ref, ndim):
    y = np.asarray(y, np.complex128)
    ref = np.asarray(ref, np.complex128)
    axes = tuple(range(y.ndim - ndim, y.ndim))
    num = np.sqrt(np.sum(np.abs(y - ref) ** 2, axis=axes))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=axes))
    return float(np.max(num / np.where(den == 0, 1, den)))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("sign", [-1, 1])
def test_nd_parity(shape, sign):
    n = int(np.prod(shape))
    batch = 3 if n <= 65536 else 1
    x = synth.uniform_complex(SEED_ND, (batch,) + shape, key=shape + (sign + 1,))
    p = api.PlanND(shape, batch, sign)
    print(f"[case] nd shape={shape} batch={batch} sign={sign} {p.describe()}", flush=True)
    y = to_cpu(p.execute(to_gpu(x)))
    ref = oracle.fftn(x.astype(np.complex128), len(shape), sign, 1.0 if sign < 0 else 1.0 / n)
    assert per_array_relerr(y, ref, len(shape)) <= TOL
    # adjoint: opposite sign, same scale
    g = synth.uniform_complex(SEED_ND, (batch,) + shape, key=shape + (sign + 5,))
    a = to_cpu(p.adjoint(to_gpu(g)))
    ref = oracle.fftn(g.astype(np.complex128), len(shape), -sign, 1.0 if sign < 0 else 1.0 / n)
    assert per_array_relerr(a, ref, len(shape)) <= TOL


def test_nd_full_size_sampled():
    """2048 x 2048, batch 16 (2^26 elements, 512 MiB each way): two arrays
    against the oracle, Parseval on every array, and the round trip."""
    shape, batch = (2048, 2048), 16
    x = synth.uniform_complex(SEED_ND, (batch,) + shape, key=(99,))
    xg = to_gpu(x)
    print(f"[case] nd full size {shape} batch={batch}", flush=True)
    y = api.PlanND(shape, batch, -1).execute(xg)
    for b in (0, batch - 1):
        ys = to_cpu(y[b])
        assert per_array_relerr(ys[None], oracle.fftn(x[b:b + 1].astype(np.complex128), 2), 2) <= TOL
    e_in = torch.sum(torch.abs(xg.to(torch.complex128)) ** 2, dim=(1, 2))
    e_out = torch.sum(torch.abs(y.to(torch.complex128)) ** 2, dim=(1, 2))
    assert torch.max(torch.abs(e_out / (e_in * (2048 * 2048)) - 1)).item() < 1e-5
    back = api.PlanND(shape, batch, +1).execute(y)
    assert per_array_relerr(to_cpu(back), x, 2) <= 2 * TOL


def test_functional_and_autograd():
    x = synth.uniform_complex(SEED_ND, (3, 8, 32), key=(7,))
    X = to_cpu(api.fft2(to_gpu(x)))
    assert per_array_relerr(X, oracle.fftn(x.astype(np.complex128), 2), 2) <= TOL
    back = to_cpu(api.ifft2(to_gpu(X.astype(np.complex64))))
    assert per_array_relerr(back, x, 2) <= 2 * TOL
    # gradient of sum w |fftn(x)|^2 = F^H (2 w F x)
    w = synth.uniform_weights(SEED_ND, (3, 8, 32), key=(8,))
    xg = to_gpu(x).requires_grad_(True)
    y = api.fftn_differentiable(xg, 2)
    (to_gpu(w) * (y.real ** 2 + y.imag ** 2)).sum().backward()
    x64 = x.astype(np.complex128)
    ref = oracle.fftn(2.0 * w * oracle.fftn(x64, 2), 2, +1, 1.0)
    assert per_array_relerr(xg.grad.cpu().numpy(), ref, 2) <= TOL


@pytest.mark.parametrize("shape,single", [((128, 128), True), ((64, 64), True), ((2, 2), True), ((16, 2048), False),
                                          ((2, 4096), False), ((256, 128), False), ((4, 128, 128), True),
                                          ((2, 256, 256), False)])
def test_single_pass_choice(shape, single):
    """Arrays that fit one workgroup's LDS run the single-pass 2D kernel (for
    3D: over the last two axes)."""
    d = api.PlanND(shape, 2, -1).describe()
    assert (d["variant"] == 10) == single, d
    assert d["dims"] == list(shape)


@pytest.mark.parametrize("shape,single", [((16, 16, 16), True), ((4, 64, 64), False), ((16, 16, 32), True),
                                          ((4, 4, 4), True), ((2, 64, 64), False), ((8, 4, 2), False),
                                          ((4, 128, 128), False), ((4, 1024, 4), False), ((16, 32, 32), False)])
def test_single_pass_3d_choice(shape, single):
    """3D arrays of at most 16384 points with every axis at least 4 run the
    single-pass 3D kernel (variant 13) when an array fits one workgroup
    (N / EPT <= 1024 threads, EPT the smallest axis up to 16 points): every
    axis's passes in one kernel.  4 x 64 x 64 (4 points per thread, 4096
    threads) does not, nor does 16 x 32 x 32 (200 KiB of exchange regions)."""
    d = api.PlanND(shape, 2, -1).describe()
    assert (d["variant"] == 13) == single, d
    assert d["dims"] == list(shape) and d["rank"] == 3
    if single:
        assert int(np.prod(d["radices"][:d["npasses"]])) == int(np.prod(shape))


def test_single_pass_3d_full_size():
    """16 x 16 x 32, batch 8192 (2^26 elements): sampled arrays against the
    oracle, and the round trip over the whole batch."""
    shape, batch = (16, 16, 32), 8192
    x = synth.uniform_complex(SEED_ND, (batch,) + shape, key=(97,))
    xg = to_gpu(x)
    print(f"[case] nd3 full size {shape} batch={batch}", flush=True)
    p = api.PlanND(shape, batch, -1)
    assert p.describe()["variant"] == 13
    y = p.execute(xg)
    idx = [0, 1, batch // 2, batch - 1]
    ys = to_cpu(y[idx])
    assert per_array_relerr(ys, oracle.fftn(x[idx].astype(np.complex128), 3), 3) <= TOL
    back = api.PlanND(shape, batch, +1).execute(y)
    assert per_array_relerr(to_cpu(back), x, 3) <= 2 * TOL


def test_single_pass_full_size():
    """128 x 128, batch 4096 (2^26 elements): sampled arrays against the
    oracle and the round trip over the whole batch."""
    shape, batch = (128, 128), 4096
    x = synth.uniform_complex(SEED_ND, (batch,) + shape, key=(98,))
    xg = to_gpu(x)
    print(f"[case] nd2 full size {shape} batch={batch}", flush=True)
    y = api.PlanND(shape, batch, -1).execute(xg)
    idx = [0, 1, batch // 2, batch - 1]
    ys = to_cpu(y[idx])
    assert per_array_relerr(ys, oracle.fftn(x[idx].astype(np.complex128), 2), 2) <= TOL
    back = api.PlanND(shape, batch, +1).execute(y)
    assert per_array_relerr(to_cpu(back), x, 2) <= 2 * TOL


@pytest.mark.parametrize("shape", [(128, 128), (64, 128), (256, 32), (32, 256), (256, 16)],
                         ids=lambda s: "x".join(map(str, s)))
def test_single_pass_persistent_every_array(shape):
    """Arrays that fill more than half of a CU's LDS, or of one-thread rows
    whose LDS leaves the one-shot grid at most 16 wavefronts per CU, run
    persistent, as many workgroups as are resident at once walking the
    batch (describe()'s grid is then below the batch): a batch of
    2.5x that grid plus 3, so workgroups take two or three arrays through
    the prefetching loop body and the last one after it.  Every array
    against the oracle, both signs."""
    big = 1 << 14
    grid = api.PlanND(shape, big, -1).describe()["grid"]
    assert grid < big
    batch = grid * 5 // 2 + 3
    n = int(np.prod(shape))
    x = synth.uniform_complex(SEED_ND, (batch,) + shape, key=shape + (40,))
    xg = to_gpu(x)
    x64 = x.astype(np.complex128)
    for sign in (-1, 1):
        p = api.PlanND(shape, batch, sign)
        print(f"[case] nd2 persistent {shape} batch={batch} sign={sign} {p.describe()}", flush=True)
        assert p.describe()["grid"] == grid
        y = to_cpu(p.execute(xg))
        ref = oracle.fftn(x64, 2, sign, 1.0 if sign < 0 else 1.0 / n)
        assert per_array_relerr(y, ref, 2) <= TOL


@pytest.mark.parametrize("shape", [(16, 16, 16), (16, 16, 32), (8, 8, 128)],
                         ids=lambda s: "x".join(map(str, s)))
def test_single_pass_3d_persistent_every_array(shape):
    """3D arrays of one workgroup each whose first two axes are one thread
    per line (N0 = N1 = points per thread) and whose LDS leaves a CU at most
    16 wavefronts of the one-shot grid run persistent: as many
    workgroups as fit the device at once walk the batch (describe()'s grid
    is then below the batch), prefetching the next array during axes 1 and
    0.  A batch of 2.5x that grid plus 3, so workgroups take two or three
    arrays through the loop body and the last one after it.  Every array
    against the oracle, both signs."""
    big = 1 << 16
    grid = api.PlanND(shape, big, -1).describe()["grid"]
    assert grid < big
    batch = grid * 5 // 2 + 3
    n = int(np.prod(shape))
    x = synth.uniform_complex(SEED_ND, (batch,) + shape, key=shape + (41,))
    xg = to_gpu(x)
    x64 = x.astype(np.complex128)
    for sign in (-1, 1):
        p = api.PlanND(shape, batch, sign)
        print(f"[case] nd3 persistent {shape} batch={batch} sign={sign} {p.describe()}", flush=True)
        assert p.describe()["variant"] == 13 and p.describe()["grid"] == grid
        y = to_cpu(p.execute(xg))
        ref = oracle.fftn(x64, 3, sign, 1.0 if sign < 0 else 1.0 / n)
        assert per_array_relerr(y, ref, 3) <= TOL


@pytest.mark.parametrize("shape", [(8, 8, 32), (4, 4, 64), (4, 4, 4)], ids=lambda s: "x".join(map(str, s)))
def test_single_pass_3d_one_shot_grid(shape):
    """Shapes whose one-shot grid already fills a CU with wavefronts keep a
    workgroup per group of arrays."""
    d = api.PlanND(shape, 1 << 16, -1).describe()
    assert d["variant"] == 13 and d["grid"] == (1 << 16) // d["transforms_per_wg"]


@pytest.mark.parametrize("shape,batch", [((1024, 1024), 10), ((2048, 1024), 5)], ids=["1024x1024", "2048x1024"])
@pytest.mark.parametrize("sign", [-1, 1])
def test_axis_pass_persistent_every_array(shape, batch, sign):
    """1024-point axis passes whose tiles are all whole run one persistent
    workgroup per CU: 1024 x 1024, batch 10, is 640 tiles of 16 columns, so
    every workgroup takes two or three tiles (the prefetching body, then the
    last tile).  2048 x 1024, batch 5 (640 tiles of 8 columns) runs the
    one-shot 2048-point pass next to it.  Every array against the oracle."""
    n = int(np.prod(shape))
    x = synth.uniform_complex(SEED_ND, (batch,) + shape, key=(41, shape[0], sign + 1))
    p = api.PlanND(shape, batch, sign)
    print(f"[case] axis persistent {shape} batch={batch} sign={sign}", flush=True)
    y = to_cpu(p.execute(to_gpu(x)))
    ref = oracle.fftn(x.astype(np.complex128), 2, sign, 1.0 if sign < 0 else 1.0 / n)
    assert per_array_relerr(y, ref, 2) <= TOL


@pytest.mark.parametrize("shape", [(128, 128), (2048, 64), (4, 64, 64)], ids=lambda s: "x".join(map(str, s)))
def test_nd_run_to_run_bitwise_and_scaled_adjoint(shape):
    """Repeated executes give identical bits, and the inverse equals the
    forward plan's adjoint times 1/prod(dims) bit for bit (the same kernels,
    a power-of-two scale)."""
    n = int(np.prod(shape))
    batch = 3
    x = to_gpu(synth.uniform_complex(SEED_ND, (batch,) + shape, key=shape + (30,)))
    pf, pi = api.PlanND(shape, batch, -1), api.PlanND(shape, batch, +1)
    y0 = pf.execute(x)
    for _ in range(3):
        assert torch.equal(pf.execute(x), y0)
    inv = to_cpu(pi.execute(x))
    adj = to_cpu(pf.adjoint(x))
    assert np.array_equal(inv, (adj / np.float32(n)).astype(np.complex64))
