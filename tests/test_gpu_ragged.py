"""Ragged batches (mixed lengths, one launch) against the FP64 oracle.

Workload of record: 4096 transforms, lengths 2^L with L uniform on 3..11,
packed back to back; bar: every transform within relative L2 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, synth
from paper_2203_09384_amd.native import MifftError
from gpu_util import need_gpu, to_cpu, to_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def max_seg_err(y, ref, off):
    worst = 0.0
    for b in range(len(off) - 1):
        s = slice(off[b], off[b + 1])
        den = np.linalg.norm(ref[s])
        worst = max(worst, float(np.linalg.norm(y[s] - ref[s]) / (den if den else 1.0)))
    return worst


def workload(count=4096, lo=3, hi=11, seed=synth.SEED_RAGGED):
    lengths = synth.ragged_lengths(seed, count, lo, hi)
    off = synth.offsets_from_lengths(lengths)
    x = synth.uniform_complex(seed, (int(off[-1]),), key=(1,))
    return off, x


@pytest.mark.parametrize("sign", [-1, 1])
def test_config4_workload(sign):
    off, x = workload()
    p = api.RaggedPlan(off, sign)
    print(f"[case] ragged config4 sign={sign} {p.describe()}", flush=True)
    y = to_cpu(p.execute(to_gpu(x)))
    ref = oracle.fft_ragged(x.astype(np.complex128), off, sign, inverse_scale=sign > 0)
    assert max_seg_err(y, ref, off) <= TOL


def test_every_length_including_2_and_4():
    off, x = workload(600, 1, 11, seed=7)
    p = api.RaggedPlan(off, -1)
    y = to_cpu(p.execute(to_gpu(x)))
    ref = oracle.fft_ragged(x.astype(np.complex128), off, -1)
    assert max_seg_err(y, ref, off) <= TOL


def test_repeated_launches_agree():
    off, x = workload(1000, 3, 11, seed=11)
    p = api.RaggedPlan(off, -1)
    xg = to_gpu(x)
    a = p.execute(xg)
    b = p.execute(xg)
    c = p.execute(xg)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(b, c)


def test_adjoint():
    off, x = workload(500, 3, 11, seed=13)
    for sign in (-1, 1):
        p = api.RaggedPlan(off, sign)
        y = to_cpu(p.adjoint(to_gpu(x)))
        # adjoint of (sign, scale): opposite sign, same per-transform scale
        ref = oracle.fft_ragged(x.astype(np.complex128), off, -sign, inverse_scale=sign > 0)
        assert max_seg_err(y, ref, off) <= TOL


def test_graph_replay_matches_eager():
    """One launch captured in a graph; replays interleaved with
    other eager work all equal the eager result bit for bit."""
    off, x = workload(4096, 3, 11, seed=17)
    p = api.RaggedPlan(off, -1)
    xg = to_gpu(x)
    eager = p.execute(xg).clone()
    out = torch.empty_like(xg)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.execute(xg, out)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.execute(xg, out)
    for i in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), i
        _ = (xg * 2).sum().item()  # unrelated eager work between replays
        p.execute(xg)              # and an eager launch of the same plan


DEFAULT_EPT = [0, 2, 4, 8, 4, 4, 4, 8, 8, 8, 8, 8]  # the built-in per-length choice


@pytest.mark.parametrize("wg", [64, 128, 256])
@pytest.mark.parametrize("table", ["small", "default", "large"])
def test_forced_configs(wg, table):
    """Every compiled workgroup size with small, default and large elements
    per thread.  A length's threads (2^L / ept) must fit one workgroup, so
    the workload's longest length is the largest that the (wg, table) pair
    holds: 64-thread kernels run lengths up to 256..1024, the others to
    512..2048.  No case is skipped."""
    eps = {"small": [0, 2, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4],
           "default": None,
           "large": [0, 2, 4, 8, 16, 16, 16, 16, 16, 16, 16, 16]}[table]
    table_e = eps or DEFAULT_EPT
    hi = max(L for L in range(1, 12) if (1 << L) // table_e[L] <= wg)
    off, x = workload(800, 1, hi, seed=19)
    p = api.RaggedPlan(off, -1, ept_by_log2n=eps, wg=wg)
    d = p.describe()
    print(f"[case] ragged wg={wg} table={table} lengths 2..{1 << hi} {d}", flush=True)
    assert d["wg"] == wg
    y = to_cpu(p.execute(to_gpu(x)))
    ref = oracle.fft_ragged(x.astype(np.complex128), off, -1)
    assert max_seg_err(y, ref, off) <= TOL


def test_too_long_for_the_workgroup_is_refused():
    """A 2048-point length needs at least 128 threads (16 per thread at
    most): a 64-thread launch is refused at planning."""
    off, _ = workload(50, 11, 11, seed=21)
    with pytest.raises(MifftError) as ei:
        api.RaggedPlan(off, -1, wg=64)
    assert ei.value.status == "FFT_EINVAL_CONFIG"


def test_single_transform_and_ctas_limit():
    off = np.array([0, 2048], np.int64)
    x = synth.uniform_complex(23, (2048,))
    p = api.RaggedPlan(off, -1, ctas_per_cu=1)
    y = to_cpu(p.execute(to_gpu(x)))
    assert max_seg_err(y, oracle.forward(x.astype(np.complex128)), off) <= TOL


@pytest.mark.parametrize("ctas", [1, 2, 3])
def test_several_rounds_per_workgroup(ctas):
    """A grid smaller than the tile list: each workgroup takes tiles in
    rounds, every other round reversed.  The result is bitwise that of the
    one-round launch (same per-tile kernels) and within tolerance of the
    oracle."""
    off, x = workload(4096, 3, 11, seed=29)
    xg = to_gpu(x)
    full = api.RaggedPlan(off, -1, wg=128)
    p = api.RaggedPlan(off, -1, wg=128, ctas_per_cu=ctas)
    d, dfull = p.describe(), full.describe()
    print(f"[case] ragged rounds ctas={ctas} grid={d['grid']} tiles={d['tiles']}", flush=True)
    assert d["grid"] < d["tiles"] and d["tiles"] == dfull["tiles"]
    y = p.execute(xg)
    assert torch.equal(y, full.execute(xg))
    ref = oracle.fft_ragged(x.astype(np.complex128), off, -1)
    assert max_seg_err(to_cpu(y), ref, off) <= TOL


def test_one_plan_on_two_streams():
    """A ragged launch keeps no device state, so executes of one plan may
    overlap on two streams."""
    off, _ = workload(2000, 3, 11, seed=31)
    p = api.RaggedPlan(off, -1)
    xs = [to_gpu(synth.uniform_complex(31, (int(off[-1]),), key=(i,))) for i in range(2)]
    refs = [p.execute(x).clone() for x in xs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty_like(x) for x in xs]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    for _ in range(20):
        for s, x, o in zip(streams, xs, outs):
            with torch.cuda.stream(s):
                p.execute(x, o, stream=s)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
