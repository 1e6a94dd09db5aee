"""Every execute entry point only enqueues work, so it can be captured into a
graph.  Each graph is replayed several times with unrelated eager work and
synchronisations in between, and every replay must equal the eager result
bit for bit."""
import numpy as np
import pytest
import torch

from paper_2203_09384_amd import api, synth
from gpu_util import need_gpu, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def replay_and_check(g, outs, refs, scratch):
    for i in range(4):
        for o in outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r), i
        _ = (scratch * 3).sum().item()


@pytest.mark.parametrize("n", [2, 64, 2048])
def test_plain_and_adjoint_in_graph(n):
    batch = (1 << 20) // n
    x = to_gpu(synth.uniform_complex(51, (batch, n), key=(n,)))
    p = api.Plan(n, batch, -1)
    ref_y, ref_a = p.execute(x), p.adjoint(x)
    y, a = torch.empty_like(x), torch.empty_like(x)

    def fn():
        p.execute(x, y)
        p.adjoint(x, a)
    replay_and_check(capture(fn), [y, a], [ref_y, ref_a], x)


def test_fused_loss_in_graph():
    n, batch = 2048, 512
    x = to_gpu(synth.uniform_complex(53, (batch, n)))
    w = to_gpu(synth.uniform_weights(53, (batch, n), key=(1,)))
    p = api.Plan(n, batch, -1)
    ref_l, ref_g = p.loss_grad(x, w)
    ref_l, ref_g = ref_l.clone(), ref_g.clone()
    lv, gr = torch.empty_like(ref_l), torch.empty_like(ref_g)
    replay_and_check(capture(lambda: p.loss_grad(x, w, gr, lv)), [lv, gr], [ref_l, ref_g], x)


@pytest.mark.parametrize("dtype,tdt", [("c16", torch.float16), ("cbf16", torch.bfloat16)])
def test_half_in_graph(dtype, tdt):
    n, batch = 2048, 1000
    x = synth.uniform_complex(55, (batch, n), dtype=np.complex128)
    xh = torch.from_numpy(np.stack([x.real, x.imag], -1).astype(np.float32)).to(tdt).cuda().contiguous()
    p = api.Plan(n, batch, -1, dtype=dtype)
    ry, re = p.execute_scaled(xh)
    ry, re = ry.clone(), re.clone()
    y, e = torch.empty_like(ry), torch.empty_like(re)
    replay_and_check(capture(lambda: p.execute_scaled(xh, out=y, out_exp=e)), [y, e], [ry, re], xh.float())


@pytest.mark.parametrize("n", [2, 64, 2048, 1 << 15])
def test_real_input_in_graph(n):
    batch = max(1, (1 << 19) // n) + 1
    x = to_gpu(synth.uniform_real(57, (batch, n), key=(n,)))
    pf, pi = api.Plan(n, batch, -1, "r32"), api.Plan(n, batch, +1, "r32")
    ref_X, ref_a = pf.execute(x), pf.adjoint(pf.execute(x))
    ref_x = pi.execute(ref_X)
    X, a, xb = torch.empty_like(ref_X), torch.empty_like(ref_a), torch.empty_like(ref_x)

    def fn():
        pf.execute(x, X)
        pf.adjoint(X, a)
        pi.execute(X, xb)
    replay_and_check(capture(fn), [X, a, xb], [ref_X, ref_a, ref_x], x)


@pytest.mark.parametrize("shape", [(128, 128), (2048, 64), (4, 64, 64), (8, 16, 512)],
                         ids=lambda s: "x".join(map(str, s)))
def test_nd_in_graph(shape):
    """Single-pass and multi-kernel multidimensional plans."""
    n = int(np.prod(shape))
    batch = max(1, (1 << 20) // n)
    x = to_gpu(synth.uniform_complex(59, (batch,) + shape, key=shape))
    p = api.PlanND(shape, batch, -1)
    ref_y, ref_a = p.execute(x), p.adjoint(x)
    y, a = torch.empty_like(x), torch.empty_like(x)

    def fn():
        p.execute(x, y)
        p.adjoint(x, a)
    replay_and_check(capture(fn), [y, a], [ref_y, ref_a], x)


def test_four_step_in_graph():
    n, batch = 1 << 16, 8
    x = to_gpu(synth.uniform_complex(61, (batch, n)))
    p = api.Plan(n, batch, +1)
    ref = p.execute(x)
    y = torch.empty_like(x)
    replay_and_check(capture(lambda: p.execute(x, y)), [y], [ref], x)


def test_one_plan_on_two_streams():
    """A batched plan is immutable after creation: executes of it on two
    streams at once give the eager results."""
    n, batch = 2048, 4096
    p = api.Plan(n, batch, -1)
    xs = [to_gpu(synth.uniform_complex(63, (batch, n), key=(i,))) for i in range(2)]
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


def test_plan_creation_during_capture_is_refused():
    """Plan creation allocates and waits for its tables, which no capture can
    hold.  The binding refuses an uncached shape under capture before
    touching the device (the capture itself stays valid and replays), and
    the C ABI called directly during a capture returns NULL with
    FFT_ECAPTURE; plans created afterwards work as usual."""
    import ctypes
    import oracle
    from paper_2203_09384_amd import native
    from paper_2203_09384_amd.native import MifftError
    from gpu_util import per_transform_relerr
    n, batch = 512, 8
    x = to_gpu(synth.uniform_complex(41, (batch, n)))
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    # 1. the binding: an uncached shape inside a capture
    api._cache.pop((torch.cuda.current_device(), n // 4, batch * 4, -1, "c32"), None)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        y.copy_(x)
        with pytest.raises(MifftError) as ei:
            api.fft(x.view(batch * 4, n // 4))  # no plan cached for (128, 32)
        y.mul_(2.0)
    assert ei.value.status == "FFT_ECAPTURE"
    y.zero_()
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(y, 2.0 * x)
    # 2. the C ABI directly, inside a capture
    L = native.lib()
    g2 = torch.cuda.CUDAGraph()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g2.capture_begin()
        try:
            h = L.fft_plan_create(n, batch, -1, 0)
            rc, msg = L.fft_last_error(), L.fft_last_error_string().decode()
        finally:
            try:
                g2.capture_end()
            except RuntimeError as e:  # the runtime may have invalidated the capture
                print("capture end:", e)
    torch.cuda.synchronize()
    print(f"[case] plan create under capture: handle={h} status={rc} {msg!r}", flush=True)
    if h:
        L.fft_plan_destroy(h)
    assert not h and native.STATUS.get(rc) == "FFT_ECAPTURE", (rc, msg)
    # 3. afterwards the library works as usual
    p = api.Plan(n, batch, -1)
    out = p.execute(x)
    ref = oracle.forward(x.cpu().numpy().astype(np.complex128))
    assert per_transform_relerr(out.cpu().numpy(), ref) <= 1e-5
