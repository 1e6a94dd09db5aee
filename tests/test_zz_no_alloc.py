"""fft_execute_static_scratch (the execute that allocates nothing) against
fft_execute, called through the C ABI.

Real-input plans above 2^15 run the half-length four-step transform into a
workspace; the static-scratch execute puts that intermediate in the
library's static array instead.  Both run the same kernels in the same
order, so the outputs must agree bit for bit; each is also held to the FP32
bar (relative L2 <= 1e-5 per transform) against the FP64 oracle on sampled
transforms.  Two calls in a row, the second on a smaller input (the array
keeps the first call's contents), both directions, a plan without a
workspace (plain execute), and the size limit's error.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, native, synth
from gpu_util import need_gpu, per_transform_relerr

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _run(entry, plan, x, out):
    L = native.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = entry(ctypes.c_void_p(plan._h), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), stream)
    torch.cuda.synchronize()
    if rc != 0:
        raise native.MifftError(rc, L.fft_last_error_string().decode())


def _pair(n, batch, sign, seed_key):
    """One plan, both executes on the same input; returns (plain, static, input)."""
    L = native.lib()
    if sign < 0:
        x_np = synth.uniform_real(synth.SEED_REAL, (batch, n), key=seed_key)
        out_shape, out_dtype = (batch, n // 2 + 1), torch.complex64
    else:
        x_np = synth.uniform_complex(synth.SEED_REAL, (batch, n // 2 + 1), key=seed_key)
        out_shape, out_dtype = (batch, n), torch.float32
    x = torch.from_numpy(x_np).cuda()
    plan = api.Plan(n, batch, sign, "r32")
    print(f"[case] static scratch n={n} batch={batch} sign={sign} {plan.describe()}", flush=True)
    # stale values in the outputs, so an element left unwritten would show
    y_plain = torch.full(out_shape, 7.0, dtype=torch.float32).to(out_dtype).cuda()
    y_static = torch.full(out_shape, -3.0, dtype=torch.float32).to(out_dtype).cuda()
    _run(L.fft_execute, plan, x, y_plain)
    _run(L.fft_execute_static_scratch, plan, x, y_static)
    return y_plain.cpu().numpy(), y_static.cpu().numpy(), x_np


def _check_oracle(y, x_np, sign, rows):
    x64 = x_np[rows].astype(np.complex128 if sign > 0 else np.float64)
    ref = oracle.rfft(x64) if sign < 0 else oracle.irfft(x64, y.shape[-1])
    assert per_transform_relerr(y[rows], ref) <= TOL


@pytest.mark.parametrize("sign", [-1, +1])
def test_two_calls_second_smaller(sign):
    # first call: 2^17 reals x 40 transforms (20 MiB of scratch); second:
    # 2^16 x 8 (2 MiB), after the first left its spectra in the array
    for n, batch in ((1 << 17, 40), (1 << 16, 8)):
        y_plain, y_static, x_np = _pair(n, batch, sign, (n, batch, sign + 1))
        assert y_plain.tobytes() == y_static.tobytes()
        _check_oracle(y_static, x_np, sign, [0, batch // 2, batch - 1])


def test_largest_batch_that_fits():
    n = 1 << 21
    batch = native.STATIC_SCRATCH_BYTES // ((n // 2) * 8)  # 8 transforms: the array exactly
    y_plain, y_static, x_np = _pair(n, batch, -1, (n, batch))
    assert y_plain.tobytes() == y_static.tobytes()
    _check_oracle(y_static, x_np, -1, [batch - 1])


def test_plan_without_workspace_is_plain_execute():
    n, batch = 2048, 33
    x_np = synth.uniform_complex(synth.SEED_PLAIN, (batch, n), key=(n, 77))
    x = torch.from_numpy(x_np).cuda()
    plan = api.Plan(n, batch, -1)
    y1 = torch.empty_like(x)
    y2 = torch.empty_like(x)
    L = native.lib()
    _run(L.fft_execute, plan, x, y1)
    _run(L.fft_execute_static_scratch, plan, x, y2)
    assert y1.cpu().numpy().tobytes() == y2.cpu().numpy().tobytes()


def test_beyond_the_array_is_refused():
    n = 1 << 20
    batch = native.STATIC_SCRATCH_BYTES // ((n // 2) * 8) + 1  # one transform more than fits
    x = torch.zeros((batch, n), dtype=torch.float32, device="cuda")
    y = torch.zeros((batch, n // 2 + 1), dtype=torch.complex64, device="cuda")
    plan = api.Plan(n, batch, -1, "r32")
    with pytest.raises(native.MifftError) as ei:
        _run(native.lib().fft_execute_static_scratch, plan, x, y)
    assert ei.value.status == "FFT_EINVAL_BATCH"
    assert "static scratch" in str(ei.value)
