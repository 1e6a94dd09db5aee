"""C ABI checks that need no GPU: exports, argument validation before any HIP
call, and host-side planning."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

from paper_2203_09384_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mifft.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fft_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = native.lib()
    declared = header_functions()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(native.EXPORTS)
    assert L.fft_version().decode().startswith("mifft")


def q(n, batch=1, sign=-1, dtype=0):
    d = native.PlanDesc()
    rc = native.lib().fft_plan_query(n, batch, sign, dtype, ctypes.byref(d))
    return rc, d


@pytest.mark.parametrize("n", [0, 1, 3, 12, 1 << 21, -8, 2049, 4097])
def test_bad_n(n):
    assert q(n)[0] == 1


@pytest.mark.parametrize("L", range(12, 21))
def test_large_lengths_plan(L):
    """2^12..2^14: one pass with the whole transform in one workgroup's LDS;
    above: the two-pass four-step split (variant 9)."""
    n = 1 << L
    rc, d = q(n, 3, -1)
    assert rc == 0 and (d.variant == 9) == (L > 14)
    assert int(np.prod(list(d.radices)[: d.npasses])) == n
    assert q(n, 3, -1, 1)[0] == 1  # above 2048 only FP32


def test_bad_batch_sign_dtype_null():
    assert q(256, 0)[0] == 2
    assert q(256, -5)[0] == 2
    assert q(2048, 1 << 40)[0] == 2
    assert q(256, 1, 0)[0] == 3
    assert q(256, 1, 2)[0] == 3
    assert q(256, 1, -1, 7)[0] == 4
    L = native.lib()
    assert L.fft_plan_query(256, 1, -1, 0, None) == 5
    assert L.fft_execute(None, None, None, None) == 5
    assert L.fft_last_error() == 5
    assert b"NULL" in L.fft_last_error_string()
    assert L.fft_plan_describe(None, None) == 5
    L.fft_plan_destroy(None)  # NULL-safe


@pytest.mark.parametrize("L", range(1, 12))
def test_query_plans_are_consistent(L):
    n = 1 << L
    for sign in (-1, 1):
        rc, d = q(n, 1000, sign)
        assert rc == 0
        assert int(np.prod(list(d.radices)[: d.npasses])) == n
        assert d.ept * (d.wg // d.transforms_per_wg) == n
        assert d.grid == -(-1000 // d.transforms_per_wg)
        assert d.scale == (1.0 if sign < 0 else np.float32(1.0 / n))
        assert all(r in (2, 4, 8, 16) for r in list(d.radices)[: d.npasses])


def test_validation_happens_before_hip():
    """Bad arguments report their own status even where no device exists."""
    L = native.lib()
    assert L.fft_plan_create(12, 1, -1, 0) is None and L.fft_last_error() == 1
    assert L.fft_plan_create(256, 0, -1, 0) is None and L.fft_last_error() == 2
    assert L.fft_plan_create(256, 1, 3, 0) is None and L.fft_last_error() == 3
    assert L.fft_plan_create(256, 1, -1, 9) is None and L.fft_last_error() == 4
    assert L.fft_plan_create_config(256, 1, -1, 0, 3, 256, 0) is None and L.fft_last_error() == 10
    bad = [np.array([0, 8, 20], np.int64), np.array([1, 9], np.int64),
           np.array([0, 4096], np.int64), np.array([0, 8, 8], np.int64)]
    for off in bad:
        p = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        assert L.fft_plan_create_ragged(len(off) - 1, p, -1, 0) is None
        assert L.fft_last_error() == 7, off
    off = np.array([0, 8, 16], np.int64)
    p = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    assert L.fft_plan_create_ragged(2, None, -1, 0) is None and L.fft_last_error() == 5
    assert L.fft_plan_create_ragged(0, p, -1, 0) is None and L.fft_last_error() == 2
    assert L.fft_plan_create_ragged(2, p, 0, 0) is None and L.fft_last_error() == 3


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device path")
def test_no_device_is_reported_as_hip_error():
    L = native.lib()
    assert L.fft_plan_create(256, 4, -1, 0) is None
    assert L.fft_last_error() == 8
    assert b"hipGetDevice" in L.fft_last_error_string()


def test_half_precision_queries():
    rc, d = q(2048, 32768, -1, 1)
    assert rc == 0 and d.radices[:3] == [8, 16, 16] and d.wg == 256
    rc, d = q(2048, 4, 1, 2)
    assert rc == 0 and d.scale == np.float32(1.0 / 2048)
    for L in range(1, 11):               # FP16/BF16 below 2048: FP32 passes, 16-bit storage
        rc, d = q(1 << L, 100, 1, 1)
        assert rc == 0 and int(np.prod(list(d.radices)[: d.npasses])) == 1 << L
        assert d.scale == np.float32(1.0 / (1 << L))
    assert q(4096, 4, -1, 1)[0] == 1     # half precision stops at 2048
    # N = 2048: runs of 4 consecutive transforms per workgroup, longer runs
    # only when the grid would pass one launch's 2^32 - 1 work-items
    max_grid = ((1 << 32) - 1) // 256
    for batch in (1, 3, 4, 5, 32768, 4 * max_grid, 4 * max_grid + 1, 1 << 29):  # 2^40 elements
        rc, d = q(2048, batch, -1, 2)
        t = d.transforms_per_wg
        assert rc == 0 and d.grid == -(-batch // t) and d.grid <= max_grid, batch
        assert t == 4 if batch <= 4 * max_grid else (t - 1) * max_grid < batch <= t * max_grid, batch
    L = native.lib()
    assert L.fft_execute_scaled(None, None, None, None, None, None) == 5


def test_fused_loss_argument_checks():
    L = native.lib()
    assert L.fft_execute_loss_grad(None, None, None, None, None, None) == 5


def test_tune_table_is_read(tmp_path):
    """MIFFT_TUNE_TABLE overrides the built-in variant choice (host-only query)."""
    import subprocess
    import sys
    table = tmp_path / "tune.txt"
    table.write_text("# test table\nc32 8 4 64 2\nc32 11 8 256 4  # comment\nragged 5 8\n")
    code = ("import ctypes, sys; sys.path.insert(0, %r);"
            "from paper_2203_09384_amd import native;"
            "L = native.lib(); d = native.PlanDesc();"
            "assert L.fft_plan_query(256, 10, -1, 0, ctypes.byref(d)) == 0;"
            "print(d.ept, d.wg, d.variant);"
            "assert L.fft_plan_query(2048, 10, -1, 0, ctypes.byref(d)) == 0;"
            "print(d.ept, d.wg, d.variant)") % ROOT
    env = dict(os.environ, MIFFT_TUNE_TABLE=str(table))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["4", "64", "2", "8", "256", "4"]


# ---------------------------------------------------------------- real input
@pytest.mark.parametrize("L", range(1, 16))
def test_real_input_queries(L):
    """FFT_R32 plans describe the half-length complex transform they run;
    every built-in choice is a compiled kernel (query checks that)."""
    n, m = 1 << L, 1 << (L - 1)
    for sign in (-1, 1):
        rc, d = q(n, 1000, sign, 3)
        assert rc == 0, native.lib().fft_last_error_string()
        assert d.dtype == 3 and d.n == n
        assert int(np.prod(list(d.radices)[: d.npasses])) == m
        assert d.ept * (d.wg // d.transforms_per_wg) == m
        assert d.grid == -(-1000 // d.transforms_per_wg)
        assert d.scale == (1.0 if sign < 0 else np.float32(1.0 / n))


@pytest.mark.parametrize("L", range(16, 22))
def test_large_real_input_queries(L):
    """Above 2^15 a real-input plan runs the half-length four-step split."""
    n, m = 1 << L, 1 << (L - 1)
    for sign in (-1, 1):
        rc, d = q(n, 7, sign, 3)
        assert rc == 0, native.lib().fft_last_error_string()
        assert d.dtype == 3 and d.n == n and d.variant == 9
        assert int(np.prod(list(d.radices)[: d.npasses])) == m
        assert d.scale == (1.0 if sign < 0 else np.float32(1.0 / n))


def test_real_input_validation():
    L = native.lib()
    assert q(1 << 22, 1, -1, 3)[0] == 1      # real lengths stop at 2^21
    assert q(24, 1, -1, 3)[0] == 1
    assert L.fft_plan_create(1 << 22, 1, -1, 3) is None and L.fft_last_error() == 1
    assert L.fft_plan_create_config(256, 1, -1, 3, 4, 64, 5) is None and L.fft_last_error() == 10
    assert L.fft_plan_create_config(256, 1, -1, 3, 4, 48, 2) is None and L.fft_last_error() == 10


def test_nd_validation():
    """fft_plan_create_nd checks its arguments before touching a device."""
    L = native.lib()

    def create(dims, batch=1, sign=-1, dtype=0, rank=None):
        arr = (ctypes.c_int64 * max(1, len(dims)))(*dims)
        h = L.fft_plan_create_nd(len(dims) if rank is None else rank, arr, batch, sign, dtype)
        return h, L.fft_last_error()

    assert create([4, 4], rank=0) == (None, 1)
    assert create([4, 4, 4, 4]) == (None, 1)
    assert create([4096, 4]) == (None, 1)       # non-last axes stop at 2048
    assert create([12, 4]) == (None, 1)
    assert create([4, 1 << 21]) == (None, 1)
    assert create([4, 4], batch=0) == (None, 2)
    assert create([4, 4], sign=0) == (None, 3)
    assert create([4, 4], dtype=1) == (None, 4)
    assert L.fft_plan_create_nd(2, None, 1, -1, 0) is None and L.fft_last_error() == 5


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device path")
def test_nd_axis_kernels_are_compiled():
    """Valid multidimensional plans get past the kernel lookup for every
    axis length (they fail only for want of a device here)."""
    L = native.lib()
    for d0 in [1 << k for k in range(1, 12)]:
        arr = (ctypes.c_int64 * 3)(d0, 4, 8)
        assert L.fft_plan_create_nd(3, arr, 2, -1, 0) is None
        assert L.fft_last_error() == 8, (d0, L.fft_last_error_string())
        arr = (ctypes.c_int64 * 2)(d0, 16)
        assert L.fft_plan_create_nd(2, arr, 2, 1, 0) is None
        assert L.fft_last_error() == 8, (d0, L.fft_last_error_string())


@pytest.mark.parametrize("L", range(1, 12))
def test_compiled_variant_listing(L):
    """fft_c32_variants lists distinct configurations, each consistent with
    n, and includes the tuned default that fft_plan_query picks."""
    from paper_2203_09384_amd import api
    n = 1 << L
    vs = api.c32_variants(n)
    assert len(vs) == len(set(vs)) >= 1
    for ept, wg, var in vs:
        assert ept in (2, 4, 8, 16) and 64 <= wg <= 1024 and (0 <= var <= 8 or (var == 11 and ept == n) or (var == 12 and 32 <= n <= 1024))
        assert ept <= n
    rc, d = q(n, 1000, -1)
    assert rc == 0 and (d.ept, d.wg, d.variant) in vs
    Lib = native.lib()
    assert Lib.fft_c32_variants(n, None, 0) == len(vs)
    assert Lib.fft_c32_variants(3, None, 0) == -1 and Lib.fft_last_error() == 1
    assert Lib.fft_c32_variants(4096, None, 0) == -1
    assert Lib.fft_c32_variants(n, None, 1) == -1 and Lib.fft_last_error() == 5

