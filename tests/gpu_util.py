"""Helpers shared by the GPU tests: device checks and error measures."""
import numpy as np
import pytest
import torch


def need_gpu():
    """GPU tests run only where a GPU is visible; the library itself must then
    be built (no fallback exists, a missing library fails the test)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def per_transform_relerr(y, ref):
    """max_b ||y_b - ref_b||_2 / ||ref_b||_2 over transforms b (last axis), in FP64."""
    y = np.asarray(y, np.complex128)
    ref = np.asarray(ref, np.complex128)
    num = np.linalg.norm((y - ref).reshape(-1, y.shape[-1]), axis=-1)
    den = np.linalg.norm(ref.reshape(-1, ref.shape[-1]), axis=-1)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den))


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_cpu(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()
