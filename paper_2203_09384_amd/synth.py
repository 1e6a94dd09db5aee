"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no transform arithmetic: it only draws numbers.  Both the
GPU path and the CPU oracle consume what it returns, so neither side's
inputs ever come from the other.

Streams are numpy PCG64 generators keyed by ``(seed, *key)`` through
``SeedSequence`` so that, for example, every length of a sweep draws from
its own reproducible stream.  Values are drawn in float64 and rounded once
to the storage type; the oracle reads exactly the stored values.
"""
from __future__ import annotations

import numpy as np

# Seeds of the workloads (recorded in every bench line).
SEED_PLAIN = 20220317        # N=256 batch 64 and the per-N sweep
SEED_AUTOGRAD = 20220318     # x and w of the differentiable-loss workload
SEED_RAGGED = 20220319       # ragged lengths and values
SEED_HALF = 20220320         # reduced-precision inputs
SEED_REAL = 20220321         # real-input transforms


def rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=tuple(int(k) for k in key))))


def uniform_complex(seed: int, shape, key=(), dtype=np.complex64) -> np.ndarray:
    """re, im i.i.d. uniform[-1, 1), drawn in float64 then rounded to dtype."""
    g = rng(seed, *key)
    shape = tuple(np.atleast_1d(shape))
    re = g.uniform(-1.0, 1.0, size=shape)
    im = g.uniform(-1.0, 1.0, size=shape)
    out = np.empty(shape, dtype=dtype)
    out.real = re
    out.imag = im
    return out


def uniform_real(seed: int, shape, key=(), dtype=np.float32) -> np.ndarray:
    """i.i.d. uniform[-1, 1), drawn in float64 then rounded to dtype."""
    g = rng(seed, *key)
    return g.uniform(-1.0, 1.0, size=tuple(np.atleast_1d(shape))).astype(dtype)


def log_uniform_polar(seed: int, shape, key=(), lo: float = 1e-3, hi: float = 1e3) -> np.ndarray:
    """Magnitude log-uniform in [lo, hi], phase uniform in [0, 2 pi); complex128."""
    g = rng(seed, *key)
    shape = tuple(np.atleast_1d(shape))
    mag = np.exp(g.uniform(np.log(lo), np.log(hi), size=shape))
    ph = g.uniform(0.0, 2.0 * np.pi, size=shape)
    return mag * np.cos(ph) + 1j * (mag * np.sin(ph))


def uniform_weights(seed: int, shape, key=(), dtype=np.float32) -> np.ndarray:
    """w i.i.d. uniform[0, 1)."""
    g = rng(seed, *key)
    return g.uniform(0.0, 1.0, size=tuple(np.atleast_1d(shape))).astype(dtype)


def ramp(n: int, batch: int = 1, dtype=np.complex64) -> np.ndarray:
    """The paper's evaluation signal f(x) = x sampled as x_n = n (imaginary 0)."""
    return np.tile(np.arange(n, dtype=np.float64), (batch, 1)).astype(dtype)


def ragged_lengths(seed: int, count: int, lo_log2: int = 3, hi_log2: int = 11, key=()) -> np.ndarray:
    """Lengths 2^L with L uniform on {lo_log2, ..., hi_log2}; int64."""
    g = rng(seed, *key)
    L = g.integers(lo_log2, hi_log2 + 1, size=count)
    return (np.int64(1) << L.astype(np.int64)).astype(np.int64)


def offsets_from_lengths(lengths) -> np.ndarray:
    """Packed, contiguous CSR-style offsets: offsets[0] = 0, offsets[b+1] - offsets[b] = lengths[b]."""
    lengths = np.asarray(lengths, dtype=np.int64)
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off
