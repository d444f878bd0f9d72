"""Seeded synthetic inputs shared by the tests and the benchmark.

Nothing here computes any part of the permutation: these are only the
input recipes (shapes, value distributions, seeds).  The paper measures on
arrays of complex doubles of n = 2^8 .. 2^30 elements (Results) and uses no
public dataset; these recipes stand in for that workload at the sizes the
benchmark configurations name.  All randomness is numpy's PCG64
(``default_rng(seed)``).
"""
from __future__ import annotations

import numpy as np

SEEDS = {"c1": 1, "c2": 2, "c3a": 3, "c3b": 4, "c4": 5, "c5": 6}
EXTRA_PARITY_SEEDS = (7, 8)


def uint32_uniform(k: int, seed: int) -> np.ndarray:
    """2^k uint32 values uniform over [0, 2^32)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, size=1 << k, dtype=np.uint32)


def iota(k: int, dtype=np.uint32) -> np.ndarray:
    """0, 1, ..., 2^k - 1: after the permutation, entry j must hold rev_k(j)."""
    return np.arange(1 << k, dtype=dtype)


def complex64_normal(k: int, seed: int) -> np.ndarray:
    """2^k complex64 values with real and imaginary parts i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    n = 1 << k
    out = np.empty(n, dtype=np.complex64)
    parts = out.view(np.float32).reshape(n, 2)
    parts[:, 0] = rng.standard_normal(n, dtype=np.float32)
    parts[:, 1] = rng.standard_normal(n, dtype=np.float32)
    return out


def complex128_normal(k: int, seed: int, chunk_log2: int = 24) -> np.ndarray:
    """2^k complex128 values, real and imaginary parts i.i.d. N(0, 1),
    generated in chunks of 2^chunk_log2 so that peak host memory stays at the
    output plus one chunk."""
    rng = np.random.default_rng(seed)
    n = 1 << k
    out = np.empty(n, dtype=np.complex128)
    parts = out.view(np.float64).reshape(n, 2)
    step = 1 << min(chunk_log2, k)
    for lo in range(0, n, step):
        parts[lo:lo + step, 0] = rng.standard_normal(step)
        parts[lo:lo + step, 1] = rng.standard_normal(step)
    return out


def float32_normal(k: int, seed: int, chunk_log2: int = 26) -> np.ndarray:
    """2^k float32 values i.i.d. N(0, 1), generated in chunks."""
    rng = np.random.default_rng(seed)
    n = 1 << k
    out = np.empty(n, dtype=np.float32)
    step = 1 << min(chunk_log2, k)
    for lo in range(0, n, step):
        out[lo:lo + step] = rng.standard_normal(step, dtype=np.float32)
    return out


def batched_layout(num_arrays: int, kmin: int, kmax: int, seed: int):
    """Uneven batch: log2n[a] uniform integer in [kmin, kmax], arrays packed
    back to back; offsets (int64, num_arrays + 1 entries) count elements."""
    rng = np.random.default_rng(seed)
    log2n = rng.integers(kmin, kmax + 1, size=num_arrays).astype(np.int32)
    offsets = np.zeros(num_arrays + 1, dtype=np.int64)
    np.cumsum(np.left_shift(np.int64(1), log2n.astype(np.int64)), out=offsets[1:])
    return offsets, log2n


def batched_complex64(num_arrays: int, kmin: int, kmax: int, seed: int):
    """(data, offsets, log2n): the uneven batch filled with complex64 values,
    real and imaginary parts i.i.d. N(0, 1) (one stream after the layout)."""
    offsets, log2n = batched_layout(num_arrays, kmin, kmax, seed)
    data = complex64_normal_flat(int(offsets[-1]), seed + 1000)
    return data, offsets, log2n


def complex64_normal_flat(n: int, seed: int, chunk: int = 1 << 24) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.complex64)
    parts = out.view(np.float32).reshape(n, 2)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        parts[lo:hi, 0] = rng.standard_normal(hi - lo, dtype=np.float32)
        parts[lo:hi, 1] = rng.standard_normal(hi - lo, dtype=np.float32)
    return out


def rows_float32(rows: int, k: int, seed: int):
    """(x, w): two [rows, 2^k] float32 arrays, i.i.d. N(0, 1) (x first)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((rows, 1 << k), dtype=np.float32)
    w = rng.standard_normal((rows, 1 << k), dtype=np.float32)
    return x, w


def sample_coordinates(total: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct flat coordinates out of `total`, sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(total, size=count, replace=False))


def byte_pattern(n_bytes: int, seed: int) -> np.ndarray:
    """Uniform random bytes (element-size agnostic payload)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=n_bytes, dtype=np.uint8)


def device_normal(n: int, seed: int, dtype=None, device: str = "cuda"):
    """n i.i.d. N(0, 1) values generated on the device with torch's seeded
    Philox generator (for the multi-GiB configurations, where host generation
    and upload would dominate).  Complex dtypes get i.i.d. N(0, 1) real and
    imaginary parts."""
    import torch
    dtype = dtype or torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if dtype.is_complex:
        real = torch.float32 if dtype == torch.complex64 else torch.float64
        return torch.randn(2 * n, dtype=real, device=device, generator=g).view(dtype)
    return torch.randn(n, dtype=dtype, device=device, generator=g)
