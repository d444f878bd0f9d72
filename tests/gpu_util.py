"""Helpers for the GPU parity tests: move opaque s-byte elements between numpy
and the device, and compare byte for byte."""
from __future__ import annotations

import numpy as np

NP_DTYPE = {1: np.uint8, 2: np.int16, 4: np.int32, 8: np.int64, 16: np.complex128}


def torch_dtype(s: int):
    import torch
    return {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64,
            16: torch.complex128}[s]


def to_device(host_bytes: np.ndarray, s: int, pad_front: int = 0):
    """Upload raw bytes as a contiguous tensor of s-byte elements.  With
    pad_front > 0 the returned view starts pad_front elements into a larger
    allocation (a base pointer that is only s-byte aligned)."""
    import torch
    buf = np.ascontiguousarray(host_bytes).view(np.uint8)
    assert buf.nbytes % s == 0
    n = buf.nbytes // s
    t = torch.empty(n + pad_front, dtype=torch_dtype(s), device="cuda")
    if n:
        t[pad_front:].copy_(torch.from_numpy(buf.view(NP_DTYPE[s]).copy()))
    return t[pad_front:]


def to_host_bytes(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().contiguous().cpu().numpy().view(np.uint8).reshape(-1)


def assert_bytes_equal(got: np.ndarray, want: np.ndarray, what: str = "") -> None:
    got = np.ascontiguousarray(got).view(np.uint8).reshape(-1)
    want = np.ascontiguousarray(want).view(np.uint8).reshape(-1)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError("%s: %d bytes differ, first at byte %d" % (what, bad.size, bad[0]))


def assert_device_equal(t, want: np.ndarray, what: str = "", chunk: int = 1 << 28) -> None:
    """Byte-exact comparison of a device tensor with a host array of the same
    size, copied back a chunk at a time through one pinned host buffer, so a
    multi-GiB result is compared in full without a second host copy of it."""
    import torch
    torch.cuda.synchronize()
    dev = t.detach().contiguous().view(torch.uint8).reshape(-1)
    want = np.ascontiguousarray(want).view(np.uint8).reshape(-1)
    assert dev.numel() == want.size, (what, dev.numel(), want.size)
    buf = torch.empty(min(chunk, max(1, dev.numel())), dtype=torch.uint8, pin_memory=True)
    view = buf.numpy()
    for lo in range(0, dev.numel(), chunk):
        hi = min(dev.numel(), lo + chunk)
        buf[:hi - lo].copy_(dev[lo:hi])
        torch.cuda.synchronize()
        got = view[:hi - lo]
        if not np.array_equal(got, want[lo:hi]):
            bad = np.flatnonzero(got != want[lo:hi])
            raise AssertionError("%s: %d bytes differ in [%d, %d), first at byte %d"
                                 % (what, bad.size, lo, hi, lo + bad[0]))
