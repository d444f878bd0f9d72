"""Bit-reversal generators that are independent of the oracle's arithmetic.

Each one follows a different passage of arXiv:1708.01873 and shares nothing
with ``oracle/oracle.c``; the oracle's pins compare against them.
"""
from __future__ import annotations

import os

# Reversed-byte table (Introduction, bytewise bit reversal): entry B is the
# byte B with its 8 bits in reverse order.  Built by reversing the binary
# string, not by shifting bits, so it cannot share a mistake with a shift loop.
BYTE_TABLE = [int(format(b, "08b")[::-1], 2) for b in range(256)]


def rev_bytetable(i: int, k: int) -> int:
    """Reverse the low k bits of i (0 <= k <= 64) eight bits at a time."""
    r = 0
    for byte in range(8):
        r = (r << 8) | BYTE_TABLE[(i >> (8 * byte)) & 0xFF]
    return r >> (64 - k)


def rev_bytetable_array(idx, k: int):
    """rev_bytetable on a numpy array of indices (uint64 arithmetic, the same
    string-built table), for brute force at millions of indices."""
    import numpy as np
    table = np.array(BYTE_TABLE, dtype=np.uint64)
    i = np.asarray(idx, dtype=np.uint64)
    r = np.zeros_like(i)
    for byte in range(8):
        r = (r << np.uint64(8)) | table[(i >> np.uint64(8 * byte)) & np.uint64(0xFF)]
    return r >> np.uint64(64 - k) if k else np.zeros_like(i)


def rev_sequence_xor(k: int) -> list[int]:
    """rev_k(i) for i = 0 .. 2^k - 1 by the inductive XOR method (Methods,
    inductive XOR): i ^ (i+1) is a run of t low ones; reversed within k bits it
    is that run shifted left by k - t, and flipping those bits of rev(i) gives
    rev(i+1)."""
    n = 1 << k
    out = [0] * n
    r = 0
    for i in range(n - 1):
        mask = i ^ (i + 1)
        t = mask.bit_length()
        r ^= mask << (k - t)
        out[i + 1] = r
    return out


def evenodd_step(a: list) -> list:
    """One even-odd (Stockham) split: even positions first, then odd ones
    (Introduction, the n/2 x 2 transpose)."""
    return list(a[0::2]) + list(a[1::2])


def bitrev_evenodd_chain(a: list) -> list:
    """Bit-reversed order as the nested chain of even-odd splits (Introduction:
    doing every recursive even-odd split up front is the bit-reversed
    permutation)."""
    if len(a) <= 1:
        return list(a)
    h = evenodd_step(a)
    half = len(a) // 2
    return bitrev_evenodd_chain(h[:half]) + bitrev_evenodd_chain(h[half:])


def read_golden(name: str) -> dict[str, str]:
    """Parse a ``key = value`` fixture under tests/golden (``#`` comments)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition("=")
            out[key.strip()] = val.strip()
    return out
