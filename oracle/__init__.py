"""CPU oracle for the bit-reversed permutation (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and this
package never imports the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc); this module
only compiles it and marshals numpy arrays into it.  Each wrapper names the
passage of arXiv:1708.01873 that its C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")


def compile_source(src: str, out: str) -> str:
    """Compile an oracle C source into a shared library at ``out``."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-fopenmp", "-fPIC", "-shared",
         src, "-o", tmp])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(LIBRARY):
        compile_source(SOURCE, LIBRARY)
    return LIBRARY


def _check_contig(a: np.ndarray) -> None:
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("oracle: arrays must be C-contiguous")


def _log2_exact(n: int) -> int:
    k = n.bit_length() - 1
    if n <= 0 or (1 << k) != n:
        raise ValueError("oracle: length %d is not a power of two" % n)
    return k


class Oracle:
    """numpy front for one compiled copy of the oracle's C functions."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        L.oracle_rev.argtypes = [ctypes.c_uint64, ctypes.c_int]
        L.oracle_rev.restype = ctypes.c_uint64
        L.oracle_inplace.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
        L.oracle_inplace.restype = ctypes.c_int
        L.oracle_outofplace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_size_t]
        L.oracle_outofplace.restype = ctypes.c_int
        L.oracle_outofplace_mt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_size_t]
        L.oracle_outofplace_mt.restype = ctypes.c_int
        L.oracle_rows.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                  ctypes.c_int64, ctypes.c_size_t]
        L.oracle_rows.restype = ctypes.c_int
        L.oracle_batched.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_size_t]
        L.oracle_batched.restype = ctypes.c_int
        L.oracle_version.restype = ctypes.c_int
        L.oracle_digit_rev.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
        L.oracle_digit_rev.restype = ctypes.c_uint64
        L.oracle_digit_outofplace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_size_t]
        L.oracle_digit_outofplace.restype = ctypes.c_int
        L.oracle_digit_inplace.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_size_t]
        L.oracle_digit_inplace.restype = ctypes.c_int
        L.oracle_evenodd.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_size_t]
        L.oracle_evenodd.restype = ctypes.c_int
        self.lib = L
        self.path = path

    @staticmethod
    def _elems(a: np.ndarray, elem_size):
        _check_contig(a)
        s = a.itemsize if elem_size is None else int(elem_size)
        if s <= 0 or a.nbytes % s:
            raise ValueError("oracle: buffer size is not a multiple of elem_size")
        return s, a.nbytes // s

    def rev(self, i: int, k: int) -> int:
        """Bitwise reversal of the low k bits of i (Introduction, bitwise rev)."""
        return int(self.lib.oracle_rev(int(i), int(k)))

    def inplace(self, a: np.ndarray, elem_size: int | None = None) -> np.ndarray:
        """Permute ``a`` in place, swapping i and rev(i) once per pair
        (Introduction, the in-place listing).  ``a`` holds 2^k elements of
        ``elem_size`` bytes (default: its itemsize).  Returns ``a``."""
        s, n = self._elems(a, elem_size)
        k = _log2_exact(n)
        if self.lib.oracle_inplace(a.ctypes.data, k, s) != 0:
            raise ValueError("oracle_inplace rejected its arguments")
        return a

    def outofplace(self, a: np.ndarray, elem_size: int | None = None) -> np.ndarray:
        """Return dst with dst[rev(i)] = a[i] (Introduction, the buffered
        method's out-of-place statement)."""
        s, n = self._elems(a, elem_size)
        k = _log2_exact(n)
        out = np.empty_like(a)
        if self.lib.oracle_outofplace(a.ctypes.data, out.ctypes.data, k, s) != 0:
            raise ValueError("oracle_outofplace rejected its arguments")
        return out

    def outofplace_mt(self, a: np.ndarray, elem_size: int | None = None):
        """outofplace with the index range split over the host's OpenMP
        threads: the CPU baseline on all cores, and the expected result of
        the full-size comparisons of multi-GiB arrays.  Returns (dst, threads
        used)."""
        s, n = self._elems(a, elem_size)
        k = _log2_exact(n)
        out = np.empty_like(a)
        t = self.lib.oracle_outofplace_mt(a.ctypes.data, out.ctypes.data, k, s)
        if t < 1:
            raise ValueError("oracle_outofplace_mt rejected its arguments")
        return out, t

    def rows(self, a: np.ndarray, k: int, elem_size: int | None = None,
             inplace: bool = False) -> np.ndarray:
        """Permute each consecutive row of 2^k elements independently."""
        s, n = self._elems(a, elem_size)
        if n % (1 << k):
            raise ValueError("oracle: buffer is not a whole number of rows")
        out = a if inplace else np.empty_like(a)
        if self.lib.oracle_rows(a.ctypes.data, out.ctypes.data, k, n >> k, s) != 0:
            raise ValueError("oracle_rows rejected its arguments")
        return out

    def batched(self, data: np.ndarray, offsets, log2n,
                elem_size: int | None = None) -> np.ndarray:
        """Permute each packed array [offsets[a], offsets[a+1]) in place."""
        s, n = self._elems(data, elem_size)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        log2n = np.ascontiguousarray(log2n, dtype=np.int32)
        num = log2n.shape[0]
        if offsets.shape[0] != num + 1 or (num and offsets[-1] > n) or (num and offsets[0] < 0):
            raise ValueError("oracle: offsets do not fit the data")
        if self.lib.oracle_batched(data.ctypes.data, offsets.ctypes.data, log2n.ctypes.data,
                                   num, s) != 0:
            raise ValueError("oracle_batched rejected its arguments")
        return data

    def digit_rev(self, i: int, k: int, d: int) -> int:
        """Reverse the order of the d-bit digits of the k-bit index i."""
        return int(self.lib.oracle_digit_rev(int(i), int(k), int(d)))

    def digit_outofplace(self, a: np.ndarray, d: int, elem_size: int | None = None) -> np.ndarray:
        """dst[drev(i)] = a[i], digits of d bits."""
        s, n = self._elems(a, elem_size)
        k = _log2_exact(n)
        out = np.empty_like(a)
        if self.lib.oracle_digit_outofplace(a.ctypes.data, out.ctypes.data, k, d, s) != 0:
            raise ValueError("oracle_digit_outofplace rejected its arguments")
        return out

    def digit_inplace(self, a: np.ndarray, d: int, elem_size: int | None = None) -> np.ndarray:
        s, n = self._elems(a, elem_size)
        k = _log2_exact(n)
        if self.lib.oracle_digit_inplace(a.ctypes.data, k, d, s) != 0:
            raise ValueError("oracle_digit_inplace rejected its arguments")
        return a

    def evenodd(self, a: np.ndarray, elem_size: int | None = None) -> np.ndarray:
        """One even-odd split: evens first, then odds (Introduction, Stockham)."""
        s, n = self._elems(a, elem_size)
        k = _log2_exact(n)
        out = np.empty_like(a)
        if self.lib.oracle_evenodd(a.ctypes.data, out.ctypes.data, k, s) != 0:
            raise ValueError("oracle_evenodd rejected its arguments")
        return out

    def rev_table(self, k: int) -> np.ndarray:
        """rev_k(j) for every j, read off the in-place permutation of 0..n-1."""
        return self.inplace(np.arange(1 << k, dtype=np.int64))


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(LIBRARY):
            build(force=True)
        _default = Oracle(LIBRARY)
    return _default


def rev(i: int, k: int) -> int:
    return default().rev(i, k)


def inplace(a, elem_size=None):
    return default().inplace(a, elem_size)


def outofplace(a, elem_size=None):
    return default().outofplace(a, elem_size)


def outofplace_mt(a, elem_size=None):
    return default().outofplace_mt(a, elem_size)


def rows(a, k, elem_size=None, inplace=False):
    return default().rows(a, k, elem_size, inplace)


def batched(data, offsets, log2n, elem_size=None):
    return default().batched(data, offsets, log2n, elem_size)


def rev_table(k: int) -> np.ndarray:
    return default().rev_table(k)


def digit_rev(i: int, k: int, d: int) -> int:
    return default().digit_rev(i, k, d)


def digit_outofplace(a, d, elem_size=None):
    return default().digit_outofplace(a, d, elem_size)


def digit_inplace(a, d, elem_size=None):
    return default().digit_inplace(a, d, elem_size)


def evenodd(a, elem_size=None):
    return default().evenodd(a, elem_size)
