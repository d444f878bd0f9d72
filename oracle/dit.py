"""CPU oracle: bit reversal followed by the first L radix-2 decimation-in-time
FFT stages (test infrastructure only; see oracle/__init__.py for who may use
it).

The paper's motivation (Introduction): the Cooley-Tukey FFT reduces a DFT of
length n to DFTs of the even- and odd-indexed halves; doing all those
even-odd splits first is the bit-reversed permutation, after which every
level of the FFT works on contiguous blocks.  After the permutation and the
first L levels (stages), the block J of 2^L consecutive outputs holds the
length-2^L DFT of the subsequence x[r + 2^(k-L) u], u = 0 .. 2^L - 1, with
r = rev_{k-L}(J):

    out[J 2^L + f] = sum_u x[rev_{k-L}(J) + 2^(k-L) u] exp(-+ 2 pi i u f / 2^L).

``dit_stages`` is that closed form in complex128 (a DFT-matrix product per
column of the reshaped input, and the C oracle's reversal for the block
order).  ``dit_stages_iterative`` takes the algorithm's own steps (reverse,
then L levels of butterflies) as an independent second statement; the pins
in tests/test_dit_oracle.py check the two against each other, against
numpy's FFT when L = k, against the plain reversal when L = 0, and against an
impulse's closed form.
"""
from __future__ import annotations

import numpy as np

from . import default as _default


def _k_of(n: int) -> int:
    k = int(n).bit_length() - 1
    if n <= 0 or (1 << k) != n:
        raise ValueError("length %d is not a power of two" % n)
    return k


def dit_stages(x: np.ndarray, stages: int, inverse: bool = False,
               precision=np.complex128) -> np.ndarray:
    """Closed form of bit reversal + the first `stages` DIT levels, computed in
    `precision` (complex128 by default; np.clongdouble gives a reference
    clearly more accurate than a complex128 computation under test)."""
    x = np.asarray(x).astype(precision).reshape(-1)
    k = _k_of(x.size)
    L = int(stages)
    if not 0 <= L <= k:
        raise ValueError("stages must be in [0, log2 n]")
    q = 1 << L
    real = np.longdouble if precision == np.clongdouble else np.float64
    sign = real(1) if inverse else real(-1)
    u = np.arange(q)
    # angle 2 pi (u f mod q) / q, reduced before scaling so it stays accurate
    ang = (np.outer(u, u) % q).astype(real) * (real(2) * real(np.pi) if real is np.float64
                                               else real(2) * np.arccos(real(-1))) / real(q)
    W = (np.cos(ang) + 1j * sign * np.sin(ang)).astype(precision)  # W[f, u]
    cols = x.reshape(q, x.size // q)                    # cols[u, r] = x[r + 2^(k-L) u]
    F = W @ cols                                        # F[f, r]
    rev = _default().rev_table(k - L)                   # block J takes column rev(J)
    return np.ascontiguousarray(F[:, rev].T).reshape(-1)


def dit_stages_iterative(x: np.ndarray, stages: int, inverse: bool = False) -> np.ndarray:
    """The same result by the algorithm's steps: the oracle's bit reversal,
    then for s = 1 .. L the radix-2 butterflies on blocks of 2^s:
    (a, b) -> (a + w^t b, a - w^t b), w = exp(-+ 2 pi i / 2^s)."""
    y = _default().outofplace(np.asarray(x).astype(np.complex128).reshape(-1))
    sign = 1.0 if inverse else -1.0
    for s in range(1, int(stages) + 1):
        half = 1 << (s - 1)
        blocks = y.reshape(-1, 2 * half)
        w = np.exp(sign * 2j * np.pi * np.arange(half) / (2 * half))
        a = blocks[:, :half].copy()
        b = blocks[:, half:] * w
        blocks[:, :half] = a + b
        blocks[:, half:] = a - b
    return y


def higham_bound(stages: int, unit_roundoff: float, twiddle_error: float) -> float:
    """Norm-wise relative error bound of an L-level radix-2 FFT evaluated in
    floating point with precomputed twiddles of error <= twiddle_error
    (Higham, Accuracy and Stability of Numerical Algorithms, thm. 24.2):
    L eta / (1 - L eta), eta = mu + gamma_4 (sqrt 2 + mu)."""
    u = unit_roundoff
    gamma4 = 4 * u / (1 - 4 * u)
    eta = twiddle_error + gamma4 * (np.sqrt(2.0) + twiddle_error)
    L = int(stages)
    return L * eta / (1 - L * eta)
