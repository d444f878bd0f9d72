"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
when the oracle disagrees with the fact it names.  ``test_oracle_pins.py``
runs them on the real oracle; ``test_oracle_mutants.py`` runs them on copies
of the oracle with a plausible mistake planted, and requires that each
mistake is caught by at least one pin.

Sources (arXiv:1708.01873):
  * worked example n = 8 (Introduction);
  * involution rev(rev(i)) = i (Introduction);
  * bytewise reversal with a 256-entry table (Introduction) -- brute force on
    every index for every k <= 12;
  * inductive XOR generation of reversed indices (Methods);
  * the even-odd (Stockham) chain (Introduction);
  * the buffered method's split rev(x y z) = rev(z) rev(y) rev(x)
    (Introduction, matrix buffer);
  * the recursive method: two rounds of half-size reversals around a square
    transpose, and the even-odd pre-step for odd k (Methods);
  * the swap-count recurrence and closed form (Methods, unrolling).
"""
from __future__ import annotations

import math

import numpy as np

from indep_rev import (bitrev_evenodd_chain, evenodd_step, read_golden, rev_bytetable,
                       rev_bytetable_array, rev_sequence_xor)


def pin_worked_example(o) -> None:
    g = read_golden("worked_example_n8.txt")
    inp = np.array([int(t) for t in g["input"].split()], dtype=np.uint32)
    want = np.array([int(t) for t in g["output"].split()], dtype=np.uint32)
    want_bin = [int(t, 2) for t in g["output_binary"].split()]
    assert list(want) == want_bin
    got_oop = o.outofplace(inp)
    assert np.array_equal(got_oop, want), got_oop
    got_ip = inp.copy()
    o.inplace(got_ip)
    assert np.array_equal(got_ip, want), got_ip
    assert [o.rev(i, 3) for i in range(8)] == list(want)


def pin_bytetable_bruteforce(o, kmax: int = 12) -> None:
    """Every index of every size n <= 2^kmax against the byte-table reversal."""
    for k in range(0, kmax + 1):
        n = 1 << k
        want = np.array([rev_bytetable(i, k) for i in range(n)], dtype=np.int64)
        # the permutation of the identity array reads rev off directly
        iota = np.arange(n, dtype=np.int64)
        assert np.array_equal(o.outofplace(iota), want), k
        ip = iota.copy()
        o.inplace(ip)
        assert np.array_equal(ip, want), k
        # the scalar reversal too, on every index
        assert all(o.rev(i, k) == want[i] for i in range(n)), k


def pin_involution(o, kmax: int = 20) -> None:
    rng = np.random.default_rng(11)
    for k in range(0, kmax + 1):
        a = rng.integers(0, 2**32, size=1 << k, dtype=np.uint32)
        b = a.copy()
        o.inplace(b)
        o.inplace(b)
        assert np.array_equal(a, b), k
        assert np.array_equal(o.outofplace(o.outofplace(a)), a), k


def pin_xor_induction(o, kmax: int = 16) -> None:
    for k in range(0, kmax + 1):
        want = np.array(rev_sequence_xor(k), dtype=np.int64)
        assert np.array_equal(o.rev_table(k), want), k


def pin_evenodd_chain(o, kmax: int = 12) -> None:
    g = read_golden("evenodd_n8.txt")
    assert evenodd_step(list(range(8))) == [int(t) for t in g["output"].split()]
    rng = np.random.default_rng(12)
    for k in range(0, kmax + 1):
        a = rng.integers(0, 2**62, size=1 << k, dtype=np.int64)
        assert np.array_equal(o.outofplace(a), np.array(bitrev_evenodd_chain(list(a)))), k


def pin_buffer_split(o) -> None:
    """rev(x y z) = rev(z) rev(y) rev(x) for bit strings of widths (b, m, b)."""
    rng = np.random.default_rng(13)
    for k in range(0, 40):
        for b in range(0, k // 2 + 1):
            m = k - 2 * b
            for _ in range(8):
                x = int(rng.integers(0, 1 << b))
                y = int(rng.integers(0, 1 << m)) if m < 63 else 0
                z = int(rng.integers(0, 1 << b))
                i = (x << (m + b)) | (y << b) | z
                want = ((rev_bytetable(z, b) << (m + b)) | (rev_bytetable(y, m) << b)
                        | rev_bytetable(x, b))
                assert o.rev(i, k) == want, (k, b, x, y, z)


def pin_recursive_decomposition(o, kmax: int = 16) -> None:
    """Even k: reverse the low half within each row, transpose the square,
    reverse the low half again.  Odd k: even-odd split, then two (k-1)-bit
    reversals (Methods, cache-oblivious recursive permutation)."""
    rng = np.random.default_rng(14)
    for k in range(2, kmax + 1):
        a = rng.integers(0, 2**62, size=1 << k, dtype=np.int64)
        want = o.outofplace(a)
        if k % 2 == 0:
            h = k // 2
            step1 = o.rows(a, h)
            step2 = np.ascontiguousarray(step1.reshape(1 << h, 1 << h).T).reshape(-1)
            got = o.rows(step2, h)
        else:
            halves = np.ascontiguousarray(np.concatenate([a[0::2], a[1::2]]))
            got = o.rows(halves, k - 1)
        assert np.array_equal(got, want), k


def _swap_count_closed_form(k: int) -> float:
    """The paper's printed closed form for r(k) (Methods, unrolling)."""
    s2 = math.sqrt(2.0)
    return 2.0 ** (k / 2) * ((-1) ** k * (s2 - 1) / 4 - (1 + s2) / 4) + 2.0 ** (k - 1)


def pin_swap_counts(o, kmax: int = 20) -> None:
    g = read_golden("swap_counts.txt")
    r = {1: int(g["r_1"]), 2: int(g["r_2"])}
    for k in range(3, kmax + 1):
        r[k] = 2 ** (k - 2) + 2 * r[k - 2]
    for k in range(1, kmax + 1):
        assert abs(_swap_count_closed_form(k) - r[k]) < 1e-6 * max(1, r[k]), k
        assert r[k] == 2 ** (k - 1) - 2 ** ((k + 1) // 2 - 1), k
        n = 1 << k
        iota = np.arange(n, dtype=np.int64)
        perm = o.outofplace(iota)
        moved = int(np.count_nonzero(perm != iota))
        # each swap moves two elements; fixed points (palindromes) stay put
        assert moved == 2 * r[k], (k, moved, r[k])
        assert n - moved == 2 ** ((k + 1) // 2), k
        # a permutation: every index appears once
        assert np.array_equal(np.sort(perm), iota), k
        # the first and last index are fixed (Introduction listing's bounds)
        assert perm[0] == 0 and perm[-1] == n - 1, k


def pin_element_sizes(o) -> None:
    """Elements are opaque byte blocks of any size: compare with fancy indexing
    by the byte-table permutation."""
    rng = np.random.default_rng(15)
    for s in (1, 2, 3, 4, 5, 8, 12, 16, 32):
        for k in (0, 1, 2, 3, 5, 8, 11):
            n = 1 << k
            buf = rng.integers(0, 256, size=n * s, dtype=np.uint8)
            perm = np.array([rev_bytetable(j, k) for j in range(n)], dtype=np.int64)
            want = buf.reshape(n, s)[perm].reshape(-1)
            assert np.array_equal(o.outofplace(buf, s), want), (s, k)
            ip = buf.copy()
            o.inplace(ip, s)
            assert np.array_equal(ip, want), (s, k)


def pin_outofplace_threads(o) -> None:
    """The multi-threaded out-of-place form (CPU-baseline timing and the
    full-size comparisons) gives
    the byte-table permutation, for sizes that split unevenly over threads."""
    rng = np.random.default_rng(16)
    for s in (1, 3, 8, 16):
        for k in (0, 1, 2, 5, 9, 13):
            n = 1 << k
            buf = rng.integers(0, 256, size=n * s, dtype=np.uint8)
            perm = np.array([rev_bytetable(j, k) for j in range(n)], dtype=np.int64)
            want = np.empty_like(buf).reshape(n, s)
            want[perm] = buf.reshape(n, s)
            got, threads = o.outofplace_mt(buf, s)
            assert threads >= 1
            assert np.array_equal(got, want.reshape(-1)), (s, k)


def pin_outofplace_threads_large(o) -> None:
    """The multi-threaded out-of-place form, which the full-size comparisons
    of the multi-GiB configurations use, gives the byte-table permutation on
    every index of arrays of millions of elements (each thread's static share
    then spans many cache lines and pages), for 1-, 4- and 16-byte elements."""
    rng = np.random.default_rng(17)
    for k, s in ((22, 1), (21, 4), (20, 16)):
        n = 1 << k
        buf = rng.integers(0, 256, size=n * s, dtype=np.uint8)
        perm = rev_bytetable_array(np.arange(n, dtype=np.uint64), k).astype(np.int64)
        want = np.empty_like(buf).reshape(n, s)
        want[perm] = buf.reshape(n, s)
        got, threads = o.outofplace_mt(buf, s)
        assert threads >= 1
        assert np.array_equal(got, want.reshape(-1)), (s, k)


def pin_special_values(o) -> None:
    """NaN payloads, signed zeros and infinities move as bits."""
    vals = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.5, 5e-324, 1e308], dtype=np.float64)
    bits = vals.view(np.uint64).copy()
    bits[4] = 0x7FF8DEADBEEF0001  # quiet NaN with a payload
    bits[5] = 0xFFF0000000000001  # signalling NaN, sign set
    a = bits.view(np.float64)
    got = o.outofplace(a).view(np.uint64)
    perm = [rev_bytetable(j, 3) for j in range(8)]
    assert np.array_equal(got, bits[perm])
    ip = a.copy()
    o.inplace(ip)
    assert np.array_equal(ip.view(np.uint64), bits[perm])


def pin_rows_and_batched(o) -> None:
    """Several arrays at once equal the arrays done one by one, each against
    the byte-table permutation."""
    rng = np.random.default_rng(16)
    k, nrows, s = 6, 5, 8
    a = rng.integers(0, 2**63, size=nrows << k, dtype=np.int64)
    perm = np.array([rev_bytetable(j, k) for j in range(1 << k)])
    want = a.reshape(nrows, 1 << k)[:, perm].reshape(-1)
    assert np.array_equal(o.rows(a, k, s), want)
    ip = a.copy()
    o.rows(ip, k, s, inplace=True)
    assert np.array_equal(ip, want)

    log2n = np.array([0, 3, 1, 7, 2, 5, 0, 9], dtype=np.int32)
    offsets = np.concatenate([[0], np.cumsum(1 << log2n.astype(np.int64))]).astype(np.int64)
    data = rng.integers(0, 2**63, size=int(offsets[-1]), dtype=np.int64)
    want = data.copy()
    for a_, k_ in enumerate(log2n):
        seg = want[offsets[a_]:offsets[a_ + 1]]
        p = np.array([rev_bytetable(j, int(k_)) for j in range(1 << int(k_))])
        want[offsets[a_]:offsets[a_ + 1]] = seg[p]
    got = data.copy()
    o.batched(got, offsets, log2n)
    assert np.array_equal(got, want)
    # a length that is not 2^log2n is rejected
    bad = offsets.copy()
    bad[-1] -= 1
    try:
        o.batched(data.copy(), bad, log2n)
    except ValueError:
        pass
    else:
        raise AssertionError("oracle accepted an array whose length is not 2^log2n")


ALL_PINS = [
    pin_worked_example,
    pin_bytetable_bruteforce,
    pin_involution,
    pin_xor_induction,
    pin_evenodd_chain,
    pin_buffer_split,
    pin_recursive_decomposition,
    pin_swap_counts,
    pin_element_sizes,
    pin_special_values,
    pin_rows_and_batched,
]


def _digits(i: int, k: int, d: int) -> list:
    """Base-2^d digits of i, least significant first, by integer division."""
    q = 1 << d
    return [(i // q ** t) % q for t in range(k // d)]


def pin_digit_reversal(o) -> None:
    """Digit reversal for radix-2^d FFTs: d = 1 is the bit reversal; the
    digit list reversed (by divmod, independent of shifts); an involution;
    fixed points q^ceil(D/2); base 4 on n = 16 by hand."""
    # base 4, n = 16 (two digits): index 1 = (0,1) -> (1,0) = 4, 6 = (1,2) -> (2,1) = 9
    want16 = [0, 4, 8, 12, 1, 5, 9, 13, 2, 6, 10, 14, 3, 7, 11, 15]
    assert [o.digit_rev(i, 4, 2) for i in range(16)] == want16
    for d in (1, 2, 3):
        for k in range(0, 13, d):
            if k % d:
                continue
            n, q, D = 1 << k, 1 << d, k // d
            want = []
            for i in range(n):
                dg = _digits(i, k, d)[::-1]
                want.append(sum(v * q ** t for t, v in enumerate(dg)))
            got = [o.digit_rev(i, k, d) for i in range(n)]
            assert got == want, (d, k)
            if d == 1:
                assert got == [rev_bytetable(i, k) for i in range(n)]
            assert all(got[got[i]] == i for i in range(n))
            assert sum(1 for i in range(n) if got[i] == i) == q ** ((D + 1) // 2)
            a = np.arange(n, dtype=np.int64)
            assert np.array_equal(o.digit_outofplace(a, d), np.array(want).argsort()), (d, k)
            b = a.copy()
            o.digit_inplace(b, d)
            assert np.array_equal(b, np.array(want)), (d, k)
    try:
        o.digit_outofplace(np.arange(8, dtype=np.int64), 2)  # k = 3 is not a multiple of 2
    except ValueError:
        pass
    else:
        raise AssertionError("digit reversal accepted k not a multiple of d")


ALL_PINS.append(pin_digit_reversal)
ALL_PINS.append(pin_outofplace_threads)
ALL_PINS.append(pin_outofplace_threads_large)


def pin_evenodd_split(o) -> None:
    """The even-odd split against the paper's 4 x 2 example and the
    independent slicing form; applying it k times in nested halves is the
    bit reversal (Introduction)."""
    g = read_golden("evenodd_n8.txt")
    a = np.arange(8, dtype=np.int64)
    assert list(o.evenodd(a)) == [int(t) for t in g["output"].split()]
    rng = np.random.default_rng(17)
    for s in (1, 4, 8, 16):
        for k in range(1, 12):
            buf = rng.integers(0, 256, size=(1 << k) * s, dtype=np.uint8)
            el = buf.reshape(-1, s)
            want = np.concatenate([el[0::2], el[1::2]]).reshape(-1)
            assert np.array_equal(o.evenodd(buf, s), want), (s, k)
    for k in range(1, 11):
        a = rng.integers(0, 2**62, size=1 << k, dtype=np.int64)
        y = a.copy()
        for level in range(k):
            blocks = y.reshape(1 << level, -1)
            y = np.concatenate([o.evenodd(np.ascontiguousarray(b)) for b in blocks])
        assert np.array_equal(y, o.outofplace(a)), k


ALL_PINS.append(pin_evenodd_split)
