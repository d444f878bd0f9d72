"""Pins of the DIT-stages oracle (bit reversal + first L FFT levels)."""
import numpy as np
import pytest

import oracle
from oracle import dit
from indep_rev import rev_bytetable


def _rand(k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(1 << k) + 1j * rng.standard_normal(1 << k)


@pytest.mark.parametrize("k", range(0, 13))
def test_closed_form_equals_butterflies(k):
    x = _rand(k, k)
    for L in range(0, min(k, 8) + 1):
        for inv in (False, True):
            a = dit.dit_stages(x, L, inv)
            b = dit.dit_stages_iterative(x, L, inv)
            assert np.allclose(a, b, rtol=0, atol=1e-9 * max(1.0, np.abs(b).max())), (k, L, inv)


@pytest.mark.parametrize("k", range(0, 12))
def test_all_stages_is_numpy_fft(k):
    """With L = k the result is the full DFT (a library routine)."""
    x = _rand(k, 100 + k)
    assert np.allclose(dit.dit_stages(x, k), np.fft.fft(x), atol=1e-9 * 2**k)
    assert np.allclose(dit.dit_stages(x, k, inverse=True), np.fft.ifft(x) * 2**k, atol=1e-9 * 2**k)
    assert np.allclose(dit.dit_stages_iterative(x, k), np.fft.fft(x), atol=1e-9 * 2**k)


@pytest.mark.parametrize("k", range(0, 12))
def test_zero_stages_is_bit_reversal(k):
    x = _rand(k, 200 + k)
    perm = [rev_bytetable(j, k) for j in range(1 << k)]
    assert np.array_equal(dit.dit_stages(x, 0), x[perm])
    assert np.array_equal(dit.dit_stages_iterative(x, 0), x[perm])


def test_impulse_closed_form():
    """x = delta at p: block J is nonzero only if p = rev_{k-L}(J) + 2^(k-L) u,
    and then holds exp(-2 pi i u f / 2^L)."""
    k, L = 10, 4
    for p in (0, 1, 37, 1023, 512):
        x = np.zeros(1 << k, dtype=complex)
        x[p] = 1.0
        out = dit.dit_stages(x, L).reshape(-1, 1 << L)
        r, u = p % (1 << (k - L)), p >> (k - L)
        J = rev_bytetable(r, k - L)
        f = np.arange(1 << L)
        want = np.zeros_like(out)
        want[J] = np.exp(-2j * np.pi * u * f / (1 << L))
        assert np.allclose(out, want, atol=1e-12)


def test_higham_bound_values():
    u32 = 2.0 ** -24
    b = dit.higham_bound(6, u32, u32)
    assert 1e-6 < b < 3e-6
    assert dit.higham_bound(0, u32, u32) == 0.0


def test_extended_precision_reference_agrees():
    """The extended-precision form agrees with the complex128 one to complex128
    accuracy, and with numpy's FFT when L = k."""
    for k in (4, 9, 12):
        x = _rand(k, 300 + k)
        for L in (0, 3, min(k, 6)):
            a = dit.dit_stages(x, L, precision=np.clongdouble)
            b = dit.dit_stages(x, L)
            assert np.allclose(a.astype(np.complex128), b, atol=1e-12 * max(1.0, np.abs(b).max()))
        full = dit.dit_stages(x, k, precision=np.clongdouble).astype(np.complex128)
        assert np.allclose(full, np.fft.fft(x), atol=1e-9 * 2**k)
