"""Bit reversal fused with the first L radix-2 DIT levels vs the oracle's
closed form.  The tolerance is Higham's norm-wise bound for an L-level
radix-2 FFT in the element's precision (twiddles rounded once), applied to
every block of 2^L outputs."""
import numpy as np
import pytest

import paper_1708_01873_amd as br
from gpu_util import to_host_bytes
from oracle import dit
from paper_1708_01873_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = {np.complex64: 2.0 ** -24, np.complex128: 2.0 ** -53}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    br.lib()


def _check(got, x, L, inverse, dtype):
    # a complex128 result is checked against an extended-precision reference,
    # so that the reference's own rounding is far below the bound
    prec = np.clongdouble if dtype == np.complex128 else np.complex128
    want = dit.dit_stages(x, L, inverse, precision=prec)
    q = 1 << L
    g = got.astype(prec).reshape(-1, q)
    w = want.reshape(-1, q)
    err = np.linalg.norm(g - w, axis=1)
    ref = np.linalg.norm(w, axis=1)
    bound = dit.higham_bound(L, U[dtype], U[dtype])
    # the inputs are exact in the element type, so the bound applies as is
    assert np.all(err <= bound * ref + 1e-30), (float((err / np.maximum(ref, 1e-300)).max()), bound)


def _data(k, rows, dtype, seed):
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(rows << k)
    im = rng.standard_normal(rows << k)
    return (re + 1j * im).astype(dtype)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_dit_stages_sweep(dtype):
    for k in (2, 5, 8, 11, 14, 17):
        for L in range(0, min(k // 2, 6) + 1):
            x = _data(k, 1, dtype, 10 * k + L)
            for inverse in (False, True):
                t = torch.from_numpy(x).cuda()
                y = br.bitrev_dit_stages(t, stages=L, inverse=inverse)
                _check(to_host_bytes(y).view(dtype), x, L, inverse, dtype)
                br.bitrev_dit_stages(t, t, stages=L, inverse=inverse)  # in place
                _check(to_host_bytes(t).view(dtype), x, L, inverse, dtype)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_dit_forced_tile_widths(dtype):
    """Every tile width that holds the levels, in and out of place, through
    the configured entry point."""
    k = 14
    for L in range(1, 7):
        for b in range(L, 7 if k >= 12 else k // 2 + 1):
            x = _data(k, 1, dtype, 100 * L + b)
            t = torch.from_numpy(x).cuda()
            y = br.bitrev_dit_stages(t, stages=L, tile_bits=b)
            _check(to_host_bytes(y).view(dtype), x, L, False, dtype)
            br.bitrev_dit_stages(t, t, stages=L, tile_bits=b, order=br.ORDER_BALANCED)
            _check(to_host_bytes(t).view(dtype), x, L, False, dtype)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_dit_cache_hints(dtype):
    """Every cache-hint instance of the fused kernel, in and out of place."""
    k = 16
    for hints in (br.HINTS_PLAIN, br.HINTS_STREAM_LOADS, br.HINTS_STREAM_STORES,
                  br.HINTS_STREAM_WRITE_THROUGH):
        for L in (1, 4):
            x = _data(k, 1, dtype, 1000 + 10 * hints + L)
            t = torch.from_numpy(x).cuda()
            y = br.bitrev_dit_stages(t, stages=L, cache_hints=hints)
            _check(to_host_bytes(y).view(dtype), x, L, False, dtype)
            br.bitrev_dit_stages(t, t, stages=L, cache_hints=hints)
            _check(to_host_bytes(t).view(dtype), x, L, False, dtype)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("b,variant", [(5, 2), (5, 3), (6, 2), (6, 3)])
def test_dit_rectangular_tiles(dtype, b, variant):
    """Out of place with rectangular tiles (2^b source rows of 2^(b-1) or
    2^(b-2) elements): every level count up to b, odd and even array
    sizes, several rows, every cache hint, both directions."""
    for k, rows in ((2 * b - variant + 1, 1), (13, 3), (16, 1), (19, 2)):
        for L in range(0, min(b, k // 2) + 1):   # 2 L <= log2 n, as for square tiles
            x = _data(k, rows, dtype, 7000 + 100 * k + 10 * L + variant)
            t = torch.from_numpy(x).cuda().view(rows, 1 << k)
            inverse = (L + k) % 2 == 1
            hints = 1 + (L + k + variant) % 4
            y = br.bitrev_dit_stages(t, stages=L, inverse=inverse, tile_bits=b, variant=variant,
                                     cache_hints=hints)
            got = to_host_bytes(y).view(dtype).reshape(rows, -1)
            for r in range(rows):
                _check(got[r], x.reshape(rows, -1)[r], L, inverse, dtype)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("b", [4, 5, 6])
def test_dit_inplace_register_staged(b, dtype):
    """In place with the tile pair held in registers and its tiles staged
    through one LDS tile in turn: every level count up to b (the first
    levels in registers from the level count that the thread's rows hold),
    palindromic and paired tiles, several rows, every cache hint, both
    directions."""
    for k, rows in ((2 * b, 1), (2 * b + 1, 2), (15, 3), (18, 1)):
        for L in range(1, b + 1):
            x = _data(k, rows, dtype, 9000 + 100 * k + 10 * L + b)
            t = torch.from_numpy(x).cuda().view(rows, 1 << k)
            inverse = (L + k) % 2 == 0
            hints = 1 + (L + k + b) % 4
            br.bitrev_dit_stages(t, t, stages=L, inverse=inverse, tile_bits=b, variant=3,
                                 cache_hints=hints)
            got = to_host_bytes(t).view(dtype).reshape(rows, -1)
            for r in range(rows):
                _check(got[r], x.reshape(rows, -1)[r], L, inverse, dtype)


@pytest.mark.parametrize("b", [4, 5, 6])
def test_dit_element_aligned(b):
    """Complex64 arrays 8 bytes off the 16-byte grid take the element-wise
    tile accesses (and, in the register-staged kernel, eight one-element
    chunks per thread: three levels in registers): square tiles in and out
    of place and register-staged in place, every level count up to b, both
    directions."""
    dtype = np.complex64
    k, rows = 2 * b + 3, 2
    n = rows << k
    for L in range(1, b + 1):
        x = _data(k, rows, dtype, 4000 + 10 * b + L)
        inverse = L % 2 == 1
        src = torch.zeros(n + 1, dtype=torch.complex64, device="cuda")
        dst = torch.zeros(n + 1, dtype=torch.complex64, device="cuda")
        src[1:] = torch.from_numpy(x).cuda()
        s1, d1 = src[1:].view(rows, 1 << k), dst[1:].view(rows, 1 << k)
        br.bitrev_dit_stages(s1, d1, stages=L, inverse=inverse, tile_bits=b, variant=1)
        got = to_host_bytes(d1).view(dtype).reshape(rows, -1)
        for r in range(rows):
            _check(got[r], x.reshape(rows, -1)[r], L, inverse, dtype)
        for variant in (1, 3):
            src[1:] = torch.from_numpy(x).cuda()
            br.bitrev_dit_stages(s1, s1, stages=L, inverse=inverse, tile_bits=b, variant=variant)
            got = to_host_bytes(s1).view(dtype).reshape(rows, -1)
            for r in range(rows):
                _check(got[r], x.reshape(rows, -1)[r], L, inverse, dtype)


def test_dit_inplace_register_staged_full_size():
    x = workloads.complex64_normal(24, workloads.SEEDS["c2"])
    t = torch.from_numpy(x).cuda()
    br.bitrev_dit_stages(t, t, stages=6, tile_bits=6, variant=3)
    _check(to_host_bytes(t).view(np.complex64), x, 6, False, np.complex64)


def test_dit_inplace_register_staged_complex128_large():
    """Complex double, 2^22 elements (64 MiB, 2^10 tile pairs) at six levels
    in place, register-staged, inverse."""
    x = _data(22, 1, np.complex128, 77)
    t = torch.from_numpy(x).cuda()
    br.bitrev_dit_stages(t, t, stages=6, tile_bits=6, variant=3, inverse=True)
    _check(to_host_bytes(t).view(np.complex128), x, 6, True, np.complex128)


def test_dit_rectangular_tiles_full_size():
    """The complex64 2^24 array at six fused levels on 2^6 x 2^4 tiles."""
    x = workloads.complex64_normal(24, workloads.SEEDS["c2"])
    t = torch.from_numpy(x).cuda()
    y = br.bitrev_dit_stages(t, stages=6, tile_bits=6, variant=3)
    _check(to_host_bytes(y).view(np.complex64), x, 6, False, np.complex64)


def test_dit_rectangular_tiles_rejected_where_they_do_not_apply():
    t = torch.zeros(1 << 16, dtype=torch.complex64, device="cuda")
    for kw in (dict(tile_bits=6, variant=2),):
        with pytest.raises(br.BitrevError) as e:      # in place
            br.bitrev_dit_stages(t, t, stages=4, **kw)
        assert e.value.status == br.ERROR_NOT_SUPPORTED
    t2 = torch.zeros(1 << 10, dtype=torch.complex128, device="cuda")
    with pytest.raises(br.BitrevError) as e:          # register-staged: square tiles, 2b <= k
        br.bitrev_dit_stages(t2, t2, stages=4, tile_bits=6, variant=3)
    assert e.value.status == br.ERROR_NOT_SUPPORTED
    with pytest.raises(br.BitrevError) as e:          # b = 4
        br.bitrev_dit_stages(t, stages=4, tile_bits=4, variant=2)
    assert e.value.status == br.ERROR_NOT_SUPPORTED
    base = torch.zeros((1 << 16) + 1, dtype=torch.complex64, device="cuda")
    with pytest.raises(br.BitrevError) as e:          # 8-byte aligned only
        br.bitrev_dit_stages(base[1:], stages=4, tile_bits=5, variant=2)
    assert e.value.status == br.ERROR_NOT_SUPPORTED


def test_dit_rows_and_full_size():
    """Many rows, and the complex64 2^24 array at six fused levels."""
    x = _data(12, 9, np.complex64, 3).reshape(9, 1 << 12)
    y = br.bitrev_dit_stages(torch.from_numpy(x).cuda(), stages=6)
    got = to_host_bytes(y).view(np.complex64).reshape(9, -1)
    for r in range(9):
        _check(got[r], x[r], 6, False, np.complex64)
    # 128 MiB: in place the plan streams the stores, out of place the loads
    x = workloads.complex64_normal(24, workloads.SEEDS["c2"])
    t = torch.from_numpy(x).cuda()
    y = br.bitrev_dit_stages(t, stages=6)
    _check(to_host_bytes(y).view(np.complex64), x, 6, False, np.complex64)
    br.bitrev_dit_stages(t, t, stages=6)
    _check(to_host_bytes(t).view(np.complex64), x, 6, False, np.complex64)
    # complex128, 128 MiB in place: streaming loads on the 16-byte kernel
    x = _data(23, 1, np.complex128, 5)
    t = torch.from_numpy(x).cuda()
    br.bitrev_dit_stages(t, t, stages=3, inverse=True)
    _check(to_host_bytes(t).view(np.complex128), x, 3, True, np.complex128)


def test_dit_rejects():
    t = torch.zeros(1 << 10, dtype=torch.complex64, device="cuda")
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_dit_stages(t, stages=6)  # 2 * 6 > 10
    assert e.value.status == br.ERROR_NOT_SUPPORTED
    with pytest.raises(TypeError):
        br.bitrev_dit_stages(torch.zeros(16, device="cuda"), stages=1)
