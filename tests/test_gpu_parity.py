"""HIP path vs the CPU oracle, byte for byte, through the C ABI.

Sizes span single tiles, several tiles and every code path (wave shuffle,
tiles at every compiled width, both work orders, 16-byte and per-element
global access); every comparison is exact.
"""
import numpy as np
import pytest

import oracle
import paper_1708_01873_amd as br
from gpu_util import assert_bytes_equal, to_device, to_host_bytes
from paper_1708_01873_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ELEM_SIZES = (1, 2, 4, 8, 16)
MAX_B = {1: 7, 2: 7, 4: 7, 8: 6, 16: 6}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    br.lib()


def _run(host: np.ndarray, k: int, s: int, inplace: bool, pad_front: int = 0, **cfg):
    """Run the library on `host` bytes and return the result bytes."""
    x = to_device(host, s, pad_front)
    if inplace:
        br.bitrev_inplace(x, k, **cfg)
        return to_host_bytes(x)
    y = to_device(np.zeros_like(host), s, pad_front)
    br.bitrev_outofplace(x, y, k, **cfg)
    out = to_host_bytes(y)
    assert_bytes_equal(to_host_bytes(x), host, "out-of-place modified its source")
    return out


def test_c1_uint32_n1024():
    """uint32, n = 2^10, seeded uniform values and the identity array."""
    for seed in (workloads.SEEDS["c1"],) + workloads.EXTRA_PARITY_SEEDS:
        host = workloads.uint32_uniform(10, seed)
        want = oracle.outofplace(host)
        for inplace in (True, False):
            assert_bytes_equal(_run(host, 10, 4, inplace), want, "c1 seed %d" % seed)
    io = workloads.iota(10)
    want = oracle.outofplace(io)
    got = _run(io, 10, 4, True).view(np.uint32)
    assert_bytes_equal(got, want, "iota")
    assert all(int(got[j]) == oracle.rev(j, 10) for j in range(1024))


@pytest.mark.parametrize("s", ELEM_SIZES)
def test_default_plan_every_k(s):
    """Every k from 0 to 20 with the library's own plan (wave path for k <= 6,
    tiles above), in place and out of place."""
    for k in range(0, 21):
        host = workloads.byte_pattern((1 << k) * s, seed=100 * s + k)
        want = oracle.outofplace(host, s)
        for inplace in (True, False):
            assert_bytes_equal(_run(host, k, s, inplace), want, "s=%d k=%d ip=%s" % (s, k, inplace))


@pytest.mark.parametrize("s", ELEM_SIZES)
def test_forced_tile_widths(s):
    """Every compiled tile width b, at k = 2b (one tile), 2b + 1 (palindromic
    pairs only), 2b + 3 and 2b + 6 (many pairs), every work order and kernel
    variant."""
    for b in range(1, MAX_B[s] + 1):
        for extra in (0, 1, 3, 6):
            k = 2 * b + extra
            if (1 << k) * s > (64 << 20):
                continue
            host = workloads.byte_pattern((1 << k) * s, seed=7 * k + b)
            want = oracle.outofplace(host, s)
            for order in (1, 2, 3):
                for variant in (1, 2, 3):
                    for inplace in (True, False):
                        got = _run(host, k, s, inplace, tile_bits=b, order=order,
                                   variant=variant)
                        assert_bytes_equal(got, want, "s=%d b=%d k=%d order=%d variant=%d ip=%s"
                                           % (s, b, k, order, variant, inplace))


@pytest.mark.parametrize("s", (1, 2, 4, 8))
def test_element_aligned_base(s):
    """A base pointer that is only elem_size aligned takes the per-element
    access path and still matches."""
    for k in (7, 10, 13, 16):
        host = workloads.byte_pattern((1 << k) * s, seed=k)
        want = oracle.outofplace(host, s)
        for inplace in (True, False):
            got = _run(host, k, s, inplace, pad_front=1)
            assert_bytes_equal(got, want, "misaligned s=%d k=%d ip=%s" % (s, k, inplace))


@pytest.mark.parametrize("s", (1, 2, 4))
def test_element_aligned_wide_tiles(s):
    """Element-aligned bases at the widest tile, where the per-element path
    moves elements between HBM and LDS one at a time (no register staging):
    palindromic and swapped tiles, odd and even middle widths."""
    for k in (14, 15, 17):
        host = workloads.byte_pattern((1 << k) * s, seed=100 + k)
        want = oracle.outofplace(host, s)
        for variant in (1, 2):
            for inplace in (True, False):
                got = _run(host, k, s, inplace, pad_front=1, tile_bits=7, variant=variant)
                assert_bytes_equal(got, want, "misaligned b=7 s=%d k=%d variant=%d ip=%s"
                                   % (s, k, variant, inplace))


@pytest.mark.parametrize("s", ELEM_SIZES)
def test_cache_hints(s):
    """Every cache-hint instance of the one-item tile kernels and of the
    register-staged in-place kernel (plain, streaming loads, streaming
    stores, streaming loads with write-through stores), every order, in and out of place, 16-byte and per-element
    access, against the oracle."""
    for k in (13, 16):
        host = workloads.byte_pattern((1 << k) * s, seed=31 * s + k)
        want = oracle.outofplace(host, s)
        for hints in (br.HINTS_PLAIN, br.HINTS_STREAM_LOADS, br.HINTS_STREAM_STORES,
                      br.HINTS_STREAM_WRITE_THROUGH):
            for inplace, variant in ((True, 1), (True, 3), (False, 1)):
                for order in (1, 2, 3):
                    for pad in (0, 1):
                        if pad and s >= 16:
                            continue
                        got = _run(host, k, s, inplace, pad_front=pad, variant=variant,
                                   order=order, cache_hints=hints)
                        assert_bytes_equal(got, want, "s=%d k=%d hints=%d ip=%s v=%d order=%d "
                                           "pad=%d" % (s, k, hints, inplace, variant, order, pad))


def test_timed_entry():
    """bitrev_inplace_timed permutes like bitrev_inplace, and the events its
    kernel records bracket a positive time within the step's own events."""
    for k, s in ((20, 8), (24, 8), (5, 4), (1, 8)):
        host = workloads.byte_pattern((1 << k) * s, seed=k + 100)
        x = to_device(host, s)
        ka, kb, a, b = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        ka.record()
        kb.record()
        a.record()
        br.bitrev_inplace_timed(x, ka, kb, k)
        b.record()
        torch.cuda.synchronize()
        assert_bytes_equal(to_host_bytes(x), oracle.outofplace(host, s), "timed k=%d" % k)
        kernel_ms, step_ms = ka.elapsed_time(kb), a.elapsed_time(b)
        assert 0.0 <= kernel_ms <= step_ms + 1e-3, (k, kernel_ms, step_ms)
    with pytest.raises(ValueError):
        br.bitrev_inplace_timed(x, torch.cuda.Event(enable_timing=True), kb, 1)


def test_timing_events():
    """The library's fence-free timing events with both timed entries: the
    results match the oracle, and the kernel's time is positive and within
    the step's own events."""
    for k, s in ((24, 8), (16, 4), (3, 16)):
        host = workloads.byte_pattern((1 << k) * s, seed=k + 200)
        want = oracle.outofplace(host, s)
        ka, kb = br.TimingEvent(), br.TimingEvent()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        x = to_device(host, s)
        a.record()
        br.bitrev_inplace_timed(x, ka, kb, k)
        b.record()
        torch.cuda.synchronize()
        assert_bytes_equal(to_host_bytes(x), want, "timed events ip k=%d" % k)
        kernel_ms, step_ms = ka.elapsed_time(kb), a.elapsed_time(b)
        assert 0.0 <= kernel_ms <= step_ms + 1e-3, (k, kernel_ms, step_ms)
        if k == 24:
            assert kernel_ms > 0.0
        x = to_device(host, s)
        y = to_device(np.zeros_like(host), s)
        br.bitrev_outofplace_timed(x, y, ka, kb, k)
        assert ka.elapsed_time(kb) >= 0.0
        assert_bytes_equal(to_host_bytes(y), want, "timed events oop k=%d" % k)
        ka.destroy()
        kb.destroy()
        ka.destroy()  # a second destroy is a no-op


@pytest.mark.parametrize("s", (1, 2, 4))
def test_write_through_narrow_rows(s):
    """Write-through stores on tile rows narrower than 16 bytes: the 8-, 4-,
    2- and 1-byte store forms of that cache hint, in and out of place, for
    every narrow tile width, one item per workgroup and register-staged
    (8-byte elements have no row narrower than 16 bytes)."""
    k = 12
    host = workloads.byte_pattern((1 << k) * s, seed=90 + s)
    want = oracle.outofplace(host, s)
    for b in range(1, 6):
        if (s << b) >= 16:
            break
        for inplace, variant in ((True, 1), (True, 3), (False, 1)):
            got = _run(host, k, s, inplace, tile_bits=b, variant=variant,
                       cache_hints=br.HINTS_STREAM_WRITE_THROUGH)
            assert_bytes_equal(got, want, "s=%d b=%d ip=%s v=%d" % (s, b, inplace, variant))


def test_copy_hints():
    """The reference copy with each cache hint copies every byte."""
    for nbytes in (1 << 20, (1 << 20) + 7):
        host = workloads.byte_pattern(nbytes, seed=nbytes)
        x = torch.from_numpy(host).cuda()
        for hints in (0, 1, 2, 3, 4):
            y = torch.zeros_like(x)
            br.bitrev_copy(x, y, cache_hints=hints)
            assert_bytes_equal(y.cpu().numpy(), host, "copy hints=%d n=%d" % (hints, nbytes))


@pytest.mark.parametrize("grid", [8, 24, 64])
def test_persistent_grid(grid):
    """A small explicit grid makes every workgroup loop over many items."""
    k, s = 18, 8
    host = workloads.byte_pattern((1 << k) * s, seed=grid)
    want = oracle.outofplace(host, s)
    for inplace in (True, False):
        for order in (1, 2):
            for variant in (1, 2, 3):
                got = _run(host, k, s, inplace, grid_blocks=grid, order=order, variant=variant)
                assert_bytes_equal(got, want, "grid=%d ip=%s order=%d variant=%d"
                                   % (grid, inplace, order, variant))


@pytest.mark.parametrize("s", (4, 8, 16))
def test_pipelined_rows(s):
    """The persistent pipelined kernels walk items across row boundaries."""
    for k, rows in ((12, 33), (14, 5)):
        host = workloads.byte_pattern((rows << k) * s, seed=k + rows + s)
        want = oracle.rows(host, k, s)
        x = to_device(host, s)
        y = torch.empty_like(x)
        br.bitrev_rows(x, y, k, variant=2)
        assert_bytes_equal(to_host_bytes(y), want, "rows oop pipelined s=%d k=%d" % (s, k))
        br.bitrev_rows(x, x, k, variant=2, grid_blocks=16)
        assert_bytes_equal(to_host_bytes(x), want, "rows ip pipelined s=%d k=%d" % (s, k))


def test_guard_regions_untouched():
    """Bytes before and after the array are never written."""
    for s, k in ((4, 10), (8, 15), (16, 12), (1, 17), (8, 4)):
        n = 1 << k
        guard = 4096 // s
        full = workloads.byte_pattern((n + 2 * guard) * s, seed=k)
        t = to_device(full, s)
        br.bitrev_inplace(t[guard:guard + n], k)
        out = torch.empty_like(t[guard:guard + n])
        br.bitrev_outofplace(t[guard:guard + n], out, k)
        got = to_host_bytes(t)
        inner = full[guard * s:(guard + n) * s]
        assert_bytes_equal(got[:guard * s], full[:guard * s], "front guard")
        assert_bytes_equal(got[(guard + n) * s:], full[(guard + n) * s:], "back guard")
        assert_bytes_equal(got[guard * s:(guard + n) * s], oracle.outofplace(inner, s), "inner")
        # out-of-place of the permuted array is the original again
        assert_bytes_equal(to_host_bytes(out), inner, "involution")


@pytest.mark.parametrize("s", (4, 8, 16))
def test_involution_on_device(s):
    """Applying the in-place permutation twice restores the input (every tile
    pair swapped exactly once per call)."""
    for k in (8, 11, 14, 17, 20):
        host = workloads.byte_pattern((1 << k) * s, seed=k + s)
        x = to_device(host, s)
        ref = x.clone()
        br.bitrev_inplace(x, k)
        br.bitrev_inplace(x, k)
        torch.cuda.synchronize()
        assert torch.equal(x.view(torch.uint8), ref.view(torch.uint8)), (s, k)


@pytest.mark.parametrize("s", ELEM_SIZES)
def test_rows(s):
    """Independent rows, in place and out of place, against the oracle row by
    row; covers the wave path with many arrays."""
    for k, rows in ((0, 5), (3, 7), (6, 130), (9, 3), (12, 17), (16, 2)):
        host = workloads.byte_pattern((rows << k) * s, seed=k * 31 + rows)
        want = oracle.rows(host, k, s)
        x = to_device(host, s)
        y = torch.empty_like(x)
        br.bitrev_rows(x, y, k)
        assert_bytes_equal(to_host_bytes(y), want, "rows oop s=%d k=%d" % (s, k))
        br.bitrev_rows(x, x, k)
        assert_bytes_equal(to_host_bytes(x), want, "rows ip s=%d k=%d" % (s, k))


def test_special_float_bits():
    """NaN payloads, signed zeros and denormals move as bits."""
    vals = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.5, 5e-324, 1e308] * 128,
                    dtype=np.float64)
    bits = vals.view(np.uint64).copy()
    bits[4::8] = 0x7FF8DEADBEEF0001
    bits[5::8] = 0xFFF0000000000001
    want = oracle.outofplace(bits)
    for inplace in (True, False):
        assert_bytes_equal(_run(bits.view(np.uint8), 10, 8, inplace), want, "float bits")
