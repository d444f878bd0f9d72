"""The benchmark configurations at full size, in the launch configuration the
benchmark times (the library's default plan, plus the tile-width sweep).

  uint32 n=2^10                     -> test_gpu_parity.test_c1_uint32_n1024
  complex64 n=2^24, b in {4,5,6}    -> test_c2_*  (full oracle compare, every plan timed)
  complex128 n=2^28, float32 2^30   -> test_c3_*  (full oracle compare, chunked)
  4096 uneven complex64 arrays      -> test_c4_*  (full oracle compare, chunked)
  256 x 2^16 float32, autograd      -> test_c5_*  (full + FD)
  more than 2^31 elements           -> test_more_than_2p32_* (full oracle compare)

The multi-GiB results are copied back a chunk at a time and compared byte for
byte with the oracle's result for the whole array, computed on the host: the
out-of-place definition with its index range split over the host threads
(the oracle's multi-threaded form), or the in-place definition applied to
each array of a batch from a pool of host threads.
"""
import concurrent.futures as cf
import math
import os

import numpy as np
import pytest

import oracle
import paper_1708_01873_amd as br
from gpu_util import assert_bytes_equal, assert_device_equal, to_host_bytes
from paper_1708_01873_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    br.lib()


def _free_gpu():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# complex64, n = 2^24 (128 MiB)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2():
    host = workloads.complex64_normal(24, workloads.SEEDS["c2"])
    return host, oracle.outofplace(host)


@pytest.fixture(scope="module")
def c2_dev(c2):
    return torch.from_numpy(c2[0]).cuda()


# every (tile width, order) plan the benchmark times at this size, with each
# tile kernel variant and both XCD mappings
@pytest.mark.parametrize("xcd", [1, 2])
@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("b", [4, 5, 6])
def test_c2_every_timed_plan(c2, c2_dev, b, order, variant, xcd):
    _, want = c2
    cfg = dict(tile_bits=b, order=order, variant=variant, xcd_remap=xcd)
    what = "c2 b=%d order=%d variant=%d xcd=%d" % (b, order, variant, xcd)
    x = c2_dev.clone()
    y = br.bitrev_outofplace(x, **cfg)
    assert_device_equal(y, want, what + " out of place")
    br.bitrev_inplace(x, **cfg)
    assert_device_equal(x, want, what + " in place")
    del x, y


@pytest.mark.parametrize("hints", [1, 2, 3, 4])
@pytest.mark.parametrize("b", [4, 5, 6])
def test_c2_cache_hints(c2, c2_dev, b, hints):
    _, want = c2
    x = c2_dev.clone()
    y = br.bitrev_outofplace(x, tile_bits=b, cache_hints=hints)
    assert_device_equal(y, want, "c2 b=%d hints=%d out of place" % (b, hints))
    br.bitrev_inplace(x, tile_bits=b, cache_hints=hints)
    assert_device_equal(x, want, "c2 b=%d hints=%d in place" % (b, hints))
    del x, y


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("b", [0, 4, 5, 6])
def test_c2_complex64_2p24(c2, b, variant):
    host, want = c2
    x = torch.from_numpy(host).cuda()
    y = br.bitrev_outofplace(x, tile_bits=b, variant=variant)
    assert_bytes_equal(to_host_bytes(y), want, "c2 out-of-place b=%d v=%d" % (b, variant))
    br.bitrev_inplace(x, tile_bits=b, variant=variant)
    assert_bytes_equal(to_host_bytes(x), want, "c2 in-place b=%d v=%d" % (b, variant))
    del x, y
    _free_gpu()


# --------------------------------------------------------------------------
# complex128 n = 2^28 and float32 n = 2^30 (4 GiB each)
# --------------------------------------------------------------------------
def _sampled_check(x, y, k, seed, count=1 << 16):
    """y[rev(i)] == x[i] bit for bit on `count` seeded indices, rev from the
    oracle."""
    idx = workloads.sample_coordinates(1 << k, count, seed)
    rev = np.array([oracle.rev(int(i), k) for i in idx], dtype=np.int64)
    xi = x[torch.from_numpy(idx).cuda()]
    yr = y[torch.from_numpy(rev).cuda()]
    assert_bytes_equal(to_host_bytes(yr), to_host_bytes(xi), "sampled k=%d" % k)


@pytest.mark.parametrize("k,dtype,seed", [
    (28, "complex128", workloads.SEEDS["c3a"]),
    (30, "float32", workloads.SEEDS["c3b"]),
])
def test_c3_large(k, dtype, seed):
    """4 GiB arrays: out of place, in place, and in place again, each compared
    in full with the oracle (the input itself after the second application)."""
    tdt = getattr(torch, dtype)
    x = workloads.device_normal(1 << k, seed, tdt)
    s = x.element_size()
    host = to_host_bytes(x)
    y = br.bitrev_outofplace(x)
    _sampled_check(x, y, k, seed)       # quick first assertion
    want, _ = oracle.outofplace_mt(host, elem_size=s)
    assert_device_equal(y, want, "c3 k=%d out of place" % k)
    del y
    _free_gpu()
    br.bitrev_inplace(x)
    assert_device_equal(x, want, "c3 k=%d in place" % k)
    del want
    br.bitrev_inplace(x)
    assert_device_equal(x, host, "c3 k=%d in place twice" % k)
    del x
    _free_gpu()


# --------------------------------------------------------------------------
# 4096 complex64 arrays, log2 n uniform in [8, 20]
# --------------------------------------------------------------------------
def test_c4_batched_full():
    seed = workloads.SEEDS["c4"]
    offsets, log2n = workloads.batched_layout(4096, 8, 20, seed)
    total = int(offsets[-1])
    x = workloads.device_normal(total, seed + 1000, torch.complex64)
    keep = x.clone()
    off = torch.from_numpy(offsets).cuda()
    l2 = torch.from_numpy(log2n).cuda()
    ws = torch.empty(br.bitrev_batched_workspace_size(4096), dtype=torch.uint8, device="cuda")
    br.bitrev_batched(x, off, l2, ws)
    assert br.bitrev_batched_errors(ws) == (0, -1)
    # in full against the oracle: its in-place definition on every array of
    # a host copy of the input, the arrays spread over a pool of host threads
    # (each call works on its own array; the calls release the GIL)
    want = to_host_bytes(keep).view(np.complex64).copy()
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda a: oracle.inplace(want[offsets[a]:offsets[a + 1]]), range(4096)))
    assert_device_equal(x, want, "c4 batched, all 4096 arrays")
    del want
    # sampled against the oracle's rev: 64 positions per array
    rng = np.random.default_rng(seed)
    tables = {}
    src_idx, dst_idx = [], []
    for a in range(4096):
        k = int(log2n[a])
        if k not in tables:
            tables[k] = oracle.rev_table(k)
        j = rng.integers(0, 1 << k, size=64)
        src_idx.append(offsets[a] + j)
        dst_idx.append(offsets[a] + tables[k][j])
    src_idx = torch.from_numpy(np.concatenate(src_idx)).cuda()
    dst_idx = torch.from_numpy(np.concatenate(dst_idx)).cuda()
    assert_bytes_equal(to_host_bytes(x[dst_idx]), to_host_bytes(keep[src_idx]), "c4 sampled")
    # every array equals the per-array plain call's result
    y = keep.clone()
    for a in range(4096):
        br.bitrev_inplace(y[offsets[a]:offsets[a + 1]])
    torch.cuda.synchronize()
    assert torch.equal(x.view(torch.uint8), y.view(torch.uint8))
    del y
    # batched twice is the identity
    br.bitrev_batched(x, off, l2, ws)
    torch.cuda.synchronize()
    assert torch.equal(x.view(torch.uint8), keep.view(torch.uint8))
    del x, keep
    _free_gpu()


def test_c4_recipe_small_full_oracle():
    """The same recipe at 64 arrays, checked in full against the oracle."""
    data, offsets, log2n = workloads.batched_complex64(64, 8, 20, workloads.SEEDS["c4"])
    want = data.copy()
    oracle.batched(want, offsets, log2n)
    x = torch.from_numpy(data).cuda()
    br.bitrev_batched(x, torch.from_numpy(offsets).cuda(), torch.from_numpy(log2n).cuda())
    assert_bytes_equal(to_host_bytes(x), want, "c4 recipe, 64 arrays")


# --------------------------------------------------------------------------
# Graph capture
# --------------------------------------------------------------------------
def test_batched_graph_replays():
    from paper_1708_01873_amd.graph import BatchedGraph, CapturedCall
    data, offsets, log2n = workloads.batched_complex64(200, 0, 16, 77)
    want = data.copy()
    oracle.batched(want, offsets, log2n)
    x = torch.from_numpy(data).cuda()
    off = torch.from_numpy(offsets).cuda()
    l2 = torch.from_numpy(log2n).cuda()
    g = BatchedGraph(x, off, l2)
    eager = torch.from_numpy(data).cuda()
    for r in range(4):
        g.replay()
        br.bitrev_batched(eager, off, l2)       # eager work between replays
        torch.cuda.synchronize()
        expect = want if r % 2 == 0 else data
        assert_bytes_equal(to_host_bytes(x), expect, "graph replay %d" % r)
        assert_bytes_equal(to_host_bytes(eager), expect, "eager %d" % r)
    rows = torch.from_numpy(workloads.byte_pattern(8 * 4096 * 4, 5).view(np.int32).copy()).cuda()
    rows = rows.view(8, 4096)
    rows_host = to_host_bytes(rows)
    want_rows = oracle.rows(rows_host.view(np.int32).copy(), 12)
    c = CapturedCall(br.bitrev_rows, rows, rows)
    for r in range(3):
        c.replay()
        torch.cuda.synchronize()
        expect = want_rows if r % 2 == 0 else rows_host
        assert_bytes_equal(to_host_bytes(rows), expect, "rows graph replay %d" % r)


# --------------------------------------------------------------------------
# Differentiation: 256 x 2^16 float32
# --------------------------------------------------------------------------
def test_c5_autograd():
    from paper_1708_01873_amd.autograd import BitRev
    k, rows = 16, 256
    x_h, w_h = workloads.rows_float32(rows, k, workloads.SEEDS["c5"])
    x = torch.from_numpy(x_h).cuda().requires_grad_()
    w = torch.from_numpy(w_h).cuda()
    y = BitRev.apply(x)
    assert_bytes_equal(to_host_bytes(y), oracle.rows(x_h, k), "forward")
    loss = (w * y).sum()
    loss.backward()
    grad = x.grad.detach()
    # reference 1: the oracle applied to w, row by row
    assert_bytes_equal(to_host_bytes(grad), oracle.rows(w_h, k), "grad vs oracle(w)")
    # reference 2: autograd through a gather with the oracle's permutation
    perm = torch.from_numpy(oracle.rev_table(k)).cuda()
    xr = torch.from_numpy(x_h).cuda().requires_grad_()
    (w * xr[:, perm]).sum().backward()
    # The gather's backward adds into a zero tensor, so an exact -0.0 in w comes
    # back as +0.0 there (float32 normal draws do contain signed zeros); the
    # permutation kernel moves the bits.  Values must agree everywhere and the
    # bits may differ only at zeros.
    ref = to_host_bytes(xr.grad).view(np.float32)
    ours = to_host_bytes(grad).view(np.float32)
    assert np.array_equal(ref, ours)
    differ = ref.view(np.uint32) != ours.view(np.uint32)
    assert np.all(ours[differ] == 0.0) and np.all(np.signbit(ours[differ]))
    # central finite differences in float64 on 64 seeded coordinates
    coords = workloads.sample_coordinates(rows << k, 64, workloads.SEEDS["c5"])
    h = 1e-3
    g_h = to_host_bytes(grad).view(np.float32).reshape(rows, 1 << k)
    for c in coords:
        r, j = divmod(int(c), 1 << k)
        xrow = torch.from_numpy(x_h[r].astype(np.float64)).cuda()
        wrow = w_h[r].astype(np.float64)
        vals = []
        for sgn in (1.0, -1.0):
            xp = xrow.clone()
            xp[j] += sgn * h
            yp = BitRev.apply(xp.view(1, -1)).view(-1).cpu().numpy()
            vals.append(math.fsum((wrow * yp).tolist()))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - float(g_h[r, j])) <= 1e-6, (r, j, fd, float(g_h[r, j]))


def test_autograd_gradcheck_and_double_backward():
    from paper_1708_01873_amd.autograd import BitRev
    x = torch.randn(3, 32, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(BitRev.apply, (x,))
    assert torch.autograd.gradgradcheck(BitRev.apply, (x,))


@pytest.mark.parametrize("k,s", [(32, 1), (31, 2)])
def test_more_than_2p32_elements_or_bytes(k, s):
    """Element indices beyond 2^31 (k = 31, 32): 64-bit offsets throughout.
    Out of place, in place and in place again, each compared in full with the
    oracle (the input after the second application)."""
    n = 1 << k
    dt = torch.uint8 if s == 1 else torch.int16
    x = torch.empty(n, dtype=dt, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(k)
    x.view(torch.uint8).random_(0, 256, generator=g)
    host = to_host_bytes(x)
    y = br.bitrev_outofplace(x)
    _sampled_check(x, y, k, seed=k)     # quick first assertion
    want, _ = oracle.outofplace_mt(host, elem_size=s)
    assert_device_equal(y, want, "k=%d out of place" % k)
    del y
    _free_gpu()
    br.bitrev_inplace(x)
    assert_device_equal(x, want, "k=%d in place" % k)
    del want
    br.bitrev_inplace(x)
    assert_device_equal(x, host, "k=%d in place twice" % k)
    del x
    _free_gpu()
