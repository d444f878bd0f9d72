"""Batched (uneven lengths, one persistent launch) vs the oracle, and its
metadata checks."""
import numpy as np
import pytest

import oracle
import paper_1708_01873_amd as br
from gpu_util import assert_bytes_equal, to_device, to_host_bytes
from paper_1708_01873_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    br.lib()


def _meta(offsets, log2n):
    return (torch.from_numpy(np.asarray(offsets, dtype=np.int64)).cuda(),
            torch.from_numpy(np.asarray(log2n, dtype=np.int32)).cuda())


@pytest.mark.parametrize("s", (1, 2, 4, 8, 16))
def test_batched_mixed_sizes(s):
    """k from 0 to 16, including arrays below 16 bytes that leave later
    arrays misaligned, at every batched tile width."""
    offsets, log2n = workloads.batched_layout(97, 0, 16, seed=40 + s)
    host = workloads.byte_pattern(int(offsets[-1]) * s, seed=s)
    want = host.copy()
    oracle.batched(want, offsets, log2n, s)
    for b in range(2, {1: 7, 2: 7, 4: 7, 8: 6, 16: 6}[s] + 1):
        for order in (1, 2):
            x = to_device(host, s)
            off, l2 = _meta(offsets, log2n)
            ws = torch.empty(br.bitrev_batched_workspace_size(len(log2n)), dtype=torch.uint8,
                             device="cuda")
            br.bitrev_batched(x, off, l2, ws, tile_bits=b, order=order)
            assert_bytes_equal(to_host_bytes(x), want, "batched s=%d b=%d order=%d" % (s, b, order))
            assert br.bitrev_batched_errors(ws) == (0, -1)


@pytest.mark.parametrize("s", (1, 2, 4, 8))
@pytest.mark.parametrize("oop", (False, True))
def test_batched_misaligned_large_arrays(s, oop):
    """Arrays long enough for the tile path that start off the 16-byte grid
    (after a 1-element array): they take the element-by-element tile routine,
    in place at every batched tile width, out of place at the default one."""
    log2n = np.array([0, 14, 0, 0, 13, 1, 12, 0, 15, 2, 12], dtype=np.int32)
    offsets = np.concatenate([[0], np.cumsum(1 << log2n.astype(np.int64))]).astype(np.int64)
    assert any((int(o) * s) % 16 for o, k in zip(offsets[:-1], log2n) if k >= 12)
    host = workloads.byte_pattern(int(offsets[-1]) * s, seed=70 + s)
    want = host.copy()
    oracle.batched(want, offsets, log2n, s)
    # out of place has no config: its default plan only
    for b in ((0,) if oop else range(2, {1: 7, 2: 7, 4: 7, 8: 6}[s] + 1)):
        x = to_device(host, s)
        off, l2 = _meta(offsets, log2n)
        ws = torch.empty(br.bitrev_batched_workspace_size(len(log2n)), dtype=torch.uint8,
                         device="cuda")
        if oop:
            y = torch.empty_like(x)
            br.bitrev_batched_outofplace(x, y, off, l2, ws)
            got = to_host_bytes(y)
        else:
            br.bitrev_batched(x, off, l2, ws, tile_bits=b)
            got = to_host_bytes(x)
        assert_bytes_equal(got, want, "misaligned batched s=%d b=%d oop=%s" % (s, b, oop))
        assert br.bitrev_batched_errors(ws) == (0, -1)


def test_batched_default_plan_and_grids():
    offsets, log2n = workloads.batched_layout(300, 0, 18, seed=5)
    host = workloads.byte_pattern(int(offsets[-1]) * 8, seed=9)
    want = host.copy()
    oracle.batched(want, offsets, log2n, 8)
    for grid in (0, 8, 40, 4096):
        x = to_device(host, 8)
        off, l2 = _meta(offsets, log2n)
        br.bitrev_batched(x, off, l2, grid_blocks=grid)
        assert_bytes_equal(to_host_bytes(x), want, "grid=%d" % grid)


def test_batched_rejects_bad_arrays():
    """An array whose length is not 2^log2n, or that runs past the data, is
    left untouched and reported; the others are still permuted."""
    log2n = np.array([10, 5, 12, 7, 3], dtype=np.int32)
    offsets = np.concatenate([[0], np.cumsum(1 << log2n.astype(np.int64))]).astype(np.int64)
    host = workloads.byte_pattern(int(offsets[-1]) * 4, seed=3)
    bad_l2 = log2n.copy()
    bad_l2[1] = 6          # length 32 but claims 64
    bad_l2[3] = -2         # out of range
    want = host.copy()
    for a in (0, 2, 4):
        seg = want[offsets[a] * 4:offsets[a + 1] * 4]
        want[offsets[a] * 4:offsets[a + 1] * 4] = oracle.outofplace(seg, 4)
    x = to_device(host, 4)
    off, l2 = _meta(offsets, bad_l2)
    ws = torch.empty(br.bitrev_batched_workspace_size(5), dtype=torch.uint8, device="cuda")
    br.bitrev_batched(x, off, l2, ws)
    assert_bytes_equal(to_host_bytes(x), want, "batched with rejected arrays")
    assert br.bitrev_batched_errors(ws) == (2, 1)
    # data_elems smaller than the last array's end: that array is rejected
    x = to_device(host, 4)
    x_short = x[:int(offsets[-1]) - 1]
    off, l2 = _meta(offsets, log2n)
    br.bitrev_batched(x_short, off, l2, ws)
    assert br.bitrev_batched_errors(ws) == (1, 4)


def test_batched_workspace_too_small():
    offsets, log2n = workloads.batched_layout(4, 4, 6, seed=1)
    x = torch.zeros(int(offsets[-1]), dtype=torch.int64, device="cuda")
    off, l2 = _meta(offsets, log2n)
    ws = torch.empty(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_batched(x, off, l2, ws)
    assert e.value.status == br.ERROR_WORKSPACE
