"""The allocation-free batched entry point (bitrev_batched_noalloc), through
the C ABI, against the workspace form (bitrev_batched) and the oracle: two
calls in a row on one device, the second on a smaller batch, so the second
call runs on the scratch array the first one left behind."""
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


def _batch(num, kmin, kmax, seed, s):
    offsets, log2n = workloads.batched_layout(num, kmin, kmax, seed)
    host = workloads.byte_pattern(int(offsets[-1]) * s, seed + 500)
    return host, offsets, log2n


def _meta(offsets, log2n):
    return (torch.from_numpy(np.asarray(offsets, dtype=np.int64)).cuda(),
            torch.from_numpy(np.asarray(log2n, dtype=np.int32)).cuda())


def _one_call(host, offsets, log2n, s, what):
    want = host.copy()
    oracle.batched(want, offsets, log2n, s)
    off, l2 = _meta(offsets, log2n)
    x = to_device(host, s)
    ref = to_device(host, s)
    ws = torch.empty(br.bitrev_batched_workspace_size(len(log2n)), dtype=torch.uint8,
                     device="cuda")
    br.bitrev_batched(ref, off, l2, ws)
    br.bitrev_batched_noalloc(x, off, l2)
    got = to_host_bytes(x)
    assert_bytes_equal(got, to_host_bytes(ref), what + ": noalloc vs bitrev_batched")
    assert_bytes_equal(got, want, what + ": noalloc vs oracle")
    assert br.bitrev_batched_errors(ws) == (0, -1)


@pytest.mark.parametrize("s", (8, 4))
def test_noalloc_two_calls_second_smaller(s):
    # first call: many uneven arrays, tile path and whole-array path mixed
    host, offsets, log2n = _batch(3000, 0, 16, 900 + s, s)
    _one_call(host, offsets, log2n, s, "first call, 3000 arrays")
    # second call: fewer and shorter arrays on the scratch the first left
    host, offsets, log2n = _batch(37, 2, 13, 950 + s, s)
    _one_call(host, offsets, log2n, s, "second call, 37 arrays")


def test_noalloc_at_the_limit_then_small():
    n = br.NOALLOC_MAX_ARRAYS
    host, offsets, log2n = _batch(n, 0, 8, 977, 8)
    _one_call(host, offsets, log2n, 8, "%d arrays" % n)
    host, offsets, log2n = _batch(5, 10, 18, 978, 8)
    _one_call(host, offsets, log2n, 8, "5 arrays after the limit")


def test_noalloc_rejects_more_than_its_scratch_holds():
    n = br.NOALLOC_MAX_ARRAYS + 1
    offsets = np.arange(n + 1, dtype=np.int64)
    log2n = np.zeros(n, dtype=np.int32)
    x = torch.zeros(n, dtype=torch.int64, device="cuda")
    off, l2 = _meta(offsets, log2n)
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_batched_noalloc(x, off, l2)
    assert e.value.status == br.ERROR_WORKSPACE
