"""Out-of-place batched, strided rows and the even-odd split vs the oracle."""
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


@pytest.mark.parametrize("s", (1, 4, 8, 16))
def test_batched_outofplace(s):
    offsets, log2n = workloads.batched_layout(150, 0, 17, seed=60 + s)
    host = workloads.byte_pattern(int(offsets[-1]) * s, seed=s + 1)
    want = host.copy()
    oracle.batched(want, offsets, log2n, s)
    x = to_device(host, s)
    y = torch.empty_like(x)
    off = torch.from_numpy(offsets).cuda()
    l2 = torch.from_numpy(log2n).cuda()
    ws = torch.empty(br.bitrev_batched_workspace_size(150), dtype=torch.uint8, device="cuda")
    br.bitrev_batched_outofplace(x, y, off, l2, ws)
    assert_bytes_equal(to_host_bytes(y), want, "batched oop s=%d" % s)
    assert_bytes_equal(to_host_bytes(x), host, "source untouched")
    assert br.bitrev_batched_errors(ws) == (0, -1)


@pytest.mark.parametrize("s", (2, 8, 16))
def test_rows_strided(s):
    for k, rows, ss, ds in ((4, 9, 20, 16), (10, 5, 1024 + 16, 2048), (13, 3, 8192 + 4, 8192 + 64)):
        n = 1 << k
        host = workloads.byte_pattern(((rows - 1) * ss + n) * s, seed=k + s)
        x = to_device(host, s)
        y = torch.zeros(((rows - 1) * ds + n), dtype=x.dtype, device="cuda")
        br.bitrev_rows_strided(x, y, k, rows, ss, ds)
        got = to_host_bytes(y).reshape(-1)
        el = host.reshape(-1, s)
        for r in range(rows):
            want = oracle.outofplace(np.ascontiguousarray(el[r * ss:r * ss + n]).reshape(-1), s)
            assert_bytes_equal(got[r * ds * s:(r * ds + n) * s], want, "strided row %d" % r)
            if r + 1 < rows:  # the gaps between destination rows stay zero
                assert not got[(r * ds + n) * s:(r + 1) * ds * s].any()
        # in place with equal strides
        br.bitrev_rows_strided(x, x, k, rows, ss, ss)
        gx = to_host_bytes(x).reshape(-1, s)
        for r in range(rows):
            want = oracle.outofplace(np.ascontiguousarray(el[r * ss:r * ss + n]).reshape(-1), s)
            assert_bytes_equal(gx[r * ss:r * ss + n].reshape(-1), want, "strided ip row %d" % r)
            if r + 1 < rows:
                assert_bytes_equal(gx[r * ss + n:(r + 1) * ss].reshape(-1),
                                   el[r * ss + n:(r + 1) * ss].reshape(-1), "gap untouched")


@pytest.mark.parametrize("s", (1, 2, 4, 8, 16))
def test_evenodd(s):
    for k, rows in ((1, 3), (4, 5), (11, 2), (20, 1)):
        host = workloads.byte_pattern((rows << k) * s, seed=k * 7 + s)
        want = np.concatenate([oracle.evenodd(np.ascontiguousarray(r), s)
                               for r in host.reshape(rows, -1)])
        x = to_device(host, s)
        y = br.bitrev_evenodd(x.view(rows, -1))
        assert_bytes_equal(to_host_bytes(y), want, "evenodd s=%d k=%d" % (s, k))
