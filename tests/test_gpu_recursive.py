"""The paper's recursive scheme (A/B baseline) and the square transpose vs
the oracle and numpy."""
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


@pytest.mark.parametrize("s", (1, 2, 4, 8, 16))
def test_transpose_inplace(s):
    for h in range(0, 12):
        n = 1 << h
        host = workloads.byte_pattern(n * n * s, seed=h + 10 * s)
        want = host.reshape(n, n, s).transpose(1, 0, 2).reshape(-1)
        x = to_device(host, s)
        br.bitrev_transpose_inplace(x, h)
        assert_bytes_equal(to_host_bytes(x), want, "transpose s=%d h=%d" % (s, h))


@pytest.mark.parametrize("s", (1, 4, 8, 16))
def test_recursive_matches_oracle(s):
    for k in range(0, 23, 2):
        host = workloads.byte_pattern((1 << k) * s, seed=k + s)
        x = to_device(host, s)
        br.bitrev_inplace_recursive(x, k)
        assert_bytes_equal(to_host_bytes(x), oracle.outofplace(host, s),
                           "recursive s=%d k=%d" % (s, k))


def test_recursive_c2_full():
    host = workloads.complex64_normal(24, workloads.SEEDS["c2"])
    x = torch.from_numpy(host).cuda()
    br.bitrev_inplace_recursive(x)
    assert_bytes_equal(to_host_bytes(x), oracle.outofplace(host), "recursive c2")
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_inplace_recursive(x[: 1 << 23])
    assert e.value.status == br.ERROR_NOT_SUPPORTED
