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


@pytest.mark.parametrize("levels", (0, 1, 2))
@pytest.mark.parametrize("s", (1, 2, 4, 8, 16))
def test_recursive_matches_oracle(s, levels):
    for k in range(0, 23, 2):
        h = k // 2
        two_fits = h % 2 == 0 and (s << h) <= 65536
        host = workloads.byte_pattern((1 << k) * s, seed=k + s)
        x = to_device(host, s)
        if levels == 2 and not two_fits:
            with pytest.raises(br.BitrevError) as e:
                br.bitrev_inplace_recursive(x, k, levels=2)
            assert e.value.status == br.ERROR_NOT_SUPPORTED
            continue
        br.bitrev_inplace_recursive(x, k, levels=levels)
        assert_bytes_equal(to_host_bytes(x), oracle.outofplace(host, s),
                           "recursive s=%d k=%d levels=%d" % (s, k, levels))


@pytest.mark.parametrize("s", (1, 2, 4, 8, 16))
def test_recursive_two_levels_unaligned_base(s):
    """The LDS stage of the second level with a base that is only
    element-aligned (element-wise block loads)."""
    k = 16
    host = workloads.byte_pattern((1 << k) * s, seed=99 + s)
    x = to_device(host, s, pad_front=1)
    br.bitrev_inplace_recursive(x, k, levels=2)
    assert_bytes_equal(to_host_bytes(x), oracle.outofplace(host, s), "recursive unaligned s=%d" % s)


@pytest.mark.parametrize("k,dtype", [(24, "complex128"), (28, "float32")])
def test_recursive_two_levels_64kib_blocks(k, dtype):
    """The paper's own workload (complex doubles, k = 24) and float32 2^28:
    2^(k/2)-element blocks of exactly 64 KiB in the LDS stage."""
    tdt = getattr(torch, dtype)
    x = workloads.device_normal(1 << k, k, tdt)
    host = to_host_bytes(x)
    br.bitrev_inplace_recursive(x, levels=2)
    want, _ = oracle.outofplace_mt(host, elem_size=x.element_size())
    assert_bytes_equal(to_host_bytes(x), want, "recursive two levels k=%d %s" % (k, dtype))
    del x
    torch.cuda.empty_cache()


def test_recursive_c2_full():
    host = workloads.complex64_normal(24, workloads.SEEDS["c2"])
    x = torch.from_numpy(host).cuda()
    br.bitrev_inplace_recursive(x)
    assert_bytes_equal(to_host_bytes(x), oracle.outofplace(host), "recursive c2")
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_inplace_recursive(x[: 1 << 23])
    assert e.value.status == br.ERROR_NOT_SUPPORTED
