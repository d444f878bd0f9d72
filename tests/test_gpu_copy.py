"""The reference copies that bound the permutation: the linear streaming copy
in its four cache-hint forms and the copy in the tile kernels' order.  A copy
must return its source byte for byte."""
import numpy as np
import pytest

import paper_1708_01873_amd as br
from gpu_util import assert_device_equal, to_device, to_host_bytes
from paper_1708_01873_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    br.lib()


@pytest.mark.parametrize("s", (1, 2, 4, 8, 16))
@pytest.mark.parametrize("k", (0, 3, 6, 7, 12, 17, 20))
def test_copy_tiled_default_plan(s, k):
    host = workloads.byte_pattern((1 << k) * s, 300 + 7 * k + s)
    x = to_device(host, s)
    y = torch.zeros_like(x)
    br.bitrev_copy_tiled(x, y)
    assert_device_equal(y, host, "tiled copy k=%d s=%d" % (k, s))


@pytest.mark.parametrize("hints", (1, 2, 3, 4))
@pytest.mark.parametrize("order", (1, 2, 3))
@pytest.mark.parametrize("s,b", [(1, 7), (2, 4), (4, 6), (8, 4), (8, 5), (8, 6), (16, 5), (16, 3)])
def test_copy_tiled_forced_plans(s, b, order, hints):
    k = 2 * b + 5
    host = workloads.byte_pattern((1 << k) * s, 400 + 13 * b + s + order)
    x = to_device(host, s)
    y = torch.zeros_like(x)
    br.bitrev_copy_tiled(x, y, tile_bits=b, order=order, cache_hints=hints,
                         xcd_remap=1 + (order % 2), grid_blocks=64 if hints == 2 else 0)
    assert_device_equal(y, host, "tiled copy s=%d b=%d order=%d hints=%d" % (s, b, order, hints))


def test_copy_tiled_rejects_unaligned_and_overlap():
    x = torch.zeros(1 << 16 + 1, dtype=torch.int32, device="cuda")
    y = torch.zeros(1 << 16 + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_copy_tiled(x[1:1 + (1 << 16)], y[:1 << 16])
    assert e.value.status == br.ERROR_NOT_SUPPORTED
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_copy_tiled(x[:1 << 16], x[1 << 15:(1 << 15) + (1 << 16)])
    assert e.value.status == br.ERROR_ALIAS


@pytest.mark.parametrize("hints", (0, 1, 2, 3, 4))
def test_copy_linear_hints(hints):
    host = workloads.byte_pattern((1 << 22) + 13, 500 + hints)
    x = torch.from_numpy(host).cuda()
    y = torch.zeros_like(x)
    br.bitrev_copy(x, y, cache_hints=hints)
    assert_device_equal(y, host, "linear copy hints=%d" % hints)


def test_copy_tiled_4gib_float32():
    """The 4 GiB float32 array of the large configuration, in the default
    out-of-place plan's tile order: the copy equals its source."""
    x = workloads.device_normal(1 << 30, workloads.SEEDS["c3b"], torch.float32)
    y = torch.empty_like(x)
    br.bitrev_copy_tiled(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x.view(torch.int32), y.view(torch.int32))
    del x, y
    torch.cuda.empty_cache()
