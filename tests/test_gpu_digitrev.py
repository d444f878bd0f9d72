"""Digit reversal (radix-4, radix-8 orders) vs the oracle, byte for byte."""
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
@pytest.mark.parametrize("d", (1, 2, 3))
def test_digitrev_every_k(s, d):
    for k in range(0, 22, d):
        host = workloads.byte_pattern((1 << k) * s, seed=31 * k + d + s)
        want = oracle.digit_outofplace(host, d, s)
        x = to_device(host, s)
        y = br.bitrev_digitrev_outofplace(x, None, d, k)
        assert_bytes_equal(to_host_bytes(y), want, "oop s=%d d=%d k=%d" % (s, d, k))
        assert_bytes_equal(to_host_bytes(x), host, "source untouched")
        br.bitrev_digitrev_inplace(x, d, k)
        assert_bytes_equal(to_host_bytes(x), want, "ip s=%d d=%d k=%d" % (s, d, k))


def test_digitrev_complex64_2p24():
    """Full-size arrays, where the plans take the streaming cache hints:
    complex64 128 MiB (loads out of place, stores in place) and float32
    64 MiB (loads in and out of place)."""
    for name, host, s in (("c64", workloads.complex64_normal(24, workloads.SEEDS["c2"]), 8),
                          ("f32", workloads.byte_pattern((1 << 24) * 4, seed=44), 4)):
        for d in (2, 3):
            want = oracle.digit_outofplace(host, d, s)
            x = to_device(host, s)
            y = br.bitrev_digitrev_outofplace(x, None, d)
            assert_bytes_equal(to_host_bytes(y), want, "%s digits d=%d oop" % (name, d))
            br.bitrev_digitrev_inplace(x, d)
            assert_bytes_equal(to_host_bytes(x), want, "%s digits d=%d ip" % (name, d))


@pytest.mark.parametrize("s", (4, 8, 16))
def test_digitrev_forced_configs(s):
    """The configurable entries: every tile width that is a whole number of
    digits, every out-of-place tile order and XCD mapping, each cache hint;
    a width that is not a whole number of digits is refused."""
    for d, k in ((2, 16), (3, 18)):
        host = workloads.byte_pattern((1 << k) * s, seed=7 * s + d)
        want = oracle.digit_outofplace(host, d, s)
        for b in range(d, 7 if s < 16 else 6, d):
            for order in (1, 2, 3):
                for xcd, hints in ((1, 1), (2, 4), (1, 2), (2, 3)):
                    x = to_device(host, s)
                    y = br.bitrev_digitrev_outofplace(x, None, d, k, tile_bits=b, order=order,
                                                      xcd_remap=xcd, cache_hints=hints)
                    assert_bytes_equal(to_host_bytes(y), want, "oop s=%d d=%d b=%d o=%d x=%d h=%d"
                                       % (s, d, b, order, xcd, hints))
                    if order == 1:
                        br.bitrev_digitrev_inplace(x, d, k, tile_bits=b, xcd_remap=xcd,
                                                   cache_hints=hints)
                        assert_bytes_equal(to_host_bytes(x), want, "ip s=%d d=%d b=%d x=%d h=%d"
                                           % (s, d, b, xcd, hints))
        with pytest.raises(br.BitrevError) as e:
            br.bitrev_digitrev_inplace(to_device(host, s), d, k, tile_bits=d + 1)
        assert e.value.status == br.ERROR_NOT_SUPPORTED


def test_digitrev_misaligned_and_errors():
    host = workloads.byte_pattern((1 << 14) * 4, seed=5)
    want = oracle.digit_outofplace(host, 2, 4)
    x = to_device(host, 4, pad_front=1)
    br.bitrev_digitrev_inplace(x, 2, 14)
    assert_bytes_equal(to_host_bytes(x), want, "misaligned")
    with pytest.raises(br.BitrevError) as e:
        br.bitrev_digitrev_inplace(torch.zeros(1 << 13, device="cuda"), 2)
    assert e.value.status == br.ERROR_INVALID_VALUE
