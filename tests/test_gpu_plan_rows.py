"""Every row of the built-in plan table, run on the GPU: each row's launch
configuration (tile width, workgroups per CU, order, kernel variant, XCD
mapping, cache hints) is forced on a small array of the row's element size
(every size for a row that matches any) and the result is compared with the
oracle -- byte for byte for the permutations, within Higham's bound for the
fused DIT levels.  The size-class bounds of a row only choose where it
applies; the kernels it selects must be right at any size."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1708_01873_amd as br
from gpu_util import assert_bytes_equal, to_device, to_host_bytes
from oracle import dit
from paper_1708_01873_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1708_01873_amd", "csrc", "plans_gfx950.inc")
MAX_B = {1: 7, 2: 7, 4: 7, 8: 6, 16: 6}
CUS = 256


def _rows():
    text = open(TABLE).read()
    body = re.search(r'R"PLANS\((.*)\)PLANS"', text, re.S).group(1)
    out = []
    for line in body.splitlines():
        f = line.split("#", 1)[0].split()
        if not f:
            continue
        v = [int(t) for t in f[3:]]
        out.append(dict(text=" ".join(f), kind=f[2], s=v[0], d=v[1], bm=v[2], b=v[5], wg=v[6],
                        order=v[7], variant=v[8], xcd=v[9], hints=v[10]))
    return out


ROWS = _rows()


def _ids(kinds):
    return [r for r in ROWS if r["kind"] in kinds]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    br.lib()


def _cfg(r, b):
    return dict(tile_bits=b, grid_blocks=r["wg"] * CUS, order=r["order"], xcd_remap=r["xcd"],
                cache_hints=r["hints"])


@pytest.mark.parametrize("r", _ids(("inplace", "outofplace")), ids=lambda r: r["text"])
def test_plain_row(r):
    for s in ([r["s"]] if r["s"] else [1, 2, 4, 8, 16]):
        b = r["b"] or r["bm"]
        k = 2 * (b or MAX_B[s]) + 3
        host = workloads.byte_pattern((1 << k) * s, seed=1000 + 7 * k + s)
        want = oracle.outofplace(host, s)
        x = to_device(host, s)
        cfg = dict(_cfg(r, b), variant=r["variant"])
        if r["kind"] == "inplace":
            br.bitrev_inplace(x, k, **cfg)
            got = to_host_bytes(x)
        else:
            y = torch.empty_like(x)
            br.bitrev_outofplace(x, y, k, **cfg)
            got = to_host_bytes(y)
        assert_bytes_equal(got, want, "%s, s=%d, k=%d" % (r["text"], s, k))


@pytest.mark.parametrize("r", _ids(("batched",)), ids=lambda r: r["text"])
def test_batched_row(r):
    for s in ([r["s"]] if r["s"] else [1, 2, 4, 8, 16]):
        offsets, log2n = workloads.batched_layout(48, 0, 2 * MAX_B[s] + 2, 300 + s)
        host = workloads.byte_pattern(int(offsets[-1]) * s, seed=400 + s)
        want = host.copy()
        oracle.batched(want, offsets, log2n, s)
        x = to_device(host, s)
        cfg = dict(_cfg(r, r["b"] or r["bm"]), variant=r["variant"])
        br.bitrev_batched(x, torch.from_numpy(offsets).cuda(), torch.from_numpy(log2n).cuda(), **cfg)
        assert_bytes_equal(to_host_bytes(x), want, "%s, s=%d" % (r["text"], s))


@pytest.mark.parametrize("r", _ids(("batched_oop",)), ids=lambda r: r["text"])
def test_batched_outofplace_row(r):
    """The out-of-place batch takes its plan from the table (no forced
    configuration): run it for the row's element size."""
    for s in ([r["s"]] if r["s"] else [1, 2, 4, 8, 16]):
        offsets, log2n = workloads.batched_layout(48, 0, 2 * MAX_B[s] + 2, 500 + s)
        host = workloads.byte_pattern(int(offsets[-1]) * s, seed=600 + s)
        want = host.copy()
        oracle.batched(want, offsets, log2n, s)
        x = to_device(host, s)
        y = torch.empty_like(x)
        br.bitrev_batched_outofplace(x, y, torch.from_numpy(offsets).cuda(),
                                     torch.from_numpy(log2n).cuda())
        assert_bytes_equal(to_host_bytes(y), want, "%s, s=%d" % (r["text"], s))


@pytest.mark.parametrize("r", _ids(("digit_inplace", "digit_outofplace")), ids=lambda r: r["text"])
def test_digit_row(r):
    for s in ([r["s"]] if r["s"] else [1, 2, 4, 8, 16]):
        for d in ([r["d"]] if r["d"] else [2, 3]):
            b = r["b"] or r["bm"]
            if b and b % d:
                continue                       # the row never applies to this digit width
            bb = b or (MAX_B[s] - MAX_B[s] % d)
            k = 2 * bb + d
            host = workloads.byte_pattern((1 << k) * s, seed=700 + 11 * k + s + d)
            want = oracle.digit_outofplace(host, d, s)
            x = to_device(host, s)
            cfg = _cfg(r, b)
            if r["kind"] == "digit_inplace":
                br.bitrev_digitrev_inplace(x, d, k, **cfg)
                got = to_host_bytes(x)
            else:
                got = to_host_bytes(br.bitrev_digitrev_outofplace(x, None, d, k, **cfg))
            assert_bytes_equal(got, want, "%s, s=%d, d=%d, k=%d" % (r["text"], s, d, k))


U = {8: 2.0 ** -24, 16: 2.0 ** -53}


def _check_dit(got, x, L, dtype):
    prec = np.clongdouble if dtype == np.complex128 else np.complex128
    want = dit.dit_stages(x, L, False, precision=prec)
    q = 1 << L
    g = got.astype(prec).reshape(-1, q)
    w = want.reshape(-1, q)
    err = np.linalg.norm(g - w, axis=1)
    ref = np.linalg.norm(w, axis=1)
    bound = dit.higham_bound(L, U[np.dtype(dtype).itemsize], U[np.dtype(dtype).itemsize])
    assert np.all(err <= bound * ref + 1e-30), (float((err / np.maximum(ref, 1e-300)).max()), bound)


@pytest.mark.parametrize("r", _ids(("dit_inplace", "dit_outofplace")), ids=lambda r: r["text"])
def test_dit_row(r):
    for s in ([r["s"]] if r["s"] else [8, 16]):
        dtype = np.complex64 if s == 8 else np.complex128
        b = r["b"] or r["bm"]
        bb = b or MAX_B[s]
        k = 2 * bb + 2
        rng = np.random.default_rng(800 + k + s)
        x = (rng.standard_normal(1 << k) + 1j * rng.standard_normal(1 << k)).astype(dtype)
        for L in sorted({1, min(3, bb), bb}):
            t = torch.from_numpy(x).cuda()
            cfg = dict(_cfg(r, b), variant=r["variant"])
            if r["kind"] == "dit_inplace":
                br.bitrev_dit_stages(t, t, stages=L, **cfg)
                got = to_host_bytes(t)
            else:
                got = to_host_bytes(br.bitrev_dit_stages(t, stages=L, **cfg))
            _check_dit(got.view(dtype), x, L, dtype)
