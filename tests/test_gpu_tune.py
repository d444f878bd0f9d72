"""The autotuner: candidates run, the table it writes loads into the library
and drives the plan, and tuning leaves the caller's batch unchanged."""
import numpy as np
import pytest

import oracle
import paper_1708_01873_amd as br
from gpu_util import assert_bytes_equal, to_host_bytes
from paper_1708_01873_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    br.lib()


def test_tune_plain_and_load(tmp_path):
    from paper_1708_01873_amd import tune
    r_ip = tune.tune_plain(18, 8, br.MODE_INPLACE, reps=4, flush=False)
    r_oop = tune.tune_plain(18, 8, br.MODE_OUTOFPLACE, reps=4, flush=False)
    assert r_ip.ranking and r_ip.best.ms <= min(c.ms for c in r_ip.ranking)
    path = tune.write_tuning([r_ip, r_oop], str(tmp_path / "t.txt"))
    br.bitrev_load_tuning(path)
    try:
        p = br.bitrev_plan_query(18, 8)
        assert (p["tile_bits"], p["order"], p["variant"]) == (
            r_ip.best.tile_bits, r_ip.best.order, r_ip.best.variant)
        if r_ip.best.cache_hints:
            assert p["cache_hints"] == r_ip.best.cache_hints
        # the tuned plan still computes the permutation
        host = workloads.complex64_normal(18, 3)
        x = torch.from_numpy(host).cuda()
        br.bitrev_inplace(x)
        assert_bytes_equal(to_host_bytes(x), oracle.outofplace(host), "tuned plan")
    finally:
        br.bitrev_load_tuning(None)


def test_tune_batched_keeps_data(tmp_path):
    from paper_1708_01873_amd import tune
    data, offsets, log2n = workloads.batched_complex64(300, 4, 16, 11)
    x = torch.from_numpy(data).cuda()
    off = torch.from_numpy(offsets).cuda()
    l2 = torch.from_numpy(log2n).cuda()
    r = tune.tune_batched(x, off, l2, reps=2, wg_per_cu=(0, 4), tile_bits=[4, 5])
    assert_bytes_equal(to_host_bytes(x), data, "batch after tuning")
    path = tune.write_tuning([r], str(tmp_path / "b.txt"))
    br.bitrev_load_tuning(path)
    try:
        p = br.bitrev_plan_query(0, 8, mode=br.MODE_BATCHED)
        assert p["tile_bits"] == r.best.tile_bits and p["order"] == r.best.order
        want = data.copy()
        oracle.batched(want, offsets, log2n)
        br.bitrev_batched(x, off, l2)
        assert_bytes_equal(to_host_bytes(x), want, "tuned batched plan")
    finally:
        br.bitrev_load_tuning(None)


def test_tune_table_rows_load_and_drive_the_plan(tmp_path):
    """A table swept on this device (two size classes, complex64) is written
    in the built-in table's row format, keyed by this device; loaded, it
    drives the plans of those classes, and the plans still compute the
    permutation."""
    from paper_1708_01873_amd import tune
    path = str(tmp_path / "table.txt")
    results = tune.tune_table(path, elem_sizes=(8,), classes=range(21, 23), reps=2)
    assert len(results) == 4
    arch, cus = tune.device_key()
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows and all(r[0] == arch and int(r[1]) == cus and len(r) == 14 for r in rows)
    br.bitrev_load_tuning(path)
    try:
        for r in results:
            p = br.bitrev_plan_query(r.log2n, 8, mode=r.mode)
            assert (p["tile_bits"], p["order"], p["variant"]) == (
                r.best.tile_bits, r.best.order, r.best.variant), (r.mode, r.log2n)
            host = workloads.complex64_normal(r.log2n, 4)
            x = torch.from_numpy(host).cuda()
            if r.mode == br.MODE_INPLACE:
                br.bitrev_inplace(x)
                got = x
            else:
                got = br.bitrev_outofplace(x)
            assert_bytes_equal(to_host_bytes(got), oracle.outofplace(host), "table plan")
    finally:
        br.bitrev_load_tuning(None)
