"""The built-in plan table ships as data (csrc/plans_gfx950.inc): these CPU
tests read that text, look plans up in it the way its header describes,
and check that the library's plan query gives the same plan -- for the
headline (complex64 2^24 in place), the large configurations (complex128
2^28, float32 2^30) and every element size and size class -- and that
tuning-file rows apply only on the device they name."""
import os
import re

import pytest

import paper_1708_01873_amd as br

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1708_01873_amd", "csrc", "plans_gfx950.inc")
KINDS = ("inplace", "outofplace", "batched", "batched_oop", "dit_inplace", "dit_outofplace",
         "digit_inplace", "digit_outofplace")
PARENT = {"batched_oop": "batched", "dit_inplace": "inplace", "dit_outofplace": "outofplace",
          "digit_inplace": "inplace", "digit_outofplace": "outofplace"}
FIELDS = ("tile_bits", "wg_per_cu", "order", "variant", "xcd_remap", "cache_hints")
MAX_B = {1: 7, 2: 7, 4: 7, 8: 6, 16: 6}


def read_rows(text):
    body = re.search(r'R"PLANS\((.*)\)PLANS"', text, re.S).group(1)
    rows = []
    for line in body.splitlines():
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        assert len(line) == 14, line
        arch, cus, kind = line[0], int(line[1]), line[2]
        v = [int(t) for t in line[3:]]
        assert kind in KINDS
        rows.append(dict(arch=arch, cus=cus, kind=kind, s=v[0], d=v[1], bm=v[2], cmin=v[3],
                         cmax=v[4], f=dict(zip(FIELDS, v[5:]))))
    return rows


@pytest.fixture(scope="module")
def rows():
    return read_rows(open(TABLE).read())


def lookup(rows, kind, s, c, arch="gfx950", cus=256, d=0, bm=0):
    out = dict.fromkeys(FIELDS, 0)
    k = kind
    while k:
        for r in rows:
            if r["kind"] != k or (r["s"] and r["s"] != s) or (r["d"] and r["d"] != d):
                continue
            if (r["bm"] and r["bm"] != bm) or (r["cmin"] >= 0 and c < r["cmin"]):
                continue
            if (r["cmax"] >= 0 and c > r["cmax"]) or (r["cus"] and r["cus"] != cus):
                continue
            if r["arch"] != "*" and r["arch"] != arch:
                continue
            for f in FIELDS:
                if not out[f]:
                    out[f] = r["f"][f]
        k = PARENT.get(k)
    return out


def expected_plain(rows, mode, k, s, rows_n=1):
    kind = "inplace" if mode == br.MODE_INPLACE else "outofplace"
    c = ((s << k) * rows_n).bit_length() - 1
    f = lookup(rows, kind, s, c)
    b = f["tile_bits"] or MAX_B[s]
    b = min(b, MAX_B[s], k // 2)
    return dict(tile_bits=b, order=f["order"] or 2, xcd_remap=f["xcd_remap"] or 1,
                variant=f["variant"] or 1, cache_hints=f["cache_hints"] or 1)


def test_table_parses_and_covers_every_kind(rows):
    kinds = {r["kind"] for r in rows}
    assert kinds == set(KINDS)
    assert any(r["arch"] == "*" for r in rows)
    assert all(r["arch"] in ("*", "gfx950") for r in rows)


@pytest.mark.parametrize("mode,k,s", [
    (br.MODE_INPLACE, 24, 8),      # the headline
    (br.MODE_OUTOFPLACE, 24, 8),
    (br.MODE_INPLACE, 28, 16), (br.MODE_OUTOFPLACE, 28, 16),   # complex128 2^28
    (br.MODE_INPLACE, 30, 4), (br.MODE_OUTOFPLACE, 30, 4),     # float32 2^30
])
def test_headline_and_large_configs_follow_the_table(rows, mode, k, s):
    p = br.bitrev_plan_query(k, s, mode=mode)
    want = expected_plain(rows, mode, k, s)
    assert {f: p[f] for f in want} == want


@pytest.mark.parametrize("s", (1, 2, 4, 8, 16))
@pytest.mark.parametrize("mode", (br.MODE_INPLACE, br.MODE_OUTOFPLACE))
def test_every_size_class_follows_the_table(rows, mode, s):
    for k in range(14, 33):
        if (s << k) > (1 << 36):
            continue
        p = br.bitrev_plan_query(k, s, mode=mode)
        want = expected_plain(rows, mode, k, s)
        assert {f: p[f] for f in want} == want, (mode, s, k)


def test_batched_follows_the_table(rows):
    for s in (1, 2, 4, 8, 16):
        p = br.bitrev_plan_query(0, s, mode=br.MODE_BATCHED)
        f1 = lookup(rows, "batched", s, -1)
        b = f1["tile_bits"] or MAX_B[s]
        f = lookup(rows, "batched", s, -1, bm=b)
        assert p["tile_bits"] == b and p["order"] == (f["order"] or 2), s
        assert p["xcd_remap"] == (f["xcd_remap"] or 1), s
        if f["wg_per_cu"]:
            assert p["grid_blocks"] == f["wg_per_cu"] * 256, s


def test_tuning_rows_apply_only_on_their_device(tmp_path):
    """A row for another architecture or another compute-unit count (a
    partitioned device) leaves the plan alone; a row for this device (the
    host query assumes gfx950 with 256 compute units) or for any device
    changes it."""
    base = br.bitrev_plan_query(24, 8)
    assert base["tile_bits"] == 5
    cases = [("gfx942 304", False), ("gfx950 128", False), ("gfx950 256", True), ("* 0", True),
             ("gfx950 0", True)]
    for who, applies in cases:
        path = tmp_path / ("t_%s.txt" % who.replace(" ", "_").replace("*", "any"))
        path.write_text("%s inplace 8 0 0 -1 -1   4 0 3 1 1 2\n" % who)
        br.bitrev_load_tuning(str(path))
        try:
            p = br.bitrev_plan_query(24, 8)
            got = (p["tile_bits"], p["order"], p["xcd_remap"], p["cache_hints"])
            if applies:
                assert got == (4, 3, 1, 2), who
            else:
                assert got == (base["tile_bits"], base["order"], base["xcd_remap"],
                               base["cache_hints"]), who
        finally:
            br.bitrev_load_tuning(None)


def test_malformed_table_row_is_rejected(tmp_path):
    path = tmp_path / "bad.txt"
    path.write_text("gfx950 256 inplace 8 0 0 -1 -1 4 0 3 1 1\n")   # 13 fields
    with pytest.raises(br.BitrevError):
        br.bitrev_load_tuning(str(path))
    path.write_text("gfx950 256 sideways 8 0 0 -1 -1 4 0 3 1 1 2\n")
    with pytest.raises(br.BitrevError):
        br.bitrev_load_tuning(str(path))
    assert br.bitrev_plan_query(24, 8)["tile_bits"] == 5
