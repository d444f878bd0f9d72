"""The C ABI on the host: symbols, argument validation, plans, tuning files and
the kernels' index arithmetic (host build of the same source).  No GPU needed:
every call here either fails validation before any HIP call or is host-only.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1708_01873_amd as br

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(br.LIBRARY):
        import __graft_entry__
        __graft_entry__.build()
    return br.lib()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "bitrev.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(bitrev_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(L):
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(br.EXPORTED)


def test_abi_version_and_status_strings(L):
    assert br.abi_version() == 2
    for st in range(6):
        assert br.status_string(st)
    assert br.status_string(99) == "unknown status"


FAKE = 1 << 20  # a nonzero, 16-byte aligned address never dereferenced


@pytest.mark.parametrize("args,want", [
    ((None, 10, 4), br.ERROR_INVALID_VALUE),
    ((FAKE, -1, 4), br.ERROR_INVALID_VALUE),
    ((FAKE, 41, 4), br.ERROR_INVALID_VALUE),
    ((FAKE, 10, 3), br.ERROR_INVALID_VALUE),
    ((FAKE, 10, 0), br.ERROR_INVALID_VALUE),
    ((FAKE, 10, 32), br.ERROR_INVALID_VALUE),
    ((FAKE + 2, 10, 4), br.ERROR_INVALID_VALUE),
    ((FAKE + 8, 10, 16), br.ERROR_INVALID_VALUE),
])
def test_inplace_validation(L, args, want):
    assert L.bitrev_inplace(args[0], args[1], args[2], None) == want


def test_trivial_inplace_needs_no_device(L):
    # n = 1 and n = 2 are the identity: success without touching HIP
    assert L.bitrev_inplace(FAKE, 0, 8, None) == br.SUCCESS
    assert L.bitrev_inplace(FAKE, 1, 8, None) == br.SUCCESS


def test_outofplace_validation(L):
    n4 = 4 << 10
    assert L.bitrev_outofplace(FAKE, FAKE, 10, 4, None) == br.ERROR_ALIAS
    assert L.bitrev_outofplace(FAKE, FAKE + n4 - 4, 10, 4, None) == br.ERROR_ALIAS
    assert L.bitrev_outofplace(FAKE + n4 - 4, FAKE, 10, 4, None) == br.ERROR_ALIAS
    assert L.bitrev_outofplace(None, FAKE, 10, 4, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_outofplace(FAKE, None, 10, 4, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_outofplace(FAKE, FAKE + n4 + 2, 10, 4, None) == br.ERROR_INVALID_VALUE


def test_rows_validation(L):
    assert L.bitrev_rows(FAKE, FAKE + 4096, 10, -1, 4, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_rows(FAKE, FAKE + 4096, 10, 0, 4, None) == br.SUCCESS
    # two rows of 4 KiB overlap a destination 4 KiB further on
    assert L.bitrev_rows(FAKE, FAKE + 4096, 10, 2, 4, None) == br.ERROR_ALIAS
    # absurd sizes are rejected rather than overflowing
    assert L.bitrev_rows(FAKE, FAKE, 40, 1 << 30, 16, None) == br.ERROR_INVALID_VALUE


def test_config_validation(L):
    for cfg in (br.Config(8, 0, 0, 0), br.Config(-1, 0, 0, 0), br.Config(0, -5, 0, 0),
                br.Config(0, 0, 4, 0), br.Config(0, 0, 0, 4), br.Config(0, 0, 0, -1),
                br.Config(0, 0, 0, 0, 3), br.Config(0, 0, 0, 0, 0, 5), br.Config(0, 0, 0, 0, 0, -1)):
        assert L.bitrev_inplace_ex(FAKE, 20, 8, ctypes.byref(cfg), None) == br.ERROR_INVALID_VALUE


def test_digit_config_validation(L):
    """The configurable digit-reversal entries reject a config field out of
    range before any HIP call, in and out of place."""
    for cfg in (br.Config(8, 0, 0, 0), br.Config(0, -5, 0, 0), br.Config(0, 0, 4, 0),
                br.Config(0, 0, 0, 0, 3), br.Config(0, 0, 0, 0, 0, 5)):
        assert L.bitrev_digitrev_inplace_ex(FAKE, 20, 2, 8, ctypes.byref(cfg), None) == \
            br.ERROR_INVALID_VALUE
        assert L.bitrev_digitrev_outofplace_ex(FAKE, FAKE + (1 << 30), 20, 2, 8,
                                               ctypes.byref(cfg), None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_digitrev_outofplace_ex(FAKE, FAKE, 20, 2, 8, None, None) == br.ERROR_ALIAS
    assert L.bitrev_digitrev_inplace_ex(FAKE, 21, 2, 8, None, None) == br.ERROR_INVALID_VALUE


def test_batched_validation(L):
    ws = br.bitrev_batched_workspace_size(4096)
    assert ws >= (4096 + 3) * 8 and ws % 256 == 0
    assert br.bitrev_batched_workspace_size(-1) == 0
    args = dict(data=FAKE, elems=1 << 20, off=FAKE, l2=FAKE, num=4096, s=8, ws=FAKE, wsb=ws)

    def call(**kw):
        a = dict(args, **kw)
        return L.bitrev_batched(a["data"], a["elems"], a["off"], a["l2"], a["num"], a["s"],
                                a["ws"], a["wsb"], None)

    assert call(num=0) == br.SUCCESS
    assert call(num=-1) == br.ERROR_INVALID_VALUE
    assert call(data=None) == br.ERROR_INVALID_VALUE
    assert call(off=None) == br.ERROR_INVALID_VALUE
    assert call(l2=None) == br.ERROR_INVALID_VALUE
    assert call(s=12) == br.ERROR_INVALID_VALUE
    assert call(elems=-1) == br.ERROR_INVALID_VALUE
    assert call(off=FAKE + 4) == br.ERROR_INVALID_VALUE
    assert call(data=FAKE + 4) == br.ERROR_INVALID_VALUE
    assert call(ws=None) == br.ERROR_WORKSPACE
    assert call(ws=FAKE + 4) == br.ERROR_WORKSPACE
    assert call(wsb=ws - 1) == br.ERROR_WORKSPACE


def test_recursive_levels_validation(L):
    f = L.bitrev_inplace_recursive_ex
    assert f(FAKE, 20, 8, 3, None) == br.ERROR_INVALID_VALUE
    assert f(FAKE, 20, 8, -1, None) == br.ERROR_INVALID_VALUE
    assert f(None, 20, 8, 0, None) == br.ERROR_INVALID_VALUE
    assert f(FAKE, 21, 8, 0, None) == br.ERROR_NOT_SUPPORTED      # odd k
    assert f(FAKE, 22, 8, 2, None) == br.ERROR_NOT_SUPPORTED      # k/2 odd
    assert f(FAKE, 28, 8, 2, None) == br.ERROR_NOT_SUPPORTED      # 2^14 x 8 B > 64 KiB
    assert f(FAKE, 0, 8, 2, None) == br.SUCCESS                   # n = 1: nothing to do


def test_copy_tiled_validation(L):
    assert L.bitrev_copy_tiled(None, FAKE, 10, 4, None, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy_tiled(FAKE, None, 10, 4, None, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy_tiled(FAKE, FAKE + (1 << 16), 10, 3, None, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy_tiled(FAKE, FAKE + (1 << 16), 41, 4, None, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy_tiled(FAKE, FAKE + (1 << 16), -1, 4, None, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy_tiled(FAKE + 2, FAKE + (1 << 16), 10, 4, None, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy_tiled(FAKE, FAKE + 64, 10, 4, None, None) == br.ERROR_ALIAS
    cfg = br.Config(0, 0, 4, 0, 0, 0)
    assert L.bitrev_copy_tiled(FAKE, FAKE + (1 << 16), 10, 4, ctypes.byref(cfg),
                               None) == br.ERROR_INVALID_VALUE


def test_batched_noalloc_validation(L):
    """The allocation-free batched call checks its arguments, and its array
    limit, on the host before any HIP call."""
    lim = br.NOALLOC_MAX_ARRAYS
    assert lim == 65536

    def call(data=FAKE, elems=1 << 20, off=FAKE, l2=FAKE, num=4096, s=8):
        return L.bitrev_batched_noalloc(data, elems, off, l2, num, s, None)

    assert call(num=0) == br.SUCCESS
    assert call(num=lim + 1) == br.ERROR_WORKSPACE
    assert call(num=1 << 30) == br.ERROR_WORKSPACE
    assert call(num=-1) == br.ERROR_INVALID_VALUE
    assert call(data=None) == br.ERROR_INVALID_VALUE
    assert call(off=None) == br.ERROR_INVALID_VALUE
    assert call(l2=None) == br.ERROR_INVALID_VALUE
    assert call(s=12) == br.ERROR_INVALID_VALUE
    assert call(elems=-1) == br.ERROR_INVALID_VALUE
    assert call(off=FAKE + 4) == br.ERROR_INVALID_VALUE
    assert call(l2=FAKE + 2) == br.ERROR_INVALID_VALUE
    assert call(data=FAKE + 4) == br.ERROR_INVALID_VALUE


def test_timed_entry_validation(L):
    """The timed entry points need both events (checked before any HIP call)."""
    assert L.bitrev_inplace_timed(FAKE, 20, 8, None, None, FAKE, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_inplace_timed(FAKE, 20, 8, None, FAKE, None, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_outofplace_timed(FAKE, FAKE + (8 << 20), 20, 8, None, None, None,
                                     None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_inplace_timed(None, 20, 8, None, FAKE, FAKE, None) == br.ERROR_INVALID_VALUE
    # timing events: NULL arguments are refused before any HIP call
    ms = ctypes.c_float()
    assert L.bitrev_timing_event_create(None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_timing_event_destroy(None) == br.SUCCESS
    assert L.bitrev_timing_elapsed_ms(None, FAKE, ctypes.byref(ms)) == br.ERROR_INVALID_VALUE
    assert L.bitrev_timing_elapsed_ms(FAKE, None, ctypes.byref(ms)) == br.ERROR_INVALID_VALUE
    assert L.bitrev_timing_elapsed_ms(FAKE, FAKE, None) == br.ERROR_INVALID_VALUE


def test_copy_validation(L):
    assert L.bitrev_copy_ex(FAKE, FAKE + 64, 16, 5, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy_ex(FAKE, FAKE + 64, 16, -1, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy(FAKE, FAKE + 8, 16, None) == br.ERROR_ALIAS
    assert L.bitrev_copy(None, FAKE, 16, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_copy(FAKE, FAKE + 64, 0, None) == br.SUCCESS


def test_plan_query_defaults(L):
    p = br.bitrev_plan_query(24, 8, tile_bits=5, variant=br.VARIANT_ONE_ITEM)
    assert p["path"] == br.PATH_TILE and p["tile_bits"] == 5 and p["mid_bits"] == 14
    assert p["work_items"] == (2**14 + 2**7) // 2
    assert p["grid_blocks"] % 8 == 0 and p["grid_blocks"] >= p["work_items"]
    # built-in plans measured on MI355X: complex64 in place at 128 MiB -> b = 5,
    # natural order, write-through stores; elsewhere b = 6, grouped order;
    # one item per workgroup, dispatch order
    p = br.bitrev_plan_query(24, 8)
    assert (p["tile_bits"], p["variant"], p["order"], p["xcd_remap"]) == (5, 1, 1, 2)
    assert p["cache_hints"] == br.HINTS_STREAM_WRITE_THROUGH
    for k in (23, 25):
        p = br.bitrev_plan_query(k, 8)
        assert (p["tile_bits"], p["variant"], p["order"], p["xcd_remap"]) == (6, 1, 3, 2)
        assert p["cache_hints"] == br.HINTS_STREAM_WRITE_THROUGH
    p = br.bitrev_plan_query(28, 8)
    assert (p["tile_bits"], p["variant"], p["order"], p["xcd_remap"]) == (6, 1, 3, 2)
    assert p["cache_hints"] == br.HINTS_STREAM_WRITE_THROUGH
    assert br.bitrev_plan_query(24, 8, cache_hints=br.HINTS_PLAIN)["cache_hints"] == 1
    assert br.bitrev_plan_query(24, 8, mode=br.MODE_OUTOFPLACE)["cache_hints"] == 4
    assert br.bitrev_plan_query(20, 8)["cache_hints"] == 1  # small arrays: plain
    # 1- and 2-byte elements beyond the Infinity Cache, and float32 out of
    # place at 256 MiB, keep streaming loads alone
    assert br.bitrev_plan_query(29, 1)["cache_hints"] == br.HINTS_STREAM_LOADS
    assert br.bitrev_plan_query(28, 2, mode=br.MODE_OUTOFPLACE)["cache_hints"] == 2
    assert br.bitrev_plan_query(26, 4, mode=br.MODE_OUTOFPLACE)["cache_hints"] == 2
    assert br.bitrev_plan_query(26, 4)["cache_hints"] == 4
    assert br.bitrev_plan_query(27, 1)["cache_hints"] == 4
    p = br.bitrev_plan_query(24, 8, mode=br.MODE_OUTOFPLACE)
    assert (p["tile_bits"], p["variant"], p["order"], p["xcd_remap"]) == (5, 1, 2, 1)
    assert p["work_items"] == 2**14
    # up to 32 MiB: persistent pipelined, dispatch order
    p = br.bitrev_plan_query(22, 8)
    assert (p["tile_bits"], p["variant"], p["order"], p["xcd_remap"]) == (5, 2, 1, 2)
    p = br.bitrev_plan_query(0, 8, mode=br.MODE_BATCHED)
    assert (p["tile_bits"], p["order"], p["xcd_remap"]) == (6, 1, 1)
    p = br.bitrev_plan_query(5, 4)
    assert p["path"] == br.PATH_WAVE
    p = br.bitrev_plan_query(1, 4)
    assert p["path"] == br.PATH_NONE
    p = br.bitrev_plan_query(9, 8)  # small k: b shrinks to floor(k/2)
    assert p["path"] == br.PATH_TILE and p["tile_bits"] == 4 and p["mid_bits"] == 1
    p = br.bitrev_plan_query(16, 4, rows=256, mode=br.MODE_OUTOFPLACE)
    assert p["work_items"] == 256 * 2 ** (16 - 2 * p["tile_bits"])
    for b in (4, 5, 6):
        p = br.bitrev_plan_query(24, 8, tile_bits=b)
        assert p["tile_bits"] == b and p["mid_bits"] == 24 - 2 * b
    with pytest.raises(br.BitrevError):
        br.bitrev_plan_query(24, 8, tile_bits=7)  # not compiled for 8-byte elements
    with pytest.raises(br.BitrevError):
        br.bitrev_plan_query(8, 8, tile_bits=5)  # 2b > k
    p = br.bitrev_plan_query(0, 8, mode=br.MODE_BATCHED)
    assert p["path"] == br.PATH_BATCHED and p["grid_blocks"] % 8 == 0
    # the persistent pipelined variant launches at most the resident workgroups
    p = br.bitrev_plan_query(24, 8, variant=br.VARIANT_PIPELINED)
    assert p["variant"] == br.VARIANT_PIPELINED and p["grid_blocks"] % 8 == 0
    assert 256 <= p["grid_blocks"] <= min(p["work_items"] + 7, 256 * 32)
    p = br.bitrev_plan_query(24, 8, variant=br.VARIANT_ONE_ITEM)
    assert p["variant"] == br.VARIANT_ONE_ITEM and p["grid_blocks"] >= p["work_items"]
    # register-staged: half the threads and one LDS tile; out of place it is one-item
    q = br.bitrev_plan_query(24, 8, variant=br.VARIANT_REGISTER_STAGED)
    assert q["variant"] == 3 and q["block_threads"] == p["block_threads"] // 2
    assert q["lds_bytes"] * 2 == p["lds_bytes"]
    q = br.bitrev_plan_query(24, 8, mode=br.MODE_OUTOFPLACE, variant=br.VARIANT_REGISTER_STAGED)
    assert q["variant"] == br.VARIANT_ONE_ITEM


def test_rows_plan_class_is_the_launch_footprint(L):
    """A launch of many short rows takes the plan class of its whole
    footprint: 256 rows of 2^16 float32 (64 MiB) get the one-item kernel with
    write-through stores, one such row (256 KiB) the small-array class."""
    many = br.bitrev_plan_query(16, 4, rows=256, mode=br.MODE_OUTOFPLACE)
    assert (many["variant"], many["order"], many["cache_hints"]) == (1, 1, 4)
    assert many["work_items"] == 256 * 2**4
    one = br.bitrev_plan_query(16, 4, rows=1, mode=br.MODE_OUTOFPLACE)
    assert (one["variant"], one["cache_hints"]) == (2, 1)


def test_tuning_file(L, tmp_path):
    good = tmp_path / "tune.txt"
    good.write_text("# comment\n\ninplace 8 24 4 0 2 1 2   # trailing comment\n"
                    "batched 8 -1 4 4 1 0 0\n")
    br.bitrev_load_tuning(str(good))
    try:
        p = br.bitrev_plan_query(24, 8)
        assert (p["tile_bits"], p["order"], p["variant"], p["xcd_remap"]) == (4, 2, 1, 2)
        assert br.bitrev_plan_query(25, 8)["tile_bits"] == 6  # no entry: default
        assert br.bitrev_plan_query(24, 8)["cache_hints"] == 4  # 8 fields: default hint
        p = br.bitrev_plan_query(0, 8, mode=br.MODE_BATCHED)
        assert p["tile_bits"] == 4 and p["order"] == 1 and p["grid_blocks"] == 4 * 256
        for bad in ("inplace 8 24 6 0 2 0\n", "sideways 8 24 6 0 2 0 0\n",
                    "inplace 3 24 6 0 2 0 0\n", "inplace 8 24 9 0 2 0 0\n",
                    "inplace 8 24 6 0 2 4 0\n", "inplace 8 24 6 0 2 0 3\n",
                    "inplace 8 24 6 0 2 0 0 7\n", "inplace 8 24 6 0 2 0 0 1 1\n",
                    "inplace 8 24 6 0 4 0 0\n"):
            f = tmp_path / "bad.txt"
            f.write_text(bad)
            with pytest.raises(br.BitrevError):
                br.bitrev_load_tuning(str(f))
            # a rejected file leaves the loaded table in place
            assert br.bitrev_plan_query(24, 8)["tile_bits"] == 4
        with pytest.raises(br.BitrevError):
            br.bitrev_load_tuning(str(tmp_path / "missing.txt"))
        v2 = tmp_path / "tune_v2.txt"
        v2.write_text("outofplace 4 26 7 0 3 1 1 2\n")
        br.bitrev_load_tuning(str(v2))
        p = br.bitrev_plan_query(26, 4, mode=br.MODE_OUTOFPLACE)
        assert (p["tile_bits"], p["order"], p["variant"], p["xcd_remap"], p["cache_hints"]) == \
            (7, 3, 1, 1, 2)
    finally:
        br.bitrev_load_tuning(None)
    assert br.bitrev_plan_query(24, 8)["tile_bits"] == 5
    assert "tuning" in br.bitrev_tuning_format()


def test_kernel_rev_matches_oracle(L):
    rng = np.random.default_rng(21)
    for j in range(0, 33):
        for v in list(rng.integers(0, 2**32, size=64, dtype=np.uint64)) + [0, 2**32 - 1]:
            v = int(v) & ((1 << j) - 1) if j < 32 else int(v)
            assert L.bitrev_debug_rev(v, j) == oracle.rev(v, j), (v, j)


@pytest.mark.parametrize("m", list(range(0, 17)))
@pytest.mark.parametrize("balanced", [0, 1])
def test_pair_enumeration_is_a_bijection(L, m, balanced):
    """The kernels' work items cover every tile pair {y, rev(y)} exactly once:
    the enumeration hits each y with y <= rev_m(y) once and nothing else."""
    count = L.bitrev_debug_pair_count(m)
    assert count == (2**m + 2 ** ((m + 1) // 2)) // 2
    ys = np.array([L.bitrev_debug_pair_at(m, w, balanced) for w in range(count)], dtype=np.int64)
    assert len(np.unique(ys)) == count
    revs = oracle.rev_table(m)
    assert np.all(ys < 2**m)
    assert np.all(ys <= revs[ys])
    assert count == int(np.count_nonzero(np.arange(2**m) <= revs))
    assert L.bitrev_debug_pair_at(m, count, balanced) == 0xFFFFFFFF


@pytest.mark.parametrize("m", list(range(0, 15)))
@pytest.mark.parametrize("order", [1, 2, 3])
def test_inplace_order_covers_every_pair_once(L, m, order):
    """Every order of the in-place work items (natural, balanced, grouped)
    names each tile pair {y, rev_m(y)} exactly once."""
    count = L.bitrev_debug_pair_count(m)
    revs = oracle.rev_table(m)
    ys = np.array([L.bitrev_debug_inplace_pair_at(m, w, order) for w in range(count)],
                  dtype=np.int64)
    assert np.all(ys < 2**m)
    lo = np.minimum(ys, revs[ys])
    assert len(np.unique(lo)) == count
    assert L.bitrev_debug_inplace_pair_at(m, count, order) == 0xFFFFFFFF


@pytest.mark.parametrize("m", list(range(0, 15)) + [20])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_outofplace_order_is_a_bijection(L, m, order):
    """Every out-of-place order visits each source tile of [0, 2^m) once."""
    ys = np.array([L.bitrev_debug_oop_tile_at(m, w, order) for w in range(2**m)],
                  dtype=np.int64)
    assert np.array_equal(np.sort(ys), np.arange(2**m))
    if m < 32:
        assert L.bitrev_debug_oop_tile_at(m, 2**m, order) == 0xFFFFFFFF


def test_grouped_order_runs_of_neighbouring_tiles(L):
    """The grouped order's first 4^j items (j = 3) touch 2^j runs of 2^j
    neighbouring tiles on each side of the swap."""
    m = 12
    ys = np.array([L.bitrev_debug_inplace_pair_at(m, w, 3) for w in range(64)], dtype=np.int64)
    rs = oracle.rev_table(m)[ys]
    for side in (ys, rs):
        starts = np.unique(side >> 3)
        assert len(starts) == 8
        assert np.all(np.sort(side).reshape(8, 8) - (np.sort(side).reshape(8, 8)[:, :1])
                      == np.arange(8))


@pytest.mark.parametrize("m", [20, 27, 32])
def test_pair_enumeration_large_m_sampled(L, m):
    rng = np.random.default_rng(m)
    count = L.bitrev_debug_pair_count(m)
    for w in list(rng.integers(0, count, size=2000)) + [0, count - 1]:
        for bal in (0, 1):
            y = L.bitrev_debug_pair_at(m, int(w), bal)
            assert y < 2**m and y <= oracle.rev(y, m)


@pytest.mark.parametrize("width", list(range(0, 15)) + [31, 32])
def test_spread_is_a_bijection(L, width):
    if width <= 14:
        vals = [L.bitrev_debug_spread(w, width) for w in range(1 << width)]
        assert sorted(vals) == list(range(1 << width))
    # the dealing order: bit 2t -> t, bit 2t+1 -> width-1-t
    for t in range(width):
        want = (t // 2) if t % 2 == 0 else (width - 1 - t // 2)
        assert L.bitrev_debug_spread(1 << t, width) == 1 << want, (width, t)


def test_recursive_and_transpose_validation(L):
    assert L.bitrev_inplace_recursive(FAKE, 23, 8, None) == br.ERROR_NOT_SUPPORTED
    assert L.bitrev_inplace_recursive(None, 24, 8, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_inplace_recursive(FAKE, 24, 12, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_inplace_recursive(FAKE + 4, 24, 8, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_inplace_recursive(FAKE, 0, 8, None) == br.SUCCESS
    assert L.bitrev_transpose_inplace(FAKE, 21, 8, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_transpose_inplace(FAKE, -1, 8, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_transpose_inplace(None, 4, 8, None) == br.ERROR_INVALID_VALUE


def test_triangular_tile_pairs(L):
    """The transpose kernel's tile pairs cover r <= c exactly once, in order,
    including indices large enough to stress the square-root estimate."""
    r, c = ctypes.c_uint32(), ctypes.c_uint32()
    w = 0
    for cc in range(0, 300):
        for rr in range(0, cc + 1):
            L.bitrev_debug_tri_pair(w, ctypes.byref(r), ctypes.byref(c))
            assert (r.value, c.value) == (rr, cc), w
            w += 1
    for cc in (2**15 - 1, 2**16 - 1, 2**19 - 3, 2**20 - 1):
        base = cc * (cc + 1) // 2
        for rr in (0, 1, cc // 2, cc):
            L.bitrev_debug_tri_pair(base + rr, ctypes.byref(r), ctypes.byref(c))
            assert (r.value, c.value) == (rr, cc)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_digit_pair_enumeration(L, d):
    """Digit-reversal work items cover each pair {y, drev(y)} exactly once."""
    for m in range(0, 19, d):
        count = L.bitrev_debug_digit_pair_count(m, d)
        ys = [L.bitrev_debug_digit_pair_at(m, w, d) for w in range(count)]
        dr = [oracle.digit_rev(y, m, d) for y in ys]
        assert len(set(ys)) == count, (m, d)
        assert all(y < 2**m and y <= r for y, r in zip(ys, dr)), (m, d)
        brute = sum(1 for y in range(2**m) if y <= oracle.digit_rev(y, m, d))
        assert count == brute, (m, d)
        for v in (0, 1, 5, 2**m - 1, 12345 % (2**m) if m else 0):
            assert L.bitrev_debug_digit_rev(v, m, d) == oracle.digit_rev(v, m, d)


@pytest.mark.parametrize("d", [2, 3])
def test_digit_inplace_order_covers_every_pair_once(L, d):
    """The in-place digit kernels' grouped order names each pair
    {y, drev(y)} exactly once, for every middle width."""
    for m in range(0, 19, d):
        count = L.bitrev_debug_digit_pair_count(m, d)
        ys = np.array([L.bitrev_debug_digit_inplace_pair_at(m, w, d) for w in range(count)],
                      dtype=np.int64)
        dr = np.array([oracle.digit_rev(int(y), m, d) for y in ys], dtype=np.int64)
        assert np.all(ys < 2**m), (m, d)
        assert len(np.unique(np.minimum(ys, dr))) == count, (m, d)
        assert L.bitrev_debug_digit_inplace_pair_at(m, count, d) == 0xFFFFFFFF


def test_digitrev_validation(L):
    assert L.bitrev_digitrev_inplace(FAKE, 25, 2, 8, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_digitrev_inplace(FAKE, 24, 4, 8, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_digitrev_inplace(FAKE, 24, 0, 8, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_digitrev_outofplace(FAKE, FAKE, 24, 2, 8, None) == br.ERROR_ALIAS
    assert L.bitrev_digitrev_inplace(FAKE, 3, 3, 8, None) == br.SUCCESS  # one digit


def test_variant_entry_validation(L):
    # strided rows: strides below the row length, unequal strides in place, overlap
    assert L.bitrev_rows_strided(FAKE, FAKE + (1 << 20), 10, 4, 512, 1024, 4, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_rows_strided(FAKE, FAKE, 10, 4, 2048, 1024, 4, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_rows_strided(FAKE, FAKE + 4096, 10, 4, 2048, 2048, 4, None) == br.ERROR_ALIAS
    assert L.bitrev_rows_strided(FAKE, FAKE + 4096, 10, 0, 2048, 2048, 4, None) == br.SUCCESS
    # even-odd: n >= 2, out of place only
    assert L.bitrev_evenodd(FAKE, FAKE + (1 << 20), 0, 1, 4, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_evenodd(FAKE, FAKE, 4, 1, 4, None) == br.ERROR_ALIAS
    assert L.bitrev_evenodd(FAKE, FAKE + 8, 4, 1, 4, None) == br.ERROR_ALIAS
    assert L.bitrev_evenodd(FAKE, FAKE + 64, 4, 0, 4, None) == br.SUCCESS
    # batched out of place: overlap, null source
    ws = br.bitrev_batched_workspace_size(4)
    assert L.bitrev_batched_outofplace(FAKE, FAKE + 64, 1024, FAKE, FAKE, 4, 8, FAKE, ws, None) == br.ERROR_ALIAS
    assert L.bitrev_batched_outofplace(None, FAKE, 1024, FAKE, FAKE, 4, 8, FAKE, ws, None) == br.ERROR_INVALID_VALUE
    assert L.bitrev_batched_outofplace(FAKE, FAKE + (1 << 20), 1024, FAKE, FAKE, 4, 8, FAKE, 8, None) == br.ERROR_WORKSPACE


def test_kernel_resource_remarks():
    """The build reads hipcc's per-kernel resource remarks and refuses any
    kernel that spills to scratch memory; the recorded figures of the last
    build keep every kernel in registers and LDS."""
    from paper_1708_01873_amd import build as bld
    text = "\n".join([
        "x.inl:1:1: remark: Function Name: kern_a [-Rpass-analysis=kernel-resource-usage]",
        "x.inl:1:1: remark:     VGPRs: 46 [-Rpass-analysis=kernel-resource-usage]",
        "x.inl:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.inl:1:1: remark:     Occupancy [waves/SIMD]: 8 [-Rpass-analysis=kernel-resource-usage]",
        "x.inl:1:1: remark:     LDS Size [bytes/block]: 66560 [-Rpass-analysis=kernel-resource-usage]",
        "x.inl:2:1: remark: Function Name: kern_b [-Rpass-analysis=kernel-resource-usage]",
        "x.inl:2:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]",
    ])
    ks = bld.parse_resources(text)
    assert ks == [{"name": "kern_a", "VGPRs": 46, "ScratchSize": 0, "Occupancy": 8,
                   "LDS Size": 66560},
                  {"name": "kern_b", "ScratchSize": 16}]
    if not os.path.exists(bld.RESOURCES):
        pytest.skip("no build record")
    rows = [ln.split() for ln in open(bld.RESOURCES) if not ln.startswith("#")]
    assert len(rows) > 100
    assert all(r[3] == "0" for r in rows), [r[0] for r in rows if r[3] != "0"]
    # the in-place complex64 tile kernel at b = 6: two 1024-thread
    # workgroups per CU need at most 64 VGPRs
    head = [r for r in rows if "k_tile_inplaceILi8ELi6ELb1E" in r[0]]
    assert head and all(int(r[1]) <= 64 for r in head)
