"""Autotuner for libbitrev.

The tile width b is the method's one machine-dependent parameter: the paper
notes that the buffered method's buffer size t = 2^(2b) has to be tuned per
architecture (Introduction, matrix buffer; Results, where the buffer size was
optimised per problem size).  On MI355X the kernel variant (one work item per
workgroup, persistent and software-pipelined, or register-staged), the
work-item order, the cache hints of the global accesses and,
for the batched launch, the workgroups per compute unit matter as well.

``tune_plain`` and ``tune_batched`` time every candidate with HIP events on
the launch stream and return the ranking; ``write_tuning`` writes the best
plans as plan-table rows keyed by this device (gcnArchName and compute-unit
count) and by size class, the form ``bitrev_load_tuning`` reads
(``bitrev_tuning_format()`` describes it); ``autotune`` does all three and
loads the result.  ``tune_table`` sweeps every element size over a range of
size classes and writes a whole table in the built-in table's format
(``csrc/plans_<arch>.inc`` holds the shipped one): rows tuned on one device
or partition mode do not apply on another.  In-place candidates run an
even number of times, so the caller's data ends as it started (the
permutation is an involution).  Tune before capturing a graph: a captured
launch keeps the plan it was captured with.

Command line: ``python -m paper_1708_01873_amd.tune --out FILE`` tunes the
in-place and out-of-place plans for a few sizes and the batched plan for an
uneven complex64 batch, then writes FILE; ``--table FILE`` sweeps the size
classes instead and writes a full plan table.
"""
from __future__ import annotations

import argparse
import os
import statistics
from dataclasses import dataclass, field

import torch

from . import (MODE_BATCHED, MODE_INPLACE, MODE_OUTOFPLACE, BitrevError, bitrev_batched,
               bitrev_batched_workspace_size, bitrev_inplace, bitrev_load_tuning,
               bitrev_outofplace, bitrev_plan_query)

MAX_TILE_BITS = {1: 7, 2: 7, 4: 7, 8: 6, 16: 6}
MODE_NAMES = {MODE_INPLACE: "inplace", MODE_OUTOFPLACE: "outofplace", MODE_BATCHED: "batched"}
ROW_HEADER = ("# arch cus kind elem_size digit_bits tile_match class_min class_max   "
              "tile_bits wg_per_cu order variant xcd_remap cache_hints")


def device_key(device=0) -> tuple[str, int]:
    """(gcnArchName without its feature suffix, compute units) of a device:
    the key of the plan-table rows tuned on it."""
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "") or props.name
    return arch.split(":")[0], props.multi_processor_count


def size_class(nbytes: int) -> int:
    """floor(log2(bytes)): the size class a launch of nbytes is planned by."""
    return int(nbytes).bit_length() - 1
_DTYPES = {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64, 16: torch.complex128}


@dataclass
class Candidate:
    tile_bits: int
    order: int
    variant: int = 0
    wg_per_cu: int = 0
    xcd_remap: int = 0
    cache_hints: int = 0
    ms: float = float("inf")

    def row(self, arch: str, cus: int, kind: str, elem_size: int, cmin: int, cmax: int) -> str:
        """This plan as a plan-table row for one device and size-class range."""
        return "%s %d %s %d 0 0 %d %d   %d %d %d %d %d %d" % (
            arch, cus, kind, elem_size, cmin, cmax, self.tile_bits, self.wg_per_cu, self.order,
            self.variant, self.xcd_remap, self.cache_hints)

    def config(self) -> dict:
        return dict(tile_bits=self.tile_bits, order=self.order, variant=self.variant,
                    xcd_remap=self.xcd_remap, cache_hints=self.cache_hints)


@dataclass
class TuneResult:
    mode: int
    elem_size: int
    log2n: int
    best: Candidate
    ranking: list = field(default_factory=list)
    default_ms: float = float("nan")
    rows: int = 1

    @property
    def gain_over_default(self) -> float:
        return self.default_ms / self.best.ms


class _Clock:
    """Median of per-call HIP-event times, optionally evicting the caches with
    a read of a scratch buffer before each call (outside the timed span)."""

    def __init__(self, device, flush_bytes: int):
        self.scratch = None
        if flush_bytes:
            # float32: its sum is a single read-only reduction kernel
            self.scratch = torch.ones(flush_bytes // 4, dtype=torch.float32, device=device)

    def median_ms(self, fn, reps: int) -> float:
        fn()
        fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(reps):
            if self.scratch is not None:
                self.scratch.sum()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            evs.append((a, b))
        torch.cuda.synchronize()
        return statistics.median(a.elapsed_time(b) for a, b in evs)


def _even(reps: int) -> int:
    return reps + (reps & 1)


def plain_candidates(log2n: int, elem_size: int, mode: int) -> list[Candidate]:
    out = []
    for b in range(1, MAX_TILE_BITS[elem_size] + 1):
        if 2 * b > log2n or (elem_size << b) < 16:
            continue
        for order in (1, 2, 3):
            # variant 3 (register-staged) exists in place only
            for variant in ((1, 2, 3) if mode == MODE_INPLACE else (1, 2)):
                for xcd in (1, 2):
                    # cache hints apply to the one-item and register-staged kernels
                    for hints in ((1, 2, 3, 4) if variant != 2 else (0,)):
                        out.append(Candidate(b, order, variant, 0, xcd, hints))
    return out


def tune_plain(log2n: int, elem_size: int, mode: int = MODE_INPLACE, *, rows: int = 1,
               reps: int = 10, flush: bool = True, device="cuda",
               candidates: list[Candidate] | None = None) -> TuneResult:
    """Time every candidate plan for `rows` arrays of 2^log2n elements of
    elem_size bytes (in place or out of place) on scratch buffers."""
    n = rows << log2n
    x = torch.empty(n, dtype=_DTYPES[elem_size], device=device)
    x.view(torch.uint8).random_(0, 256)
    y = torch.empty_like(x) if mode == MODE_OUTOFPLACE else None
    array_bytes = n * elem_size
    clock = _Clock(device, (1 << 30) if flush and array_bytes <= (1 << 30) else 0)
    reps = _even(reps)

    def run(**cfg):
        if mode == MODE_INPLACE:
            if rows == 1:
                bitrev_inplace(x, log2n, **cfg)
            else:
                from . import bitrev_rows
                bitrev_rows(x, x, log2n, **cfg)
        else:
            if rows == 1:
                bitrev_outofplace(x, y, log2n, **cfg)
            else:
                from . import bitrev_rows
                bitrev_rows(x, y, log2n, **cfg)

    ranking = []
    for c in candidates or plain_candidates(log2n, elem_size, mode):
        try:
            c.ms = clock.median_ms(lambda: run(**c.config()), reps)
        except BitrevError:
            continue
        ranking.append(c)
    if not ranking:
        raise RuntimeError("no candidate plan ran for log2n=%d elem_size=%d" % (log2n, elem_size))
    ranking.sort(key=lambda c: c.ms)
    default_ms = clock.median_ms(lambda: run(), reps)
    return TuneResult(mode, elem_size, log2n, ranking[0], ranking, default_ms, rows)


def tune_batched(data, offsets, log2n, *, reps: int = 6, wg_per_cu=(0, 1, 2, 4, 8),
                 tile_bits=None, orders=(1, 2, 3), xcd_remaps=(1, 2)) -> TuneResult:
    """Time the batched launch on the caller's own batch (device tensors as
    for bitrev_batched) over tile widths, orders and workgroups per CU.  Each
    candidate runs an even number of times, so `data` ends unchanged."""
    s = data.element_size()
    num = log2n.numel()
    ws = torch.empty(max(1, bitrev_batched_workspace_size(num)), dtype=torch.uint8,
                     device=data.device)
    cus = torch.cuda.get_device_properties(data.device).multi_processor_count
    clock = _Clock(data.device, 0)
    reps = _even(reps)
    bs = tile_bits or [b for b in range(2, MAX_TILE_BITS[s] + 1) if (s << b) >= 16]
    ranking = []
    for b in bs:
        for order in orders:
            for w in wg_per_cu:
                for xcd in xcd_remaps:
                    c = Candidate(b, order, 0, w, xcd)
                    grid = w * cus if w else 0
                    try:
                        c.ms = clock.median_ms(lambda: bitrev_batched(
                            data, offsets, log2n, ws, tile_bits=b, order=order, grid_blocks=grid,
                            xcd_remap=xcd), reps)
                    except BitrevError:
                        continue
                    ranking.append(c)
    if not ranking:
        raise RuntimeError("no batched candidate ran")
    ranking.sort(key=lambda c: c.ms)
    default_ms = clock.median_ms(lambda: bitrev_batched(data, offsets, log2n, ws), reps)
    return TuneResult(MODE_BATCHED, s, -1, ranking[0], ranking, default_ms)


def result_row(r: TuneResult, arch: str, cus: int) -> str:
    """The best plan of a result as a plan-table row: keyed by the device, the
    kind of launch and the size class it was measured at (any class for the
    batched launch)."""
    if r.mode == MODE_BATCHED:
        return r.best.row(arch, cus, "batched", r.elem_size, -1, -1)
    c = size_class((r.elem_size << r.log2n) * r.rows)
    return r.best.row(arch, cus, MODE_NAMES[r.mode], r.elem_size, c, c)


def write_tuning(results: list[TuneResult], path: str, note: str = "") -> str:
    """Write the best plan of each result as plan-table rows for this device."""
    arch, cus = device_key()
    props = torch.cuda.get_device_properties(0)
    lines = ["# libbitrev plan rows tuned on %s (%s, %d compute units)%s"
             % (props.name, arch, cus, ("; " + note) if note else ""), ROW_HEADER]
    for r in results:
        lines.append("%s   # %.4f ms, %.3fx the built-in plan" % (
            result_row(r, arch, cus), r.best.ms, r.gain_over_default))
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def autotune(path: str, plain=((MODE_INPLACE, 8, 24), (MODE_OUTOFPLACE, 8, 24)), batch=None,
             reps: int = 10) -> list[TuneResult]:
    """Tune the listed (mode, elem_size, log2n) plans and, if `batch` =
    (data, offsets, log2n) is given, the batched plan; write and load the
    table.  Returns the results."""
    results = [tune_plain(k, s, mode, reps=reps) for mode, s, k in plain]
    if batch is not None:
        results.append(tune_batched(*batch, reps=max(2, reps // 2)))
    write_tuning(results, path)
    bitrev_load_tuning(path)
    return results


def tune_table(path: str, elem_sizes=(1, 2, 4, 8, 16), classes=range(22, 33), reps: int = 6,
               note: str = "") -> list[TuneResult]:
    """Sweep in-place and out-of-place plans for every element size over the
    size classes (arrays of 2^c bytes, as far as device memory allows) and
    write one plan-table row per (kind, element size, run of neighbouring
    classes with the same best plan) for this device, in the built-in
    table's row format."""
    arch, cus = device_key()
    free, _ = torch.cuda.mem_get_info()
    lines = ["# libbitrev plan table tuned on %s (%d compute units)%s"
             % (arch, cus, ("; " + note) if note else ""), ROW_HEADER]
    results = []
    for mode in (MODE_INPLACE, MODE_OUTOFPLACE):
        for s in elem_sizes:
            runs = []  # [plan, first class, last class, candidate]
            for c in classes:
                k = c - (s.bit_length() - 1)
                need = (1 << c) * (1 if mode == MODE_INPLACE else 2) + (1 << 30)
                if k < 14 or need > free:
                    continue
                r = tune_plain(k, s, mode, reps=reps)
                results.append(r)
                b = r.best
                key = (b.tile_bits, b.wg_per_cu, b.order, b.variant, b.xcd_remap, b.cache_hints)
                if runs and runs[-1][0] == key and runs[-1][2] == c - 1:
                    runs[-1][2] = c
                else:
                    runs.append([key, c, c, b])
            for _, lo, hi, b in runs:
                lines.append(b.row(arch, cus, MODE_NAMES[mode], s, lo, hi))
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return results


def default_cache_path() -> str:
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "gpu").split(":")[0]
    base = os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache"))
    return os.path.join(base, "libbitrev", "tuning_%s_%dcu.txt" % (arch, props.multi_processor_count))


def main() -> None:
    ap = argparse.ArgumentParser(description="tune libbitrev plans on this GPU")
    ap.add_argument("--out", default=None, help="tuning file to write (default: user cache)")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--sizes", default="8:24,8:28,4:24,16:24",
                    help="comma-separated elem_size:log2n pairs for the plain plans")
    ap.add_argument("--batch", action="store_true",
                    help="also tune the batched plan on 4096 uneven complex64 arrays")
    ap.add_argument("--table", default=None,
                    help="sweep every element size over the size classes 2^22 .. 2^32 bytes and "
                         "write a full plan table (the built-in table's row format) to this file")
    args = ap.parse_args()
    if args.table:
        results = tune_table(args.table, reps=args.reps)
        print("tuned %d (kind, element size, class) plans; wrote %s" % (len(results), args.table))
        return
    from . import workloads
    plain = []
    for tok in args.sizes.split(","):
        s, k = (int(v) for v in tok.split(":"))
        plain += [(MODE_INPLACE, s, k), (MODE_OUTOFPLACE, s, k)]
    batch = None
    if args.batch:
        offsets, l2 = workloads.batched_layout(4096, 8, 20, workloads.SEEDS["c4"])
        data = workloads.device_normal(int(offsets[-1]), workloads.SEEDS["c4"] + 1000,
                                       torch.complex64)
        batch = (data, torch.from_numpy(offsets).cuda(), torch.from_numpy(l2).cuda())
    path = args.out or default_cache_path()
    for r in autotune(path, plain, batch, reps=args.reps):
        print("%-10s s=%-2d k=%-3d best b=%d order=%d variant=%d xcd=%d hints=%d wg/cu=%d  "
              "%.4f ms  (%.3fx built-in)" % (MODE_NAMES[r.mode], r.elem_size, r.log2n,
                                             r.best.tile_bits, r.best.order, r.best.variant,
                                             r.best.xcd_remap, r.best.cache_hints,
                                             r.best.wg_per_cu, r.best.ms, r.gain_over_default))
    print("wrote", path)


if __name__ == "__main__":
    main()
