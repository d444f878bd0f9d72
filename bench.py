"""Benchmark of libbitrev on one MI355X.

A step is one in-place bit-reversed permutation of 2^24 complex64 elements
(128 MiB, real and imaginary parts N(0, 1) from seed 2), already resident in
HBM, with the library's default plan.  Between steps (outside the timed
interval) a kernel reads a 1 GiB scratch buffer, which evicts the array from
the L2 caches and the 256 MiB Infinity Cache, so every step starts from HBM.
The flush reads rather than writes: a written flush leaves up to 256 MiB of
dirty lines whose write-back would then be charged to the timed step.  HIP
events on the launch stream time each step.

Prints one JSON line: the effective bandwidth 2 n s / t (GB/s), the roofline
block of the tile kernel, the CPU oracle baseline, and context figures (copy
bandwidth under the same flush policy, out of place, the tile-width sweep,
the batched-vs-loop speedup on 4096 uneven arrays).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD specification
FLUSH_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tile_inplace_c64_2p24.txt")
KERNEL_SOURCES = ("paper_1708_01873_amd/csrc/bitrev_device.hpp",
                  "paper_1708_01873_amd/csrc/bitrev_kernels.inl")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


class Timer:
    """Per-call HIP-event timing on torch's current stream (the stream every
    library call here is launched on), with a cache flush between calls."""

    def __init__(self, torch, flush: bool):
        self.torch = torch
        self.flush = flush
        self.scratch = None
        if flush:
            # float32, so that sum() is one reduction kernel that only reads
            # (an integer sum would first widen the buffer into a written copy)
            self.scratch = torch.ones(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")

    def _flush(self):
        if self.scratch is not None:
            self.scratch.sum()

    def time(self, fn, reps: int, warmup: int = 1) -> list[float]:
        torch = self.torch
        for _ in range(warmup):
            self._flush()
            fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(reps):
            self._flush()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            evs.append((a, b))
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]  # ms


def gbs(nbytes: float, ms: float) -> float:
    return nbytes / (ms * 1e-3) / 1e9


def read_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the same kernel and the current kernel source."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    key, _, val = line.partition(":")
                    kv[key.strip()] = val.strip()
        if kv.get("kernel_source_hash") != kernel_source_hash():
            return None
        if kv.get("kernel", "").replace(" ", "") != kernel.replace(" ", ""):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def kernel_name(inplace: bool, s: int, plan: dict) -> str:
    """The tile kernel a default plan launches (its template arguments)."""
    b, hint = plan["tile_bits"], plan["cache_hints"] - 1
    if inplace:
        if plan["variant"] == 2:
            return "k_tile_inplace_pipe<%d,%d,true>" % (s, b)
        if plan["variant"] == 3:
            return "k_tile_inplace_rs<%d,%d,true,%d>" % (s, b, hint)
        return "k_tile_inplace<%d,%d,true,%d>" % (s, b, hint)
    if plan["variant"] == 2:
        return "k_tile_outofplace_pipe<%d,%d,true>" % (s, b)
    return "k_tile_outofplace<%d,%d,true,%d>" % (s, b, hint)


def roofline_block(nbytes: float, kms: float, kernel: str, traffic=None) -> dict:
    """The roofline object of one kernel: algorithmic bytes per launch over
    its mean duration, against the HBM peak."""
    return {"bound": "hbm", "achieved": round(gbs(nbytes, kms), 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs(nbytes, kms) / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": kernel, "algorithmic_bytes_per_launch": nbytes,
            "kernel_ms_mean": round(kms, 5)}


# The paper's reported figures for its own workload (complex<double>, k = 24),
# on its own hardware (Results; Table 2 gives the CPU's caches and clock).
# The paper prints seconds; GB/s here is 2 n s / t with s = 16 bytes.
PAPER_CONTEXT = {
    "what": "the paper's reported times for the bit-reversed permutation of 2^24 "
            "complex<double> (16-byte) elements, as context only: other hardware, and "
            "the GPU figure may include host-device copies",
    "workload": "complex128 n=2^24 (256 MiB); our figure: "
                "context.other_configs.complex128_2p24_paper_workload",
    "fastest_single_thread": {"seconds": 0.13, "GBps_derived": 4.1,
                              "hardware": "x86-64 CPU, 3.8 GHz, 15360K L3 (model not named), "
                                          "g++ 6.2.0 -Ofast -march=native"},
    "semi_recursive_openmp": {"seconds": 0.1, "GBps_derived": 5.4,
                              "hardware": "the same CPU, thread count not stated"},
    "semi_recursive_cuda": {"seconds": 0.08, "GBps_derived": 6.7,
                            "hardware": "an unnamed NVIDIA GPU, nvcc"},
    "naive_bitwise": {"seconds": 1.0, "GBps_derived": 0.54, "hardware": "the same CPU"},
}


TRAFFIC_ALL_FILE = os.path.join(ROOT, "profiles", "traffic_all_configs.txt")


def read_config_traffic(config: str):
    """HBM bytes per call of one configuration of bench.py --traffic-workload
    from the committed counter summary, if it was taken on the current
    kernel source."""
    try:
        with open(TRAFFIC_ALL_FILE) as f:
            text = f.read()
        if "kernel_source_hash: %s" % kernel_source_hash() not in text:
            return None
        for line in text.splitlines():
            parts = [p.strip() for p in line.split("|")]
            if len(parts) == 5 and parts[0] == config:
                return float(parts[2])
    except (OSError, ValueError):
        pass
    return None


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(host, target_s: float = 10.0, max_reps: int = 20):
    """The oracle's in-place permutation of the same array on one host core,
    repeated until about target_s seconds have run."""
    import numpy as np
    import oracle
    a = host.copy()
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.inplace(a)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= max_reps:
            break
    ok = np.array_equal(a.view(np.uint8), (host if reps % 2 == 0 else oracle.outofplace(host)).view(np.uint8))
    return reps, el, ok


def cpu_multicore(host, target_s: float = 5.0, max_reps: int = 40):
    """The oracle's out-of-place permutation of the same array with its index
    range split over the host's OpenMP threads, repeated until about target_s
    seconds have run: the CPU on all its cores, next to the one-core figure."""
    import numpy as np
    import oracle
    reps, threads, out = 0, 0, None
    t0 = time.perf_counter()
    while True:
        out, threads = oracle.outofplace_mt(host)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= max_reps:
            break
    ok = np.array_equal(out.view(np.uint8), oracle.outofplace(host).view(np.uint8))
    return reps, el, threads, ok


def batched_speedup(torch, br, reps: int):
    """4096 complex64 arrays, log2 n uniform in [8, 20] (seed 5): one replay
    of the captured batched launch vs an eager loop of per-array in-place
    calls, and that loop captured into a graph."""
    from paper_1708_01873_amd import workloads
    from paper_1708_01873_amd.graph import BatchedGraph
    seed = workloads.SEEDS["c4"]
    offsets, log2n = workloads.batched_layout(4096, 8, 20, seed)
    total = int(offsets[-1])
    x = workloads.device_normal(total, seed + 1000, torch.complex64)
    off = torch.from_numpy(offsets).cuda()
    l2 = torch.from_numpy(log2n).cuda()
    nbytes = 2.0 * total * 8
    # autotune the batched plan on this batch (before capture; even number of
    # runs per candidate, so the data is unchanged), then load the table
    import tempfile
    from paper_1708_01873_amd import tune
    t0 = time.perf_counter()
    tuned = tune.tune_batched(x, off, l2, reps=2)
    table = tune.write_tuning([tuned], os.path.join(tempfile.mkdtemp(), "batched_tuning.txt"))
    br.bitrev_load_tuning(table)
    tune_s = time.perf_counter() - t0
    g = BatchedGraph(x, off, l2)
    views = [x[int(offsets[a]):int(offsets[a + 1])] for a in range(4096)]
    ptrs = [(v.data_ptr(), int(log2n[a])) for a, v in enumerate(views)]
    lib = br.lib()
    stream = torch.cuda.current_stream().cuda_stream

    def loop():
        for p, k in ptrs:
            st = lib.bitrev_inplace(p, k, 8, stream)
            if st:
                raise br.BitrevError(st, "bitrev_inplace")

    loop_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(loop_graph):
        cap_stream = torch.cuda.current_stream().cuda_stream
        for p, k in ptrs:
            lib.bitrev_inplace(p, k, 8, cap_stream)
    timer = Timer(torch, flush=True)
    t_graph = timer.time(g.replay, reps)
    t_loop = timer.time(loop, reps)
    t_loopg = timer.time(loop_graph.replay, reps)
    br.bitrev_load_tuning(None)
    med = statistics.median
    return {
        "workload": "4096 complex64 arrays, log2n uniform [8,20], seed 5",
        "elements": total,
        "plan": g.plan,
        "autotune": {"seconds": round(tune_s, 2), "best": {
            "tile_bits": tuned.best.tile_bits, "order": tuned.best.order,
            "wg_per_cu": tuned.best.wg_per_cu, "ms": tuned.best.ms},
            "candidates": len(tuned.ranking), "gain_over_builtin": round(tuned.gain_over_default, 3)},
        "graph_ms": med(t_graph),
        "graph_GBps": gbs(nbytes, med(t_graph)),
        "eager_loop_ms": med(t_loop),
        "eager_loop_GBps": gbs(nbytes, med(t_loop)),
        "loop_in_graph_ms": med(t_loopg),
        "speedup_vs_eager_loop": med(t_loop) / med(t_graph),
        "speedup_vs_loop_in_graph": med(t_loopg) / med(t_graph),
    }


# Where shifted copy destinations start inside their allocation: with the
# destination at the same offset as the source within their allocations, a
# linear copy's concurrent reads and writes meet the same memory channels;
# 1 MiB + 8 KiB or 17 MiB in, the 4 GiB copy ran up to 5% faster
# (write-through form; the best offset differed between array sizes).
COPY_SHIFTS = ((1 << 20) + 8192, 17 << 20)


def best_copy(torch, br, timer, x, y, reps: int) -> dict:
    """The fastest reference copy of x (the same bytes as the permutation)
    under the timer's flush policy: the linear streaming copy into y and into
    destinations shifted by COPY_SHIFTS, and the copy in the out-of-place
    tile kernels' order (the identity map, same reads and row shape as the
    permutation), each in its four cache-hint forms.  Returns the fastest
    mean step time and which copy gave it."""
    es = x.element_size()
    n = x.numel()
    shifted = torch.empty(n + max(COPY_SHIFTS) // es, dtype=x.dtype, device=x.device)
    forms = []
    for h in (1, 2, 3, 4):
        forms.append(("linear", h, lambda h=h: br.bitrev_copy(x, y, cache_hints=h)))
        for sh in COPY_SHIFTS:
            ys = shifted[sh // es: sh // es + n]
            forms.append(("linear, destination shifted %d KiB" % (sh >> 10), h,
                          lambda h=h, ys=ys: br.bitrev_copy(x, ys, cache_hints=h)))
        forms.append(("tile order", h, lambda h=h: br.bitrev_copy_tiled(x, y, cache_hints=h)))
    best = None
    for name, h, fn in forms:
        ms = statistics.fmean(timer.time(fn, reps))
        if best is None or ms < best["ms"]:
            best = {"ms": ms, "copy": name, "cache_hints": h}
    del shifted
    return best


def kernel_ms(br, timer, fn_timed, reps: int) -> float:
    """Mean duration of the one kernel a *_timed call launches (HIP events
    recorded by its own dispatch, system-scope fence off), the caches evicted
    before each launch."""
    evs = [(br.TimingEvent(), br.TimingEvent()) for _ in range(reps)]
    for a, b in evs:
        timer._flush()
        fn_timed(a, b)
    timer.torch.cuda.synchronize()
    ms = statistics.fmean(a.elapsed_time(b) for a, b in evs)
    for a, b in evs:
        a.destroy()
        b.destroy()
    return ms


def per_n_complex64(torch, br, timer, reps: int) -> dict:
    """Complex64 in place and out of place at n = 2^22 .. 2^29 (32 MiB to
    4 GiB), default plans, caches evicted before each call, next to the
    fastest reference copy of the same bytes.  Arrays up to 128 MiB can be
    held whole by the 256 MiB Infinity Cache together with what a step
    writes; from 512 MiB on no step fits it, so those rates are HBM-bound."""
    from paper_1708_01873_amd import workloads
    out = {}
    for k in range(22, 30):
        n = 1 << k
        x = workloads.device_normal(n, 100 + k, torch.complex64)
        y = torch.empty_like(x)
        nb = 2.0 * n * 8
        r = reps if k <= 26 else max(4, reps // 2)
        ip = statistics.fmean(timer.time(lambda: br.bitrev_inplace(x), r))
        oop = statistics.fmean(timer.time(lambda: br.bitrev_outofplace(x, y), r))
        ipk = kernel_ms(br, timer, lambda a, b: br.bitrev_inplace_timed(x, a, b), r)
        cp = best_copy(torch, br, timer, x, y, r)
        out["2^%d" % k] = {
            "array_MiB": (n * 8) >> 20,
            "cache_assisted": n * 8 <= (128 << 20),
            "inplace_GBps": round(gbs(nb, ip), 1),
            "inplace_kernel_GBps": round(gbs(nb, ipk), 1),
            "outofplace_GBps": round(gbs(nb, oop), 1),
            "copy_GBps": round(gbs(nb, cp["ms"]), 1),
            "copy_form": "%s, hints %d" % (cp["copy"], cp["cache_hints"]),
            "inplace_pct_of_copy": round(100.0 * cp["ms"] / ip, 1),
            "outofplace_pct_of_copy": round(100.0 * cp["ms"] / oop, 1),
            "inplace_pct_hbm_peak": round(100.0 * gbs(nb, ip) / HBM_PEAK_GBS, 1)}
        log("per-n complex64 2^%d: %s" % (k, json.dumps(out["2^%d" % k])))
        del x, y
        torch.cuda.empty_cache()
    return out


def other_configs(torch, br, timer, reps: int) -> dict:
    """The remaining configurations, timed like the headline (default plans,
    caches evicted before each call)."""
    from paper_1708_01873_amd import workloads
    from paper_1708_01873_amd.autograd import BitRev
    out = {}
    med = statistics.median
    # uint32, n = 2^10: launch-bound, reported in microseconds
    x = torch.from_numpy(workloads.uint32_uniform(10, workloads.SEEDS["c1"]).view("int32")).cuda()
    y = torch.empty_like(x)
    # (per call with its dispatch, and the kernel alone from its own events)
    out["uint32_2p10"] = {
        "inplace_us": round(1e3 * med(timer.time(lambda: br.bitrev_inplace(x), reps)), 2),
        "outofplace_us": round(1e3 * med(timer.time(lambda: br.bitrev_outofplace(x, y), reps)), 2),
        "inplace_kernel_us": round(1e3 * kernel_ms(
            br, timer, lambda a, b: br.bitrev_inplace_timed(x, a, b), reps), 2),
        "outofplace_kernel_us": round(1e3 * kernel_ms(
            br, timer, lambda a, b: br.bitrev_outofplace_timed(x, y, a, b), reps), 2)}
    # the two 4 GiB arrays: beyond every cache, so their kernels are the
    # HBM-bound rooflines (kernel time from each launch's own events)
    for name, k, dt, seed in (("complex128_2p28", 28, torch.complex128, workloads.SEEDS["c3a"]),
                              ("float32_2p30", 30, torch.float32, workloads.SEEDS["c3b"])):
        label = name.replace("_2p", " 2^")
        x = workloads.device_normal(1 << k, seed, dt)
        y = torch.empty_like(x)
        s = x.element_size()
        nb = 2.0 * x.numel() * s
        r = max(4, reps // 4)
        ip = statistics.fmean(timer.time(lambda: br.bitrev_inplace(x), r))
        oop = statistics.fmean(timer.time(lambda: br.bitrev_outofplace(x, y), r))
        ipk = kernel_ms(br, timer, lambda a, b: br.bitrev_inplace_timed(x, a, b), r)
        oopk = kernel_ms(br, timer, lambda a, b: br.bitrev_outofplace_timed(x, y, a, b), r)
        cp = best_copy(torch, br, timer, x, y, r)
        pip = br.bitrev_plan_query(k, s, mode=br.MODE_INPLACE)
        poop = br.bitrev_plan_query(k, s, mode=br.MODE_OUTOFPLACE)
        out[name] = {
            "inplace_GBps": round(gbs(nb, ip), 1),
            "outofplace_GBps": round(gbs(nb, oop), 1),
            "copy_GBps": round(gbs(nb, cp["ms"]), 1),
            "copy_form": "%s, hints %d" % (cp["copy"], cp["cache_hints"]),
            "inplace_pct_of_copy": round(100.0 * cp["ms"] / ip, 1),
            "outofplace_pct_of_copy": round(100.0 * cp["ms"] / oop, 1),
            "roofline_inplace": roofline_block(nb, ipk, kernel_name(True, s, pip),
                                               read_config_traffic("in place " + label)),
            "roofline_outofplace": roofline_block(nb, oopk, kernel_name(False, s, poop),
                                                  read_config_traffic("out of place " + label))}
        log("%s: %s" % (name, json.dumps(out[name])))
        del x, y
        torch.cuda.empty_cache()
    # the paper's own workload: complex128 (complex<double>), k = 24
    x = workloads.device_normal(1 << 24, 24, torch.complex128)
    y = torch.empty_like(x)
    nb = 2.0 * x.numel() * 16
    ip = statistics.fmean(timer.time(lambda: br.bitrev_inplace(x), reps))
    oop = statistics.fmean(timer.time(lambda: br.bitrev_outofplace(x, y), reps))
    out["complex128_2p24_paper_workload"] = {
        "inplace_GBps": round(gbs(nb, ip), 1), "outofplace_GBps": round(gbs(nb, oop), 1),
        "inplace_ms": round(ip, 5), "inplace_ns_per_element": round(1e6 * ip / (1 << 24), 6)}
    del x, y
    torch.cuda.empty_cache()
    # differentiation: 256 x 2^16 float32, forward and backward of BitRev
    xh, wh = workloads.rows_float32(256, 16, workloads.SEEDS["c5"])
    x = torch.from_numpy(xh).cuda().requires_grad_()
    w = torch.from_numpy(wh).cuda()
    nb = 2.0 * x.numel() * 4
    fwd = timer.time(lambda: BitRev.apply(x), reps)
    yv = BitRev.apply(x)
    g = torch.ones_like(yv)
    bwd = timer.time(lambda: torch.autograd.grad(yv, x, g, retain_graph=True), reps)
    out["autograd_256x2p16_f32"] = {"forward_GBps": round(gbs(nb, med(fwd)), 1),
                                    "backward_GBps": round(gbs(nb, med(bwd)), 1),
                                    "forward_us": round(1e3 * med(fwd), 2),
                                    "backward_us": round(1e3 * med(bwd), 2)}
    del x, w, yv, g
    # bit reversal fused with 6 radix-2 DIT levels, complex64 2^24, out of place
    x = workloads.device_normal(1 << 24, workloads.SEEDS["c2"], torch.complex64)
    y = torch.empty_like(x)
    nb = 2.0 * x.numel() * 8
    out["dit6_complex64_2p24"] = {
        "GBps": round(gbs(nb, med(timer.time(lambda: br.bitrev_dit_stages(x, y, 6), reps))), 1),
        "inplace_GBps": round(gbs(nb, med(timer.time(lambda: br.bitrev_dit_stages(x, x, 6),
                                                     reps))), 1),
        "plain_outofplace_GBps": round(gbs(nb, med(timer.time(lambda: br.bitrev_outofplace(x, y), reps))), 1)}
    return out


def traffic_workload(torch, br, workloads) -> None:
    """A few calls of each main configuration, the caches evicted before
    every call, for rocprofv3 counter runs: prints, per configuration in run
    order, one JSON line with its library kernel dispatches per call and its
    algorithmic bytes per call (2 n s per array)."""
    timer = Timer(torch, flush=True)

    def run(name, fn, calls, dispatches, nbytes):
        for _ in range(calls):
            timer._flush()
            fn()
        torch.cuda.synchronize()
        print(json.dumps({"config": name, "calls": calls, "dispatches_per_call": dispatches,
                          "algorithmic_bytes_per_call": int(nbytes)}), flush=True)

    x = workloads.device_normal(1 << 24, workloads.SEEDS["c2"], torch.complex64)
    y = torch.empty_like(x)
    nb = 2 * x.numel() * 8
    run("copy plain complex64 2^24 (calibration)", lambda: br.bitrev_copy(x, y, cache_hints=1),
        3, 1, nb)
    run("copy streaming loads complex64 2^24 (calibration)",
        lambda: br.bitrev_copy(x, y, cache_hints=2), 3, 1, nb)
    run("in place complex64 2^24", lambda: br.bitrev_inplace(x), 4, 1, nb)
    run("out of place complex64 2^24", lambda: br.bitrev_outofplace(x, y), 3, 1, nb)
    run("fused DIT 6 levels in place complex64 2^24", lambda: br.bitrev_dit_stages(x, x, 6), 3, 1, nb)
    run("fused DIT 6 levels out of place complex64 2^24", lambda: br.bitrev_dit_stages(x, y, 6),
        3, 1, nb)
    run("radix-4 digit reversal in place complex64 2^24",
        lambda: br.bitrev_digitrev_inplace(x, 2), 2, 1, nb)
    del x, y
    torch.cuda.empty_cache()
    for name, k, dt, seed in (("complex128 2^28", 28, torch.complex128, workloads.SEEDS["c3a"]),
                              ("float32 2^30", 30, torch.float32, workloads.SEEDS["c3b"]),
                              ("complex64 2^29", 29, torch.complex64, 129)):
        x = workloads.device_normal(1 << k, seed, dt)
        y = torch.empty_like(x)
        nb = 2 * x.numel() * x.element_size()
        run("in place " + name, lambda: br.bitrev_inplace(x), 2, 1, nb)
        run("out of place " + name, lambda: br.bitrev_outofplace(x, y), 2, 1, nb)
        run("copy, write-through, " + name, lambda: br.bitrev_copy(x, y, cache_hints=4), 2, 1, nb)
        run("copy in tile order " + name, lambda: br.bitrev_copy_tiled(x, y), 2, 1, nb)
        del x, y
        torch.cuda.empty_cache()
    offsets, log2n = workloads.batched_layout(4096, 8, 20, workloads.SEEDS["c4"])
    data = workloads.device_normal(int(offsets[-1]), workloads.SEEDS["c4"] + 1000, torch.complex64)
    off = torch.from_numpy(offsets).cuda()
    l2 = torch.from_numpy(log2n).cuda()
    ws = torch.empty(br.bitrev_batched_workspace_size(len(log2n)), dtype=torch.uint8,
                     device="cuda")
    run("batched 4096 complex64 arrays, log2n in [8, 20] (prep + main kernel)",
        lambda: br.bitrev_batched(data, off, l2, ws), 2, 2, 2 * int(offsets[-1]) * 8)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline steps (for profiler runs)")
    ap.add_argument("--hot", action="store_true", help="do not flush caches between steps")
    ap.add_argument("--tile-bits", type=int, default=0, help="force b (0: library plan)")
    ap.add_argument("--variant", type=int, default=0, help="force the tile kernel variant")
    ap.add_argument("--order", type=int, default=0, help="force the work-item order")
    ap.add_argument("--traffic-workload", action="store_true",
                    help="only run each main configuration a few times, for counter runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs on one device and has no "
              "multi-GPU form, so --gpus must be 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1708_01873_amd as br
    from paper_1708_01873_amd import workloads

    if not os.path.exists(br.LIBRARY):
        import __graft_entry__
        __graft_entry__.build()
    br.lib()
    torch.cuda.set_device(0)
    if args.traffic_workload:
        traffic_workload(torch, br, workloads)
        return 0
    k, s = 24, 8
    n = 1 << k
    nbytes = 2.0 * n * s
    log("generating complex64 n=2^24 (seed %d)" % workloads.SEEDS["c2"])
    host = workloads.complex64_normal(k, workloads.SEEDS["c2"])
    x = torch.from_numpy(host).cuda()
    cfg = dict(tile_bits=args.tile_bits, variant=args.variant, order=args.order)
    plan = br.bitrev_plan_query(k, s, **cfg)
    timer = Timer(torch, flush=not args.hot)

    def step():
        br.bitrev_inplace(x, k, **cfg)

    log("headline: %d warmup + %d timed in-place steps, plan %s" % (args.warmup, args.steps, plan))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times = timer.time(step, args.steps, warmup=args.warmup)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mean_ms = statistics.fmean(times)
    value = gbs(nbytes, mean_ms)

    # the kernel alone, for the roofline: the same steps under the same cache
    # flush, each launch recording HIP events from its own dispatch (that
    # launch path adds dispatch latency to the step, so it is not the step
    # timed above).  The events skip the system-scope fence, whose L2
    # writeback would otherwise land inside the stop timestamp.
    kernel_events = [(br.TimingEvent(), br.TimingEvent()) for _ in range(args.steps)]
    for ka, kb in kernel_events:
        timer._flush()
        br.bitrev_inplace_timed(x, ka, kb, k, **cfg)
    torch.cuda.synchronize()
    kernel_ms = statistics.fmean(ka.elapsed_time(kb) for ka, kb in kernel_events)
    for ev in kernel_events:
        ev[0].destroy()
        ev[1].destroy()
    applied_extra = args.steps

    # parity of the final state: an even number of applications is the input
    import oracle
    applied = args.steps + args.warmup + applied_extra
    got = x.cpu().numpy()
    want = host if applied % 2 == 0 else oracle.outofplace(host)
    bit_exact = bool(np.array_equal(got.view(np.uint8), want.view(np.uint8)))
    log("headline %.1f GB/s (mean %.4f ms), bit_exact=%s" % (value, mean_ms, bit_exact))

    # the reference copy of the same bytes under the same flush policy
    y = torch.empty_like(x)
    # the fastest copy measured (linear and tile-order copies, each in its
    # four cache-hint forms): the denominator is never a slower copy
    copy_best = best_copy(torch, br, timer, x, y, args.steps)
    copy_ms = copy_best["ms"]
    copy_gbs = gbs(nbytes, copy_ms)
    log("copy %.1f GB/s (mean %.4f ms, %s)" % (copy_gbs, copy_ms, copy_best))

    if plan["variant"] == 2:
        kernel = "k_tile_inplace_pipe<8,%d,true>" % plan["tile_bits"]
    else:  # the one-item kernel's last template argument is its cache hint (plan value - 1)
        kernel = "k_tile_inplace<8,%d,true,%d>" % (plan["tile_bits"], plan["cache_hints"] - 1)
    traffic = read_traffic(kernel)
    out = {
        "metric": "effective GB/s and % of HBM peak per n; batched vs per-array-loop speedup",
        "value": round(value, 2),
        "value_is": "effective GB/s (2*n*elem_size/time) of the in-place bit-reversed "
                    "permutation, complex64 n=2^24; % of HBM peak in pct_hbm_peak, the batched "
                    "speedup in batched_speedup_vs_loop",
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mean_ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic: real and imaginary parts i.i.d. N(0,1) float32, numpy PCG64 seed 2",
        "config": {"workload": "in-place bitrev, complex64, n=2^24 (128 MiB), HBM-resident, "
                               "caches flushed between steps" if not args.hot else
                               "in-place bitrev, complex64, n=2^24 (128 MiB), hot caches",
                   "log2n": k, "elem_size": s, "tile_bits": plan["tile_bits"],
                   "grid_blocks": plan["grid_blocks"], "block_threads": plan["block_threads"],
                   "variant": plan["variant"], "order": plan["order"],
                   "xcd_remap": plan["xcd_remap"], "cache_hints": plan["cache_hints"]},
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "copy_GBps": round(copy_gbs, 2),
        "copy_form": "%s, hints %d" % (copy_best["copy"], copy_best["cache_hints"]),
        "pct_of_copy": round(100.0 * value / copy_gbs, 2),
        "bit_exact": bit_exact,
        "wall_s_timed_loop": round(wall, 4),
        "step_ms_min_median_max": [round(min(times), 5), round(statistics.median(times), 5),
                                   round(max(times), 5)],
        "roofline": {
            "bound": "hbm",
            # algorithmic bytes per launch / the kernel's mean duration, from
            # HIP events its own dispatch recorded (kernel-timing loop)
            "achieved": round(gbs(nbytes, kernel_ms), 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs(nbytes, kernel_ms) / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic, 1),
            "kernel": kernel,
            "algorithmic_bytes_per_launch": nbytes,
            "kernel_ms_mean": round(kernel_ms, 5),
            "step_ms_mean": round(mean_ms, 5),
        },
    }

    if not args.no_extras:
        extras = {}
        c2 = timer.time(lambda: y.copy_(x), args.steps)
        extras["torch_copy_GBps"] = round(gbs(nbytes, statistics.fmean(c2)), 2)
        o = timer.time(lambda: br.bitrev_outofplace(x, y), args.steps)
        extras["outofplace_GBps"] = round(gbs(nbytes, statistics.fmean(o)), 2)
        sweep = {}
        for b in (4, 5, 6):
            for order in (1, 2, 3):
                ti = timer.time(lambda: br.bitrev_inplace(x, k, tile_bits=b, order=order), args.steps)
                to = timer.time(lambda: br.bitrev_outofplace(x, y, k, tile_bits=b, order=order),
                                args.steps)
                sweep["b%d_%s" % (b, ("natural", "balanced", "grouped")[order - 1])] = {
                    "inplace_GBps": round(gbs(nbytes, statistics.fmean(ti)), 2),
                    "outofplace_GBps": round(gbs(nbytes, statistics.fmean(to)), 2)}
        extras["tile_sweep"] = sweep
        rec_ms = statistics.fmean(
            timer.time(lambda: br.bitrev_inplace_recursive(x, k, levels=2), args.steps))
        rec1_ms = statistics.fmean(
            timer.time(lambda: br.bitrev_inplace_recursive(x, k, levels=1), args.steps))
        extras["paper_recursive_scheme"] = {
            "what": "the paper's recursive method as its GPU variant runs it, two recursion "
                    "levels: block-local reversals of 2^12 elements (each reversed in LDS by "
                    "the same three steps on 2^6 x 2^6), in-place square transpose, block-local "
                    "reversals (3 passes over HBM)",
            "GBps_effective": round(gbs(nbytes, rec_ms), 2),
            "ms": round(rec_ms, 5),
            "slowdown_vs_one_pass": round(rec_ms / mean_ms, 3),
            "one_level": {"what": "one recursion level, the block reversals by the one-pass "
                                  "tile kernel",
                          "GBps_effective": round(gbs(nbytes, rec1_ms), 2),
                          "ms": round(rec1_ms, 5)}}
        extras["other_configs"] = other_configs(torch, br, timer, args.steps)
        extras["per_n_complex64"] = per_n_complex64(torch, br, timer, max(10, args.steps // 2))
        extras["paper"] = PAPER_CONTEXT
        hot_timer = Timer(torch, flush=False)
        hot = hot_timer.time(step, args.steps)
        hot_copy = min((hot_timer.time(lambda: br.bitrev_copy(x, y, cache_hints=h), args.steps)
                        for h in (1, 2, 3, 4)), key=statistics.fmean)
        extras["hot_cache_inplace_GBps"] = round(gbs(nbytes, statistics.fmean(hot)), 2)
        extras["hot_cache_copy_GBps"] = round(gbs(nbytes, statistics.fmean(hot_copy)), 2)
        # the paper's unit: seconds per element (median of the timed steps)
        extras["ns_per_element"] = round(1e6 * statistics.median(times) / n, 6)
        log("extras: %s" % json.dumps(extras))
        try:
            extras["batched"] = batched_speedup(torch, br, reps=5)
            log("batched: %s" % json.dumps(extras["batched"]))
            out["batched_speedup_vs_loop"] = round(extras["batched"]["speedup_vs_eager_loop"], 3)
        except torch.cuda.OutOfMemoryError as e:  # pragma: no cover
            extras["batched"] = {"error": str(e)}
        out["context"] = extras

    if not args.no_cpu:
        log("cpu baseline: oracle in place on the same array, one core")
        reps, el, ok = cpu_baseline(host)
        out["cpu_baseline"] = {
            "value": round(gbs(nbytes * reps, el * 1e3), 4),
            "unit": "GB/s",
            "cores": 1,
            "kind": "oracle",
            "sample": "the full 2^24 complex64 array, in place, %d repetitions in %.1f s" % (reps, el),
            "bit_exact_vs_oracle_outofplace": ok,
            "cpu_model": cpu_model(),
            "host_cores_available": len(os.sched_getaffinity(0)),
        }
        log("cpu baseline: oracle out of place over all host threads")
        reps, el, threads, ok = cpu_multicore(host)
        out["cpu_baseline"]["all_cores"] = {
            "value": round(gbs(nbytes * reps, el * 1e3), 4),
            "unit": "GB/s",
            "cores": threads,
            "kind": "oracle, out of place, index range split over OpenMP threads",
            "sample": "the full 2^24 complex64 array, %d repetitions in %.1f s" % (reps, el),
            "bit_exact_vs_oracle_outofplace": ok,
        }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
