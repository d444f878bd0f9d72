"""libbitrev: the bit-reversed permutation of n = 2^k elements on MI355X.

A thin ctypes binding over the C ABI in ``include/bitrev.h`` (the shared
library ``libbitrev.so`` built from ``csrc/`` by ``build.py``).  The functions
here have the C entry points' names and only marshal arguments: tensors give
their device pointer and element size, the stream defaults to torch's current
stream.  Every step of the permutation runs in the HIP kernels; if the library
is not built, every call raises.

The operation (arXiv:1708.01873, Introduction): element i of an array of
2^k elements moves to index rev_k(i), the low k bits of i reversed.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PKG_DIR, "libbitrev.so")

SUCCESS = 0
ERROR_INVALID_VALUE = 1
ERROR_ALIAS = 2
ERROR_WORKSPACE = 3
ERROR_HIP = 4
ERROR_NOT_SUPPORTED = 5

PATH_NONE, PATH_WAVE, PATH_TILE, PATH_BATCHED = 0, 1, 2, 3
MODE_INPLACE, MODE_OUTOFPLACE, MODE_BATCHED = 0, 1, 2
ORDER_DEFAULT, ORDER_NATURAL, ORDER_BALANCED, ORDER_GROUPED = 0, 1, 2, 3
VARIANT_DEFAULT, VARIANT_ONE_ITEM, VARIANT_PIPELINED, VARIANT_REGISTER_STAGED = 0, 1, 2, 3
XCD_DEFAULT, XCD_REMAP, XCD_DISPATCH_ORDER = 0, 1, 2
HINTS_DEFAULT, HINTS_PLAIN, HINTS_STREAM_LOADS, HINTS_STREAM_STORES = 0, 1, 2, 3
HINTS_STREAM_WRITE_THROUGH = 4  # streaming loads, write-through (device-scope) stores


class BitrevError(RuntimeError):
    """A libbitrev call returned a status other than BITREV_SUCCESS."""

    def __init__(self, status: int, where: str):
        self.status = status
        msg = "%s: %s" % (where, status_string(status))
        if status == ERROR_HIP:
            msg += " (hipError %d)" % _load().bitrev_last_hip_error()
        super().__init__(msg)


class Config(ctypes.Structure):
    """bitrev_config_t: zero fields mean "library choice"."""
    _fields_ = [("tile_bits", ctypes.c_int), ("grid_blocks", ctypes.c_int),
                ("order", ctypes.c_int), ("variant", ctypes.c_int), ("xcd_remap", ctypes.c_int),
                ("cache_hints", ctypes.c_int)]


class Plan(ctypes.Structure):
    """bitrev_plan_t."""
    _fields_ = [("path", ctypes.c_int), ("tile_bits", ctypes.c_int), ("mid_bits", ctypes.c_int),
                ("block_threads", ctypes.c_int), ("grid_blocks", ctypes.c_int),
                ("order", ctypes.c_int), ("vector_access", ctypes.c_int),
                ("variant", ctypes.c_int), ("xcd_remap", ctypes.c_int),
                ("cache_hints", ctypes.c_int), ("work_items", ctypes.c_uint64),
                ("lds_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib: Optional[ctypes.CDLL] = None

_VP, _I, _I64, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
_CFGP = ctypes.POINTER(Config)
_SIGNATURES = {
    "bitrev_inplace": ([_VP, _I, _SZ, _VP], _I),
    "bitrev_outofplace": ([_VP, _VP, _I, _SZ, _VP], _I),
    "bitrev_rows": ([_VP, _VP, _I, _I64, _SZ, _VP], _I),
    "bitrev_batched_workspace_size": ([_I64], _SZ),
    "bitrev_batched": ([_VP, _I64, _VP, _VP, _I64, _SZ, _VP, _SZ, _VP], _I),
    "bitrev_batched_noalloc": ([_VP, _I64, _VP, _VP, _I64, _SZ, _VP], _I),
    "bitrev_batched_errors": ([_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64), _VP], _I),
    "bitrev_inplace_ex": ([_VP, _I, _SZ, _CFGP, _VP], _I),
    "bitrev_outofplace_ex": ([_VP, _VP, _I, _SZ, _CFGP, _VP], _I),
    "bitrev_inplace_timed": ([_VP, _I, _SZ, _CFGP, _VP, _VP, _VP], _I),
    "bitrev_outofplace_timed": ([_VP, _VP, _I, _SZ, _CFGP, _VP, _VP, _VP], _I),
    "bitrev_timing_event_create": ([ctypes.POINTER(_VP)], _I),
    "bitrev_timing_event_destroy": ([_VP], _I),
    "bitrev_timing_elapsed_ms": ([_VP, _VP, ctypes.POINTER(ctypes.c_float)], _I),
    "bitrev_rows_ex": ([_VP, _VP, _I, _I64, _SZ, _CFGP, _VP], _I),
    "bitrev_batched_ex": ([_VP, _I64, _VP, _VP, _I64, _SZ, _VP, _SZ, _CFGP, _VP], _I),
    "bitrev_plan_query": ([_I, _SZ, _I64, _I, _CFGP, ctypes.POINTER(Plan)], _I),
    "bitrev_load_tuning": ([ctypes.c_char_p], _I),
    "bitrev_tuning_format": ([], ctypes.c_char_p),
    "bitrev_digitrev_inplace_ex": ([_VP, _I, _I, _SZ, _CFGP, _VP], _I),
    "bitrev_digitrev_outofplace_ex": ([_VP, _VP, _I, _I, _SZ, _CFGP, _VP], _I),
    "bitrev_copy": ([_VP, _VP, _SZ, _VP], _I),
    "bitrev_copy_ex": ([_VP, _VP, _SZ, _I, _VP], _I),
    "bitrev_copy_tiled": ([_VP, _VP, _I, _SZ, _CFGP, _VP], _I),
    "bitrev_inplace_recursive": ([_VP, _I, _SZ, _VP], _I),
    "bitrev_inplace_recursive_ex": ([_VP, _I, _SZ, _I, _VP], _I),
    "bitrev_dit_stages": ([_VP, _VP, _I, _I64, _I, _I, _I, _VP], _I),
    "bitrev_dit_stages_ex": ([_VP, _VP, _I, _I64, _I, _I, _I, _CFGP, _VP], _I),
    "bitrev_digitrev_inplace": ([_VP, _I, _I, _SZ, _VP], _I),
    "bitrev_rows_strided": ([_VP, _VP, _I, _I64, _I64, _I64, _SZ, _VP], _I),
    "bitrev_evenodd": ([_VP, _VP, _I, _I64, _SZ, _VP], _I),
    "bitrev_batched_outofplace": ([_VP, _VP, _I64, _VP, _VP, _I64, _SZ, _VP, _SZ, _VP], _I),
    "bitrev_digitrev_outofplace": ([_VP, _VP, _I, _I, _SZ, _VP], _I),
    "bitrev_debug_digit_rev": ([ctypes.c_uint32, _I, _I], ctypes.c_uint32),
    "bitrev_debug_digit_pair_count": ([_I, _I], ctypes.c_uint64),
    "bitrev_debug_digit_inplace_pair_at": ([_I, ctypes.c_uint64, _I], ctypes.c_uint32),
    "bitrev_debug_digit_pair_at": ([_I, ctypes.c_uint64, _I], ctypes.c_uint32),
    "bitrev_transpose_inplace": ([_VP, _I, _SZ, _VP], _I),
    "bitrev_status_string": ([_I], ctypes.c_char_p),
    "bitrev_last_hip_error": ([], _I),
    "bitrev_abi_version": ([], _I),
    "bitrev_debug_rev": ([ctypes.c_uint32, _I], ctypes.c_uint32),
    "bitrev_debug_pair_count": ([_I], ctypes.c_uint64),
    "bitrev_debug_pair_at": ([_I, ctypes.c_uint64, _I], ctypes.c_uint32),
    "bitrev_debug_inplace_pair_at": ([_I, ctypes.c_uint64, _I], ctypes.c_uint32),
    "bitrev_debug_oop_tile_at": ([_I, ctypes.c_uint32, _I], ctypes.c_uint32),
    "bitrev_debug_spread": ([ctypes.c_uint32, _I], ctypes.c_uint32),
    "bitrev_debug_tri_pair": ([ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32),
                               ctypes.POINTER(ctypes.c_uint32)], None),
}
EXPORTED = tuple(_SIGNATURES)


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError(
                "libbitrev.so is not built (%s); run `python -m paper_1708_01873_amd.build` "
                "or __graft_entry__.build()" % LIBRARY)
        lib = ctypes.CDLL(LIBRARY)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def lib() -> ctypes.CDLL:
    """The loaded C library (raises if it is not built)."""
    return _load()


def status_string(status: int) -> str:
    return _load().bitrev_status_string(int(status)).decode()


def abi_version() -> int:
    return _load().bitrev_abi_version()


def _check(status: int, where: str) -> None:
    if status != SUCCESS:
        raise BitrevError(status, where)


def _config(tile_bits=0, grid_blocks=0, order=0, config=None, variant=0, xcd_remap=0,
            cache_hints=0):
    if config is not None:
        return config
    if tile_bits or grid_blocks or order or variant or xcd_remap or cache_hints:
        return Config(int(tile_bits), int(grid_blocks), int(order), int(variant), int(xcd_remap),
                      int(cache_hints))
    return None


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tensor_args(t, what: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % what)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor (libbitrev runs on the GPU only)" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return t.data_ptr(), t.element_size()


def _log2_exact(n: int) -> int:
    k = int(n).bit_length() - 1
    if n <= 0 or (1 << k) != n:
        raise ValueError("length %d is not a power of two" % n)
    return k


def bitrev_inplace(data, log2n: Optional[int] = None, *, tile_bits=0, grid_blocks=0, order=0,
                   variant=0, xcd_remap=0, cache_hints=0, config=None, stream=None):
    """Replace ``data`` (2^log2n contiguous elements) by its bit-reversed
    permutation.  ``log2n`` defaults to log2(data.numel())."""
    ptr, s = _tensor_args(data, "data")
    k = _log2_exact(data.numel()) if log2n is None else int(log2n)
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    L = _load()
    if cfg is None:
        _check(L.bitrev_inplace(ptr, k, s, _stream(stream)), "bitrev_inplace")
    else:
        _check(L.bitrev_inplace_ex(ptr, k, s, ctypes.byref(cfg), _stream(stream)),
               "bitrev_inplace_ex")
    return data


class TimingEvent:
    """A HIP timing event from bitrev_timing_event_create (system-scope fence
    disabled, so that it timestamps the kernel's end and not the L2 writeback
    such a fence adds): the start or stop event of the *_timed calls."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(_load().bitrev_timing_event_create(ctypes.byref(h)), "bitrev_timing_event_create")
        self.handle = h.value

    def elapsed_time(self, stop: "TimingEvent") -> float:
        """Milliseconds from this event to ``stop`` (waits for ``stop``)."""
        ms = ctypes.c_float()
        _check(_load().bitrev_timing_elapsed_ms(ctypes.c_void_p(self.handle),
                                                 ctypes.c_void_p(stop.handle), ctypes.byref(ms)),
               "bitrev_timing_elapsed_ms")
        return ms.value

    def destroy(self) -> None:
        if self.handle:
            _check(_load().bitrev_timing_event_destroy(ctypes.c_void_p(self.handle)),
                   "bitrev_timing_event_destroy")
            self.handle = None


def _event_handle(event, name):
    handle = event.handle if isinstance(event, TimingEvent) else getattr(event, "cuda_event", 0)
    if not handle:
        raise ValueError("%s must be a TimingEvent, or a torch.cuda.Event(enable_timing=True) "
                         "that has been recorded once (torch creates the HIP event on its "
                         "first record)" % name)
    return ctypes.c_void_p(handle)


def bitrev_inplace_timed(data, start_event, stop_event, log2n: Optional[int] = None, *,
                         tile_bits=0, grid_blocks=0, order=0, variant=0, xcd_remap=0,
                         cache_hints=0, config=None, stream=None):
    """bitrev_inplace whose kernel launch records ``start_event`` as the
    kernel starts and ``stop_event`` as it ends, so that
    ``start_event.elapsed_time(stop_event)`` is the kernel's own duration
    (TimingEvent: without the L2 writeback of a system-scope fence)."""
    ptr, s = _tensor_args(data, "data")
    k = _log2_exact(data.numel()) if log2n is None else int(log2n)
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    _check(_load().bitrev_inplace_timed(ptr, k, s, cfg, _event_handle(start_event, "start_event"),
                                        _event_handle(stop_event, "stop_event"), _stream(stream)),
           "bitrev_inplace_timed")
    return data


def bitrev_outofplace_timed(src, dst, start_event, stop_event, log2n: Optional[int] = None, *,
                            tile_bits=0, grid_blocks=0, order=0, variant=0, xcd_remap=0,
                            cache_hints=0, config=None, stream=None):
    """bitrev_outofplace with the kernel timed as in bitrev_inplace_timed."""
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2 or src.numel() != dst.numel():
        raise ValueError("src and dst must have the same element size and length")
    k = _log2_exact(src.numel()) if log2n is None else int(log2n)
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    _check(_load().bitrev_outofplace_timed(sp, dp, k, s, cfg,
                                           _event_handle(start_event, "start_event"),
                                           _event_handle(stop_event, "stop_event"),
                                           _stream(stream)),
           "bitrev_outofplace_timed")
    return dst


def bitrev_outofplace(src, dst=None, log2n: Optional[int] = None, *, tile_bits=0, grid_blocks=0,
                      order=0, variant=0, xcd_remap=0, cache_hints=0, config=None, stream=None):
    """dst[rev(i)] = src[i]; allocates ``dst`` like ``src`` when not given."""
    if dst is None:
        import torch
        dst = torch.empty_like(src)
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2 or src.numel() != dst.numel():
        raise ValueError("src and dst must have the same element size and length")
    k = _log2_exact(src.numel()) if log2n is None else int(log2n)
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    L = _load()
    if cfg is None:
        _check(L.bitrev_outofplace(sp, dp, k, s, _stream(stream)), "bitrev_outofplace")
    else:
        _check(L.bitrev_outofplace_ex(sp, dp, k, s, ctypes.byref(cfg), _stream(stream)),
               "bitrev_outofplace_ex")
    return dst


def bitrev_rows(src, dst=None, log2n: Optional[int] = None, *, tile_bits=0, grid_blocks=0,
                order=0, variant=0, xcd_remap=0, cache_hints=0, config=None, stream=None):
    """Permute every row of 2^log2n elements (default: the last dimension);
    ``dst is src`` works in place.  Allocates ``dst`` when not given."""
    if dst is None:
        import torch
        dst = torch.empty_like(src)
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2 or src.numel() != dst.numel():
        raise ValueError("src and dst must have the same element size and length")
    if log2n is None:
        if src.dim() == 0:
            raise ValueError("bitrev_rows needs at least one dimension")
        k = _log2_exact(src.shape[-1])
    else:
        k = int(log2n)
    n = 1 << k
    if src.numel() % n:
        raise ValueError("%d elements are not a whole number of rows of %d" % (src.numel(), n))
    rows = src.numel() // n
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    L = _load()
    if cfg is None:
        _check(L.bitrev_rows(sp, dp, k, rows, s, _stream(stream)), "bitrev_rows")
    else:
        _check(L.bitrev_rows_ex(sp, dp, k, rows, s, ctypes.byref(cfg), _stream(stream)),
               "bitrev_rows_ex")
    return dst


def bitrev_batched_workspace_size(num_arrays: int) -> int:
    return int(_load().bitrev_batched_workspace_size(int(num_arrays)))


def bitrev_batched(data, offsets, log2n, workspace=None, *, tile_bits=0, grid_blocks=0, order=0,
                   variant=0, xcd_remap=0, cache_hints=0, config=None, stream=None):
    """In place on every packed array [offsets[a], offsets[a+1]) of ``data``
    (lengths 2^log2n[a]).  ``offsets`` (int64, num+1) and ``log2n`` (int32,
    num) are device tensors; ``workspace`` is a device byte tensor of at least
    bitrev_batched_workspace_size(num) bytes (allocated when not given, which
    is not allowed under graph capture)."""
    import torch
    dp, s = _tensor_args(data, "data")
    if offsets.dtype != torch.int64 or log2n.dtype != torch.int32:
        raise TypeError("offsets must be int64 and log2n int32")
    op, _ = _tensor_args(offsets, "offsets")
    lp, _ = _tensor_args(log2n, "log2n")
    num = log2n.numel()
    if offsets.numel() != num + 1:
        raise ValueError("offsets must have num_arrays + 1 entries")
    need = bitrev_batched_workspace_size(num)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=data.device)
    wp, _ = _tensor_args(workspace, "workspace")
    wbytes = workspace.numel() * workspace.element_size()
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    L = _load()
    if cfg is None:
        _check(L.bitrev_batched(dp, data.numel(), op, lp, num, s, wp, wbytes, _stream(stream)),
               "bitrev_batched")
    else:
        _check(L.bitrev_batched_ex(dp, data.numel(), op, lp, num, s, wp, wbytes,
                                   ctypes.byref(cfg), _stream(stream)), "bitrev_batched_ex")
    return data


NOALLOC_MAX_ARRAYS = 65536  # BITREV_NOALLOC_MAX_ARRAYS


def bitrev_batched_noalloc(data, offsets, log2n, *, stream=None):
    """As bitrev_batched with the built-in plan, for callers that cannot
    allocate: the workspace is the library's own per-device array (at most
    NOALLOC_MAX_ARRAYS arrays); nothing is allocated here or in the library.
    Calls that overlap on one GPU race on that array."""
    import torch
    dp, s = _tensor_args(data, "data")
    if offsets.dtype != torch.int64 or log2n.dtype != torch.int32:
        raise TypeError("offsets must be int64 and log2n int32")
    op, _ = _tensor_args(offsets, "offsets")
    lp, _ = _tensor_args(log2n, "log2n")
    num = log2n.numel()
    if offsets.numel() != num + 1:
        raise ValueError("offsets must have num_arrays + 1 entries")
    _check(_load().bitrev_batched_noalloc(dp, data.numel(), op, lp, num, s, _stream(stream)),
           "bitrev_batched_noalloc")
    return data


def bitrev_batched_outofplace(src, dst, offsets, log2n, workspace=None, *, stream=None):
    """Out of place over the same packed layout: each array of ``src`` lands
    bit-reversed at the same offsets of ``dst``."""
    import torch
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2 or src.numel() != dst.numel():
        raise ValueError("src and dst must have the same element size and length")
    if offsets.dtype != torch.int64 or log2n.dtype != torch.int32:
        raise TypeError("offsets must be int64 and log2n int32")
    op, _ = _tensor_args(offsets, "offsets")
    lp, _ = _tensor_args(log2n, "log2n")
    num = log2n.numel()
    if offsets.numel() != num + 1:
        raise ValueError("offsets must have num_arrays + 1 entries")
    if workspace is None:
        workspace = torch.empty(max(bitrev_batched_workspace_size(num), 1), dtype=torch.uint8,
                                device=src.device)
    wp, _ = _tensor_args(workspace, "workspace")
    _check(_load().bitrev_batched_outofplace(sp, dp, src.numel(), op, lp, num, s, wp,
                                             workspace.numel() * workspace.element_size(),
                                             _stream(stream)), "bitrev_batched_outofplace")
    return dst


def bitrev_rows_strided(src, dst, log2n: int, rows: int, src_stride: int, dst_stride: int, *,
                        stream=None):
    """Rows of 2^log2n elements at element strides src_stride / dst_stride
    from the start of each tensor's storage (``dst is src`` in place)."""
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2:
        raise ValueError("src and dst must have the same element size")
    need_s = (rows - 1) * src_stride + (1 << log2n) if rows else 0
    need_d = (rows - 1) * dst_stride + (1 << log2n) if rows else 0
    if src.numel() < need_s or dst.numel() < need_d:
        raise ValueError("tensors are too small for the requested rows and strides")
    _check(_load().bitrev_rows_strided(sp, dp, int(log2n), int(rows), int(src_stride),
                                       int(dst_stride), s, _stream(stream)), "bitrev_rows_strided")
    return dst


def bitrev_evenodd(src, dst=None, *, stream=None):
    """One even-odd (Stockham) split of every row (last dimension): evens
    first, then odds.  Allocates ``dst`` when not given."""
    if dst is None:
        import torch
        dst = torch.empty_like(src)
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2 or src.numel() != dst.numel():
        raise ValueError("src and dst must have the same element size and length")
    k = _log2_exact(src.shape[-1])
    _check(_load().bitrev_evenodd(sp, dp, k, src.numel() >> k, s, _stream(stream)),
           "bitrev_evenodd")
    return dst


def bitrev_batched_errors(workspace, stream=None) -> tuple[int, int]:
    """(arrays rejected, first rejected or -1) of the last batched call on
    ``workspace``; waits for the stream."""
    wp, _ = _tensor_args(workspace, "workspace")
    nrej, first = ctypes.c_int64(0), ctypes.c_int64(-1)
    _check(_load().bitrev_batched_errors(wp, ctypes.byref(nrej), ctypes.byref(first),
                                         _stream(stream)), "bitrev_batched_errors")
    return nrej.value, first.value


def bitrev_copy(src, dst, stream=None, *, cache_hints=0):
    """The reference streaming copy (same bytes as an out-of-place pass);
    cache_hints as in Config (0: the library's choice for the size)."""
    sp, _ = _tensor_args(src, "src")
    dp, _ = _tensor_args(dst, "dst")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check(_load().bitrev_copy_ex(sp, dp, nbytes, int(cache_hints), _stream(stream)),
           "bitrev_copy")
    return dst


def bitrev_copy_tiled(src, dst, *, tile_bits=0, grid_blocks=0, order=0, xcd_remap=0,
                      cache_hints=0, config=None, stream=None):
    """The reference copy in the tile kernels' order (dst = src), visiting
    the tiles of the out-of-place plan for src's length; plan fields as in
    Config (0: the plan's own choice)."""
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2 or src.numel() != dst.numel():
        raise ValueError("src and dst must have the same element size and length")
    k = _log2_exact(src.numel())
    cfg = _config(tile_bits, grid_blocks, order, config, 0, xcd_remap, cache_hints)
    _check(_load().bitrev_copy_tiled(sp, dp, k, s, None if cfg is None else ctypes.byref(cfg),
                                     _stream(stream)), "bitrev_copy_tiled")
    return dst


def bitrev_digitrev_inplace(data, digit_bits: int, log2n: Optional[int] = None, *, tile_bits=0,
                            grid_blocks=0, order=0, xcd_remap=0, cache_hints=0, config=None,
                            stream=None):
    """Reverse the order of the digit_bits-bit digits of every index, in place
    (digit_bits 2: radix-4 order, 3: radix-8 order, 1: bit reversal).  The
    keyword arguments force the launch configuration (bitrev_digitrev_inplace_ex)."""
    ptr, s = _tensor_args(data, "data")
    k = _log2_exact(data.numel()) if log2n is None else int(log2n)
    cfg = _config(tile_bits, grid_blocks, order, config, 0, xcd_remap, cache_hints)
    if cfg is None:
        st = _load().bitrev_digitrev_inplace(ptr, k, int(digit_bits), s, _stream(stream))
    else:
        st = _load().bitrev_digitrev_inplace_ex(ptr, k, int(digit_bits), s, ctypes.byref(cfg),
                                                _stream(stream))
    _check(st, "bitrev_digitrev_inplace")
    return data


def bitrev_digitrev_outofplace(src, dst=None, digit_bits: int = 2, log2n: Optional[int] = None, *,
                               tile_bits=0, grid_blocks=0, order=0, xcd_remap=0, cache_hints=0,
                               config=None, stream=None):
    """dst[drev(i)] = src[i] for digits of digit_bits bits.  The keyword
    arguments force the launch configuration (bitrev_digitrev_outofplace_ex)."""
    if dst is None:
        import torch
        dst = torch.empty_like(src)
    sp, s = _tensor_args(src, "src")
    dp, s2 = _tensor_args(dst, "dst")
    if s != s2 or src.numel() != dst.numel():
        raise ValueError("src and dst must have the same element size and length")
    k = _log2_exact(src.numel()) if log2n is None else int(log2n)
    cfg = _config(tile_bits, grid_blocks, order, config, 0, xcd_remap, cache_hints)
    if cfg is None:
        st = _load().bitrev_digitrev_outofplace(sp, dp, k, int(digit_bits), s, _stream(stream))
    else:
        st = _load().bitrev_digitrev_outofplace_ex(sp, dp, k, int(digit_bits), s,
                                                   ctypes.byref(cfg), _stream(stream))
    _check(st, "bitrev_digitrev_outofplace")
    return dst


def bitrev_dit_stages(src, dst=None, stages: int = 1, *, inverse: bool = False, log2n=None,
                      tile_bits=0, grid_blocks=0, order=0, variant=0, xcd_remap=0, cache_hints=0,
                      config=None, stream=None):
    """Bit reversal of each row (last dimension, complex64 or complex128)
    followed by the first `stages` radix-2 DIT FFT levels; ``dst is src``
    works in place.  Allocates ``dst`` when not given.  variant: 1 square
    tiles, 2 / 3 rectangular tiles out of place, 3 in place the tile pair
    held in registers (see the C header)."""
    import torch
    if src.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("bitrev_dit_stages needs complex64 or complex128 data")
    if dst is None:
        dst = torch.empty_like(src)
    if dst.dtype != src.dtype or dst.numel() != src.numel():
        raise ValueError("src and dst must have the same dtype and length")
    sp, _ = _tensor_args(src, "src")
    dp, _ = _tensor_args(dst, "dst")
    k = _log2_exact(src.shape[-1]) if log2n is None else int(log2n)
    rows = src.numel() >> k
    if rows << k != src.numel():
        raise ValueError("not a whole number of rows")
    dtype = 0 if src.dtype == torch.complex64 else 1
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    _check(_load().bitrev_dit_stages_ex(sp, dp, k, rows, int(stages), 1 if inverse else 0, dtype,
                                        cfg, _stream(stream)), "bitrev_dit_stages")
    return dst


def bitrev_inplace_recursive(data, log2n: Optional[int] = None, *, levels: int = 0,
                             stream=None):
    """In place by the paper's recursive scheme (three passes: block-local
    reversals, square transpose, block-local reversals); log2n must be even.
    levels: 2 = the block reversals recurse once more in LDS (log2n divisible
    by 4, blocks of at most 64 KiB), 1 = they are the one-pass tile kernels,
    0 = two where they apply.  An A/B baseline for bitrev_inplace, which
    makes one pass."""
    ptr, s = _tensor_args(data, "data")
    k = _log2_exact(data.numel()) if log2n is None else int(log2n)
    if levels:
        _check(_load().bitrev_inplace_recursive_ex(ptr, k, s, int(levels), _stream(stream)),
               "bitrev_inplace_recursive_ex")
    else:
        _check(_load().bitrev_inplace_recursive(ptr, k, s, _stream(stream)),
               "bitrev_inplace_recursive")
    return data


def bitrev_transpose_inplace(data, log2side: Optional[int] = None, *, stream=None):
    """Transpose the square 2^log2side x 2^log2side matrix ``data`` in place
    (default: from a 2-D square tensor's shape)."""
    ptr, s = _tensor_args(data, "data")
    if log2side is None:
        if data.dim() != 2 or data.shape[0] != data.shape[1]:
            raise ValueError("give log2side or a square 2-D tensor")
        log2side = _log2_exact(data.shape[0])
    _check(_load().bitrev_transpose_inplace(ptr, int(log2side), s, _stream(stream)),
           "bitrev_transpose_inplace")
    return data


def bitrev_plan_query(log2n: int, elem_size: int, rows: int = 1, mode: int = MODE_INPLACE,
                      *, tile_bits=0, grid_blocks=0, order=0, variant=0, xcd_remap=0,
                      cache_hints=0, config=None) -> dict:
    """The plan a call would use (no launch)."""
    cfg = _config(tile_bits, grid_blocks, order, config, variant, xcd_remap, cache_hints)
    p = Plan()
    _check(_load().bitrev_plan_query(int(log2n), int(elem_size), int(rows), int(mode),
                                     ctypes.byref(cfg) if cfg is not None else None,
                                     ctypes.byref(p)), "bitrev_plan_query")
    return p.as_dict()


def bitrev_load_tuning(path: Optional[str]) -> None:
    """Load a tuning table file (None restores the built-in defaults)."""
    _check(_load().bitrev_load_tuning(None if path is None else os.fsencode(path)),
           "bitrev_load_tuning")


def bitrev_tuning_format() -> str:
    return _load().bitrev_tuning_format().decode()


__all__ = [
    "BitrevError", "Config", "Plan", "TimingEvent", "lib", "abi_version", "status_string",
    "bitrev_inplace_timed", "bitrev_outofplace_timed",
    "bitrev_inplace", "bitrev_outofplace", "bitrev_rows", "bitrev_batched",
    "bitrev_batched_workspace_size", "bitrev_batched_errors", "bitrev_copy",
    "bitrev_plan_query", "bitrev_load_tuning", "bitrev_tuning_format",
    "bitrev_inplace_recursive", "bitrev_transpose_inplace", "bitrev_dit_stages",
    "bitrev_digitrev_inplace", "bitrev_digitrev_outofplace", "bitrev_batched_outofplace",
    "bitrev_rows_strided", "bitrev_evenodd",
]
