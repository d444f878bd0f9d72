"""HIP-graph capture of the batched permutation.

``BatchedGraph`` records ``bitrev_batched`` (prep kernel + persistent kernel)
into a graph once and replays it with one launch.  The library allocates and
synchronises nothing on this path and records no memset, so the capture holds
exactly the two kernels.  Choose the configuration (e.g. with ``tune``)
before capturing: the plan is fixed at capture time.
"""
from __future__ import annotations

import torch

from . import (bitrev_batched, bitrev_batched_workspace_size, bitrev_inplace, bitrev_plan_query,
               bitrev_rows, MODE_BATCHED)


class BatchedGraph:
    """One captured in-place batched permutation of fixed buffers."""

    def __init__(self, data, offsets, log2n, *, tile_bits=0, grid_blocks=0, order=0):
        self.data, self.offsets, self.log2n = data, offsets, log2n
        num = log2n.numel()
        self.workspace = torch.empty(max(1, bitrev_batched_workspace_size(num)),
                                     dtype=torch.uint8, device=data.device)
        self.cfg = dict(tile_bits=tile_bits, grid_blocks=grid_blocks, order=order)
        # resolves and caches the device properties outside the capture
        self.plan = bitrev_plan_query(0, data.element_size(), 1, MODE_BATCHED, **self.cfg)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            bitrev_batched(self.data, self.offsets, self.log2n, self.workspace, **self.cfg)

    def replay(self) -> None:
        self.graph.replay()


class CapturedCall:
    """A captured plain call (``bitrev_inplace`` or ``bitrev_rows``)."""

    def __init__(self, fn, *args, **kwargs):
        if fn not in (bitrev_inplace, bitrev_rows):
            raise ValueError("only bitrev_inplace and bitrev_rows are captured here")
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            fn(*args, **kwargs)

    def replay(self) -> None:
        self.graph.replay()
