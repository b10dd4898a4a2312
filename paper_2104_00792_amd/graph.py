"""HIP-graph capture of library calls.

A call of the library allocates its workspace (and a build its table) as it
runs.  Under capture those blocks come from an :class:`Arena`, one device
buffer sized beforehand with ``hg_workspace_size``, through
``hg_set_allocator``; a bump allocator hands out addresses and frees
nothing, so the captured kernels keep valid addresses at every replay and
the graph holds kernel nodes only (no allocation or memset nodes).  A replay
repeats the captured calls on the same arena, inputs and outputs.
"""

from __future__ import annotations

from . import hg_set_allocator


class Arena:
    """Bump allocator over one device buffer; blocks rounded to 256 bytes as
    ``hg_workspace_size`` counts them."""

    def __init__(self, nbytes: int, device=None):
        import torch

        self.size = int(nbytes)
        self.buf = torch.empty(max(self.size, 256), dtype=torch.uint8, device=device or "cuda")
        self.base = self.buf.data_ptr()
        self.off = 0
        self.high = 0

    def alloc(self, nbytes: int, stream: int) -> int:
        r = (nbytes + 255) & ~255
        if self.off + r > self.size:
            return 0  # the library reports HG_ERR_OUT_OF_MEMORY
        p = self.base + self.off
        self.off += r
        self.high = max(self.high, self.off)
        return p

    def free(self, ptr: int, nbytes: int, stream: int) -> None:
        pass  # reclaimed by reset()

    def reset(self) -> None:
        self.off = 0


class Captured:
    """``fn()`` captured once into a HIP graph on a side stream, with every
    library allocation served by ``arena``; :meth:`replay` enqueues it again
    on the current stream."""

    def __init__(self, fn, arena: Arena):
        import torch

        self.arena = arena
        self.graph = torch.cuda.CUDAGraph()
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        arena.reset()
        hg_set_allocator(arena.alloc, arena.free)
        try:
            with torch.cuda.graph(self.graph, stream=stream):
                fn()
        finally:
            hg_set_allocator()

    def replay(self) -> None:
        self.graph.replay()
