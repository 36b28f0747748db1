"""A search of fixed shape captured once in a HIP graph and replayed.

For request loops that launch the same batch shape over and over: the
status clear, scan and merge launches of one search are recorded once and
replayed with one call.  Inputs go into the captured buffers before each
replay (outside the graph: no memset or copy node is recorded).
"""
from __future__ import annotations

import numpy as np

from . import alloc_workspace, genie_search_async


class GraphSearch:
    def __init__(self, index, n_queries: int, k: int, max_items: int, item_capacity: int):
        import torch
        self.torch = torch
        self.index, self.nq, self.k, self.max_items = index, n_queries, k, max_items
        self.cap = item_capacity
        self.off = torch.zeros(n_queries + 1, dtype=torch.int64, device="cuda")
        self.items = torch.zeros((item_capacity, 3), dtype=torch.int32, device="cuda")
        self.ids = torch.empty((n_queries, k), dtype=torch.int32, device="cuda")
        self.cts = torch.empty_like(self.ids)
        self.ws = alloc_workspace(index, n_queries, k)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):       # eager run: sets kernel attributes
            self._launch()
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._launch()

    def _launch(self):
        genie_search_async(self.index, self.off, self.items, self.k, self.max_items, self.ids,
                           self.cts, self.ws, self.torch.cuda.current_stream())

    def __call__(self, q_offsets: np.ndarray, items: np.ndarray):
        """Replay on new queries (same count); returns device (ids, counts)."""
        torch = self.torch
        q_offsets = np.asarray(q_offsets, dtype=np.uint64)
        items = np.asarray(items, dtype=np.uint32).reshape(-1, 3)
        if len(q_offsets) != self.nq + 1 or len(items) > self.cap:
            raise ValueError("batch does not fit the captured shape")
        with torch.cuda.stream(self.stream):
            self.off.copy_(torch.from_numpy(q_offsets.view(np.int64)))
            if len(items):
                self.items[:len(items)].copy_(torch.from_numpy(items.view(np.int32)))
            self.graph.replay()
        self.stream.synchronize()
        return self.ids, self.cts
