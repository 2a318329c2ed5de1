"""Batched query pipeline: sign -> band -> candidate lookup -> exact-Jaccard
refinement -> top-10 for a fixed-shape batch of queries, run eagerly or
captured once as a HIP graph and replayed per batch.  Every buffer is
allocated up front; the lookup has a fixed candidate capacity with a device
overflow flag, so no stage needs the host."""
from __future__ import annotations

import numpy as np
import torch

from . import polymh as pm


class QueryBatch:
    def __init__(self, D: pm.DevicePolys, sorted_keys, sorted_ent, box, seed: int, k: int, cap: int,
                 bands: int, rows: int, n_queries: int, max_vertices: int, cand_cap: int,
                 sign_config=None, topk: int = 10, binned=None):
        """``binned``: None signs the queries by the walk; a dict with
        horizon, bin_bits and walk_ratio signs them from binned samples
        (``polymh_sign_binned``, the same bits)."""
        dev = D.offsets.device
        self.D, self.sk, self.se = D, sorted_keys, sorted_ent
        self.box, self.seed, self.k, self.cap = box, seed, k, cap
        self.bands, self.rows, self.topk = bands, rows, topk
        self.nq = n_queries
        self.cfg = sign_config or pm.default_sign_config()
        self.xy = torch.zeros((max_vertices, 2), dtype=torch.int32, device=dev)
        self.off = torch.zeros(n_queries + 1, dtype=torch.int64, device=dev)
        self.Q = pm.DevicePolys(self.xy, self.off)
        self.sig = torch.empty((n_queries, k), dtype=torch.int32, device=dev)
        self.binned = binned
        self._binned_ready = False
        if binned is None:
            ws = pm.sign_workspace_size(n_queries, self.cfg)
        else:
            ws = pm.sign_binned_workspace_size(n_queries, k, cap, binned["horizon"], binned["bin_bits"], self.cfg)
        self.ws_sign = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.keys = torch.empty((n_queries, bands), dtype=torch.int64, device=dev)
        self.cand_off = torch.empty(n_queries + 1, dtype=torch.int64, device=dev)
        self.cand_ids = torch.empty(cand_cap, dtype=torch.int32, device=dev)
        self.cand_j = torch.empty(cand_cap, dtype=torch.float64, device=dev)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws_query = torch.empty(int(pm.lib().polymh_query_workspace_size(D.n, n_queries)),
                                    dtype=torch.uint8, device=dev)
        self.ws_refine = pm.refine_workspace(dev)
        self.top_ids = torch.empty((n_queries, topk), dtype=torch.int32, device=dev)
        self.top_j = torch.empty((n_queries, topk), dtype=torch.float64, device=dev)
        self.stream = torch.cuda.Stream()
        self.graph = None

    def load(self, polys):
        """Copy a batch of exactly n_queries polygons into the device buffers."""
        assert polys.n == self.nq, "a batch has a fixed number of queries"
        nv = polys.xy.shape[0]
        assert nv <= self.xy.shape[0], "batch has more vertices than the buffer holds"
        self.xy[:nv].copy_(torch.from_numpy(np.ascontiguousarray(polys.xy, dtype=np.int32)), non_blocking=False)
        self.off.copy_(torch.from_numpy(np.ascontiguousarray(polys.offsets, dtype=np.int64)))

    def _issue(self):
        s = torch.cuda.current_stream()
        if self.binned is None:
            pm.sign(self.Q, self.box, self.seed, self.k, self.cap, config=self.cfg, out=self.sig,
                    ws=self.ws_sign, stream=s)
        else:
            # the samples are binned by the first run only: they depend on
            # none of the query polygons
            b = self.binned
            pm.sign_binned(self.Q, self.box, self.seed, self.k, self.cap, horizon=b["horizon"],
                           bin_bits=b["bin_bits"], walk_ratio=b.get("walk_ratio", 300.0), config=self.cfg,
                           out=self.sig, ws=self.ws_sign, stream=s, rebin=not self._binned_ready)
            self._binned_ready = True
        pm.band(self.sig, self.bands, self.rows, self.seed, out=self.keys, stream=s)
        pm.query_capped(self.sk, self.se, self.D.n, self.keys, self.cand_off, self.cand_ids,
                        self.overflow, self.ws_query, stream=s)
        pm.refine(self.D, self.Q, self.cand_off, self.cand_ids, out=self.cand_j, stream=s,
                  n_cand=self.cand_ids.numel(), ws=self.ws_refine)
        pm.topk(self.cand_off, self.cand_ids, self.cand_j, self.topk, stream=s,
                out=(self.top_ids, self.top_j))

    def run_eager(self):
        with torch.cuda.stream(self.stream):
            self._issue()

    def capture(self):
        pm.check_device()
        self.run_eager()                     # first run outside the graph
        self.stream.synchronize()
        self.graph = pm.capture(self._issue, self.stream)
        return self.graph

    def run_graph(self):
        self.graph.launch()

    def result(self):
        self.stream.synchronize()
        if int(self.overflow.item()):
            raise RuntimeError("candidate capacity exceeded; rebuild the batch with a larger cand_cap")
        return self.top_ids, self.top_j
