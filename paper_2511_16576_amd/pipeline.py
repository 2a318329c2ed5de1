"""Batched query pipeline: sign -> band -> candidate lookup -> exact-Jaccard
refinement -> top-10 for a fixed-shape batch of queries, run eagerly or
captured once as a HIP graph and replayed per batch.  Every buffer is
allocated up front; the lookup has a fixed candidate capacity with a device
overflow flag, so no stage needs the host.

Three ways to refine the candidates of a batch (``method``):
  "plain"  every candidate refined, then the top-10;
  "jhat"   candidates ordered by their collision fraction (Thm. 1's estimate
           of J) and refined best-first with early stop;
  "scorer" the same order, then the learned scorer re-predicts the first
           ``head`` candidates of each query and the order is rebuilt from
           those predictions before the early-stop refinement.
The early stop runs a fixed number of rounds of F refinements per active
query on the device, then a finishing pass completes any query still
active, so the result never depends on a host read."""
from __future__ import annotations

import numpy as np
import torch

from . import polymh as pm


class QueryBatch:
    def __init__(self, D: pm.DevicePolys, sorted_keys, sorted_ent, box, seed: int, k: int, cap: int,
                 bands: int, rows: int, n_queries: int, max_vertices: int, cand_cap: int,
                 sign_config=None, topk: int = 10, binned=None, method: str = "plain", dsig=None,
                 scorer=None, dfeat=None, head: int = 32, F: int = 8, rounds: int = 4, margin: float = 0.0,
                 dpacked=None):
        """``binned``: None signs the queries by the walk; a dict with
        horizon, bin_bits and walk_ratio signs them from binned samples
        (``polymh_sign_binned``, the same bits).  ``method`` "jhat" and
        "scorer" need the data signatures ``dsig`` ([N][k]); "scorer" also
        the trained ``scorer`` (params, BF16 weights) and the data shape
        features ``dfeat``.  ``dpacked`` (``pm.sig_pack(dsig)``, optional)
        lets the collision fraction read the saturated 16-bit table of the
        data signatures (the same scores and order, half the bytes a
        candidate)."""
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
        if method not in ("plain", "jhat", "scorer"):
            raise ValueError(f"unknown method {method!r}")
        self.method = method
        self.F, self.rounds, self.margin, self.head = F, rounds, margin, head
        if method != "plain":
            if dsig is None or dsig.shape[1] != k:
                raise ValueError("ranked methods need the data signatures at the batch's k")
            self.dsig, self.dpacked = dsig, dpacked
            self.score = torch.empty(cand_cap, dtype=torch.float32, device=dev)
            self.order = torch.empty(cand_cap, dtype=torch.int32, device=dev)
            self.sorted_ok = torch.empty(n_queries, dtype=torch.uint8, device=dev)
            self.ws_rank = pm.rank_workspace(n_queries, cand_cap, F, dev)
            self.counts = torch.zeros(2, dtype=torch.int64, device=dev)
        if method == "scorer":
            if scorer is None or dfeat is None:
                raise ValueError("the scorer method needs a trained scorer and the data features")
            self.scorer, self.dfeat = scorer, dfeat
            self.qfeat = torch.empty((n_queries, 12), dtype=torch.float32, device=dev)
            if not 1 <= head <= 64:
                raise ValueError("the scorer re-scores 1 to 64 candidates per query")
            R = n_queries * head
            self.hq = torch.empty(max(R, 1), dtype=torch.int32, device=dev)
            self.hc = torch.empty(max(R, 1), dtype=torch.int64, device=dev)
            self.hid = torch.empty(max(R, 1), dtype=torch.int32, device=dev)
            self.order2 = torch.empty(cand_cap, dtype=torch.int32, device=dev)
        self.stream = torch.cuda.Stream()
        self.graph = None

    def load(self, polys):
        """Copy a batch of exactly n_queries polygons into the device buffers."""
        assert polys.n == self.nq, "a batch has a fixed number of queries"
        nv = polys.xy.shape[0]
        assert nv <= self.xy.shape[0], "batch has more vertices than the buffer holds"
        self.xy[:nv].copy_(torch.from_numpy(np.ascontiguousarray(polys.xy, dtype=np.int32)), non_blocking=False)
        self.off.copy_(torch.from_numpy(np.ascontiguousarray(polys.offsets, dtype=np.int64)))

    def _issue(self, mark=None):
        """Enqueue the batch on the current stream; ``mark(name)``, if given,
        is called after each stage (an instrumented eager run records an
        event there)."""
        mark = mark or (lambda name: None)
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
        mark("qsign")
        pm.band(self.sig, self.bands, self.rows, self.seed, out=self.keys, stream=s)
        mark("qband")
        pm.query_capped(self.sk, self.se, self.D.n, self.keys, self.cand_off, self.cand_ids,
                        self.overflow, self.ws_query, stream=s)
        mark("lookup")
        if self.method == "plain":
            pm.refine(self.D, self.Q, self.cand_off, self.cand_ids, out=self.cand_j, stream=s,
                      n_cand=self.cand_ids.numel(), ws=self.ws_refine)
            mark("refine")
            pm.topk(self.cand_off, self.cand_ids, self.cand_j, self.topk, stream=s,
                    out=(self.top_ids, self.top_j))
            mark("topk")
            return
        pm.rank_jhat_order(self.sig, self.dsig, self.cand_off, self.cand_ids, score=self.score, order=self.order,
                           sorted_ok=self.sorted_ok, stream=s, packed=self.dpacked)
        mark("jhat_order")
        order = self.order
        if self.method == "scorer":
            # the network re-predicts the first `head` candidates of each
            # query (one fused launch writes into their scores), and the
            # order is rebuilt by merging them back into the rest
            sc = self.scorer
            pm.rank_head_fixed(self.cand_off, self.cand_ids, self.order, self.head,
                               out=(self.hq, self.hc, self.hid), stream=s)
            pm.poly_features(self.Q, self.box, out=self.qfeat, stream=s)
            mark("head")
            pm.mlp_score_pairs(self.sig, self.qfeat, self.dsig, self.dfeat, self.hq, self.hid, sc.params,
                               sc.wbf16, out=self.score, out_idx=self.hc, stream=s)
            mark("scorer")
            pm.rank_reorder_head(self.cand_off, self.score, self.order, self.head, self.sorted_ok, self.order2,
                                 stream=s)
            order = self.order2
            mark("reorder")
        pm.rank_refine_ordered(self.D, self.Q, self.cand_off, self.cand_ids, self.score, order,
                               self.sorted_ok, topk=self.topk, F=self.F, rounds=self.rounds, margin=self.margin,
                               ws=self.ws_rank, out=(self.top_ids, self.top_j), counts=self.counts, stream=s)
        mark("rank_refine")

    def run_eager(self):
        with torch.cuda.stream(self.stream):
            self._issue()

    def run_instrumented(self) -> dict:
        """One eager run with a HIP event on the batch's stream after every
        stage: milliseconds per stage."""
        evs = []

        def mark(name):
            e = torch.cuda.Event(enable_timing=True)
            e.record(self.stream)
            evs.append((name, e))
        with torch.cuda.stream(self.stream):
            mark("start")
            self._issue(mark)
        self.stream.synchronize()
        return {evs[i][0]: evs[i - 1][1].elapsed_time(evs[i][1]) for i in range(1, len(evs))}

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


def _spread_bits16(v: np.ndarray) -> np.ndarray:
    """Bits 0..15 of v moved to the even positions 0, 2, .., 30."""
    v = v.astype(np.uint64) & np.uint64(0xFFFF)
    for shift, mask in ((8, 0x00FF00FF), (4, 0x0F0F0F0F), (2, 0x33333333), (1, 0x55555555)):
        v = (v | (v << np.uint64(shift))) & np.uint64(mask)
    return v


def spatial_order(polys) -> np.ndarray:
    """A permutation of a polygon set along the Z-order (Morton) curve of its
    MBR centres, quantised to 16 bits a side over the set's extent (stable:
    equal keys keep their given order; polygons without vertices first).
    Queries close along the curve are close in space and share many of their
    candidates, so a batch run in this order reads the data polygons'
    signature rows and vertices from the caches more often."""
    off = np.asarray(polys.offsets, dtype=np.int64)
    xy = np.asarray(polys.xy).reshape(-1, 2).astype(np.int64)
    n = off.shape[0] - 1
    cnt = off[1:] - off[:-1]
    live = cnt > 0
    cx = np.zeros(n, dtype=np.int64)
    cy = np.zeros(n, dtype=np.int64)
    if live.any():
        st = off[:-1][live]
        cx[live] = (np.minimum.reduceat(xy[:, 0], st) + np.maximum.reduceat(xy[:, 0], st)) // 2
        cy[live] = (np.minimum.reduceat(xy[:, 1], st) + np.maximum.reduceat(xy[:, 1], st)) // 2
    key = np.zeros(n, dtype=np.uint64)
    if live.any():
        q = []
        for c in (cx, cy):
            lo, hi = c[live].min(), c[live].max()
            q.append(((c - lo) * 65535 // max(int(hi - lo), 1)).clip(0, 65535))
        key[live] = (_spread_bits16(q[0]) | (_spread_bits16(q[1]) << np.uint64(1)))[live] + np.uint64(1)
    return np.argsort(key, kind="stable")


class SplitBatch:
    """A batch of ``n_queries`` queries run as ``parts`` sub-batches of
    consecutive queries, each a ``QueryBatch`` with its own buffers and
    stream.  The captured graph forks from the first part's stream onto the
    others with events and joins back, so the parts' kernels run
    concurrently: a part's stages are bound by different things (latency
    chains and their tails in the signing, the lookup's sorts and the
    refinement rounds; HBM in the collision-fraction order), and the other
    parts' work fills the gaps.  Every query's result is the one the whole
    batch gives (the stages treat queries independently); ``result`` and
    ``counts`` concatenate and add the parts'."""

    def __init__(self, D, sorted_keys, sorted_ent, box, seed, k, cap, bands, rows, n_queries, max_vertices,
                 cand_cap, parts: int = 4, query_order: str = "given", **kw):
        """``query_order`` "morton" runs the batch's queries in the
        ``spatial_order`` of the set ``load`` is given (the parts are then
        stretches of the curve); ``result`` returns them in the given order
        either way."""
        if not 1 <= parts <= n_queries:
            raise ValueError("parts must be between 1 and the number of queries")
        if query_order not in ("given", "morton"):
            raise ValueError("query_order must be 'given' or 'morton'")
        self.query_order, self.perm = query_order, None
        cuts = np.linspace(0, n_queries, parts + 1).round().astype(np.int64)
        self.bounds = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:])]
        self.parts = [QueryBatch(D, sorted_keys, sorted_ent, box, seed, k, cap, bands, rows, b - a, max_vertices,
                                 cand_cap, **kw) for a, b in self.bounds]
        self.nq, self.method = n_queries, self.parts[0].method
        self.stream = self.parts[0].stream
        self.graph = None

    # early-stop parameters, set on every part
    def _get(self, name):
        return getattr(self.parts[0], name)

    def _set(self, name, v):
        for p in self.parts:
            setattr(p, name, v)

    F = property(lambda self: self._get("F"), lambda self, v: self._set("F", v))
    rounds = property(lambda self: self._get("rounds"), lambda self, v: self._set("rounds", v))
    margin = property(lambda self: self._get("margin"), lambda self, v: self._set("margin", v))

    def load(self, polys):
        assert polys.n == self.nq, "a batch has a fixed number of queries"
        self.perm = spatial_order(polys) if self.query_order == "morton" else None
        src = polys if self.perm is None else polys.subset(self.perm)
        for p, (a, b) in zip(self.parts, self.bounds):
            p.load(src.subset(np.arange(a, b)))

    def _wait_all(self):
        for p in self.parts:
            p.stream.synchronize()

    def run_eager(self):
        for p in self.parts:
            with torch.cuda.stream(p.stream):
                p._issue()
        self._wait_all()

    def run_instrumented(self) -> dict:
        """The parts run one after another with events after every stage:
        each stage's milliseconds summed over the parts (GPU time, not the
        concurrent replay's wall time); the parts' own tables are kept in
        ``parts_stage_ms``."""
        self.parts_stage_ms = [p.run_instrumented() for p in self.parts]
        tot = {}
        for st in self.parts_stage_ms:
            for name, ms in st.items():
                tot[name] = tot.get(name, 0.0) + ms
        return tot

    def capture(self):
        pm.check_device()
        self.run_eager()                     # first run outside the graph
        s0 = self.stream

        def issue():
            fork = torch.cuda.Event()
            fork.record(s0)
            for p in self.parts[1:]:
                p.stream.wait_event(fork)
            for p in self.parts:
                with torch.cuda.stream(p.stream):
                    p._issue()
            for p in self.parts[1:]:
                join = torch.cuda.Event()
                join.record(p.stream)
                s0.wait_event(join)
        self.graph = pm.capture(issue, s0)
        return self.graph

    def run_graph(self):
        self.graph.launch()

    def result(self):
        res = [p.result() for p in self.parts]
        ids, js = torch.cat([r[0] for r in res]), torch.cat([r[1] for r in res])
        if self.perm is not None:
            # row r holds query perm[r]: back to the given order
            inv = torch.from_numpy(np.argsort(self.perm)).to(ids.device)
            ids, js = ids[inv], js[inv]
        return ids, js

    @property
    def counts(self):
        return sum(p.counts for p in self.parts)
