"""Seeded synthetic polygon workloads.

This module only produces inputs: integer-grid star-shaped simple polygons,
jittered copies and near-duplicate clusters, with the sizes and distributions
of the five workloads below.  It holds none of PolyMinHash's arithmetic (no
point stream, no point-in-polygon test, no hashing, no areas), so both the
CPU oracle and the GPU path can be fed from it.

Polygons are returned in CSR form: ``xy`` int32[V, 2] holds vertices (x, y)
and polygon p is ``xy[offsets[p]:offsets[p+1]]``; the ring is implicitly
closed and every polygon is counter-clockwise, star-shaped about its integer
centre and simple.

Workloads (all on a W x W integer grid, sampling box [0, W-1]^2, hash seed 0):

1. W=2^20, N=1,000, n ~ U{8..32}, R ~ U(0.05, 0.20) W, k=64, cap 2^20,
   16 bands x 4 rows, 10 queries that are 2%-jittered copies.
2. W=2^24, N=100,000, n = clip(round(LogNormal(ln 48, 1.0)), 8, 512),
   R ~ U(0.02, 0.15) W, k=128, cap 2^22.
3. W=2^20, N=1,000,000, n = clip(round(LogNormal(ln 48, 1.0)), 8, 1024),
   R ~ U(0.05, 0.20) W, 20% of polygons in near-duplicate clusters of size
   U{2..10} with per-cluster noise U[1%, 5%] of R, k=256, 32 x 8,
   1,000 queries (2% jitter).
4. pairs mined from workload 2's polygons (signed at k=256).
5. W=2^24, N=4,000,000, n = clip(round(8 (1 + Lomax(1.5))), 8, 8192),
   R ~ U(0.005, 0.03) W, k=256, cap 2^26, 32 x 8, 10,000 queries.

Polygons with holes and multipolygons (``ring_polygons``): a polygon is a
list of rings, filled rings counter-clockwise and holes clockwise (the OGC
convention); ``RingSet`` stores them as vertices, ring offsets and each
polygon's ring range.  Holes are stars inside the largest disc about the
outer ring's centre that the outer ring contains; a second component sits
3R away.

Stand-ins of Table 1's datasets (``table1_standin``): each dataset's
geometry count, query count and mean vertex count; star polygons on a 2^24
grid with R = 2^16 exp(N(0, 0.5^2)) clipped to [2^13, 2^19], vertex counts
max(4, round(LogNormal(ln(mean) - 0.18, 0.6))) (the 0.18 = 0.6^2 / 2 keeps
the mean near the table's), queries 2%-jittered copies of dataset members.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class PolySet:
    xy: np.ndarray        # int32 [V, 2]
    offsets: np.ndarray   # int64 [N + 1]
    centre: np.ndarray    # int64 [N, 2]  (star centre of each polygon)
    radius: np.ndarray    # float64 [N]   (outer radius R used to draw it)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def counts(self) -> np.ndarray:
        return np.diff(self.offsets)

    def poly(self, p: int) -> np.ndarray:
        return self.xy[self.offsets[p]:self.offsets[p + 1]]

    def subset(self, ids) -> "PolySet":
        ids = np.asarray(ids, dtype=np.int64)
        cnt = self.counts()[ids]
        off = np.zeros(ids.shape[0] + 1, dtype=np.int64)
        np.cumsum(cnt, out=off[1:])
        src = np.repeat(self.offsets[ids], cnt) + (np.arange(off[-1]) - np.repeat(off[:-1], cnt))
        return PolySet(np.ascontiguousarray(self.xy[src]), off, self.centre[ids].copy(),
                       self.radius[ids].copy())


@dataclasses.dataclass
class Workload:
    name: str
    grid_bits: int
    data: PolySet
    queries: PolySet | None
    query_source: np.ndarray | None   # dataset id each query was jittered from
    k: int
    cap: int
    bands: int
    rows: int
    seed: int = 0
    cluster: np.ndarray | None = None  # cluster id per dataset polygon (-1 = none)

    @property
    def box(self):
        w = 1 << self.grid_bits
        return (0, 0, w - 1, w - 1)


def _segments(counts: np.ndarray):
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    pid = np.repeat(np.arange(counts.shape[0], dtype=np.int64), counts)
    return off, pid


def _sort_segments(a: np.ndarray, counts: np.ndarray, off: np.ndarray) -> np.ndarray:
    """Values of ``a`` sorted within each CSR segment.  Segments are grouped
    by the power of two above their length and sorted as rows of a padded
    matrix (padding +inf sorts last), which is much faster than one global
    two-key sort of the whole array."""
    out = np.empty_like(a)
    level = np.ceil(np.log2(np.maximum(counts, 1))).astype(np.int64)
    for lv in np.unique(level):
        sel = np.flatnonzero(level == lv)
        c = counts[sel]
        width = int(c.max())
        s_off, s_row = _segments(c)
        col = np.arange(s_off[-1]) - np.repeat(s_off[:-1], c)
        src = np.repeat(off[sel], c) + col
        M = np.full((sel.size, width), np.inf)
        M[s_row, col] = a[src]
        M.sort(axis=1)
        out[src] = M[s_row, col]
    return out


def _star_angles(rng, counts, stratified=False):
    """Sorted angles per polygon, redrawn until every gap is below pi.  With
    ``stratified`` angle i is (i + U(0.25, 0.75)) * 2 pi / n, which keeps every
    gap at least pi / n (used for polygons whose uniform draws keep failing
    the lattice validity check)."""
    off, pid = _segments(counts)
    ang = np.empty(off[-1])
    todo = np.arange(counts.shape[0])
    while todo.size:
        sub_cnt = counts[todo]
        sub_off, sub_pid = _segments(sub_cnt)
        if stratified:
            idx = np.arange(sub_off[-1]) - np.repeat(sub_off[:-1], sub_cnt)
            a = (idx + rng.uniform(0.25, 0.75, sub_off[-1])) * (TWO_PI / np.repeat(sub_cnt, sub_cnt))
        else:
            a = rng.random(sub_off[-1]) * TWO_PI
        a = _sort_segments(a, sub_cnt, sub_off)
        nxt = np.empty_like(a)
        nxt[:-1] = a[1:]
        last = sub_off[1:] - 1
        gaps = nxt - a
        gaps[last] = a[sub_off[:-1]] + TWO_PI - a[last]
        bad = np.maximum.reduceat(gaps, sub_off[:-1]) >= math.pi
        dst = np.repeat(off[todo], sub_cnt) + (np.arange(sub_off[-1]) - np.repeat(sub_off[:-1], sub_cnt))
        ang[dst] = a
        todo = todo[bad]
    return ang


def _star_valid(xy: np.ndarray, counts: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """Generator validity: every edge turns strictly counter-clockwise about the
    centre and the ring winds once around it.  This makes the polygon simple
    and star-shaped about its centre (input recipe only)."""
    off, pid = _segments(counts)
    v = xy.astype(np.int64)
    nxt_idx = np.arange(off[-1]) + 1
    nxt_idx[off[1:] - 1] = off[:-1]
    c = centre[pid]
    a = v - c
    b = v[nxt_idx] - c
    cr = a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]
    ok = np.minimum.reduceat(cr, off[:-1]) > 0
    turn = np.arctan2(cr.astype(np.float64), (a * b).sum(axis=1).astype(np.float64))
    wind = np.add.reduceat(turn, off[:-1])
    ok &= np.abs(wind - TWO_PI) < 1e-6
    return ok


def star_polygons(rng, counts, centres, radii, max_rounds: int = 200) -> PolySet:
    """Star-shaped simple polygons: sorted uniform angles (max gap < pi), radii
    U[0.5R, R], vertices rounded to the grid; invalid ones are redrawn, from
    the fourth draw on with stratified angles so that the loop ends."""
    counts = np.asarray(counts, dtype=np.int64)
    centres = np.asarray(centres, dtype=np.int64)
    radii = np.asarray(radii, dtype=np.float64)
    off, pid = _segments(counts)
    xy = np.empty((off[-1], 2), dtype=np.int64)
    todo = np.arange(counts.shape[0])
    for rnd in range(max_rounds):
        if todo.size == 0:
            break
        sub_cnt = counts[todo]
        sub_off, sub_pid = _segments(sub_cnt)
        ang = _star_angles(rng, sub_cnt, stratified=rnd >= 3)
        rad = rng.uniform(0.5, 1.0, sub_off[-1]) * radii[todo][sub_pid]
        c = centres[todo][sub_pid]
        sx = np.rint(c[:, 0] + rad * np.cos(ang)).astype(np.int64)
        sy = np.rint(c[:, 1] + rad * np.sin(ang)).astype(np.int64)
        sub_xy = np.stack([sx, sy], axis=1)
        ok = _star_valid(sub_xy, sub_cnt, centres[todo])
        dst = np.repeat(off[todo], sub_cnt) + (np.arange(sub_off[-1]) - np.repeat(sub_off[:-1], sub_cnt))
        xy[dst] = sub_xy
        todo = todo[~ok]
    if todo.size:
        raise ValueError(f"{todo.size} star polygons stayed invalid after {max_rounds} draws: "
                         "too many vertices for their radius on the integer grid")
    return PolySet(xy.astype(np.int32), off, centres.copy(), radii.copy())


def _edge_ok(xy: np.ndarray, counts: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """Per-edge generator check: edge v_i -> v_{i+1} turns strictly
    counter-clockwise about the polygon's centre (input recipe only)."""
    off, pid = _segments(counts)
    v = xy.astype(np.int64)
    nxt_idx = np.arange(off[-1]) + 1
    nxt_idx[off[1:] - 1] = off[:-1]
    c = centre[pid]
    a = v - c
    b = v[nxt_idx] - c
    return (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]) > 0, nxt_idx


def _edges_ok(xy: np.ndarray, edges: np.ndarray, nxt: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """``_edge_ok`` for the listed edges only (``centre`` given per edge)."""
    a = xy[edges] - centre
    b = xy[nxt[edges]] - centre
    return (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]) > 0


def jittered(rng, base: PolySet, ids, noise, grid_bits: int, max_rounds: int = 64) -> PolySet:
    """Copies of base polygons ``ids`` with every coordinate moved by
    round(U[-d, d]), d = noise * R, clipped to the grid.  The two vertices of
    any edge that stops turning counter-clockwise about the source centre are
    redrawn, so the copy stays star-shaped and simple; a copy still invalid
    after ``max_rounds`` keeps its source vertices."""
    ids = np.asarray(ids, dtype=np.int64)
    noise = np.broadcast_to(np.asarray(noise, dtype=np.float64), ids.shape)
    src = base.subset(ids)
    counts = src.counts()
    off, pid = _segments(counts)
    hi = (1 << grid_bits) - 1
    orig = src.xy.astype(np.int64)
    d = (noise * src.radius)[pid]
    out = orig.copy()
    redo = np.arange(off[-1])
    nxt = np.arange(off[-1]) + 1
    nxt[off[1:] - 1] = off[:-1]
    prv = np.arange(off[-1]) - 1
    prv[off[:-1]] = off[1:] - 1
    for rnd in range(max_rounds):
        if redo.size == 0:
            break
        j = np.rint(rng.uniform(-1.0, 1.0, (redo.size, 2)) * d[redo][:, None]).astype(np.int64)
        out[redo] = np.clip(orig[redo] + j, 0, hi)
        if rnd == 0:
            ok, _ = _edge_ok(out, counts, src.centre)
            bad = np.flatnonzero(~ok)
        else:
            # an edge with neither end redrawn kept its vertices, and it was
            # good in the last round (a bad edge has both ends redrawn)
            edges = np.unique(np.concatenate([redo, prv[redo]]))
            bad = edges[~_edges_ok(out, edges, nxt, src.centre[pid[edges]])]
        redo = np.unique(np.concatenate([bad, nxt[bad]]))
    stuck = ~_star_valid(out, counts, src.centre)
    if stuck.any():   # rare: such copies keep their source vertices
        rows = np.flatnonzero(stuck[pid])
        out[rows] = orig[rows]
    return PolySet(out.astype(np.int32), off, src.centre.copy(), src.radius.copy())


def _centres(rng, radii, grid_bits):
    w = 1 << grid_bits
    m = np.ceil(radii).astype(np.int64)
    lo = m
    hi = (w - 1) - m
    cx = lo + np.floor(rng.random(radii.shape[0]) * (hi - lo + 1)).astype(np.int64)
    cy = lo + np.floor(rng.random(radii.shape[0]) * (hi - lo + 1)).astype(np.int64)
    return np.stack([cx, cy], axis=1)


def _lognormal_counts(rng, n, cap):
    return np.clip(np.rint(np.exp(rng.normal(math.log(48.0), 1.0, n))), 8, cap).astype(np.int64)


def random_polygons(rng, n, grid_bits, count_fn, rfrac_lo, rfrac_hi) -> PolySet:
    w = float(1 << grid_bits)
    counts = count_fn(rng, n)
    radii = rng.uniform(rfrac_lo, rfrac_hi, n) * w
    centres = _centres(rng, radii, grid_bits)
    return star_polygons(rng, counts, centres, radii)


def concat(sets) -> PolySet:
    xs = [s.xy for s in sets]
    offs = [s.counts() for s in sets]
    counts = np.concatenate(offs)
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return PolySet(np.concatenate(xs), off, np.concatenate([s.centre for s in sets]),
                   np.concatenate([s.radius for s in sets]))


@dataclasses.dataclass
class RingSet:
    xy: np.ndarray           # int32 [V, 2]
    ring_offsets: np.ndarray  # int64 [R + 1]: ring r is xy[ring_offsets[r]:ring_offsets[r+1]]
    poly_rings: np.ndarray    # int64 [N + 1]: polygon p owns rings poly_rings[p]:poly_rings[p+1]

    @property
    def n(self) -> int:
        return int(self.poly_rings.shape[0] - 1)

    def rings(self, p: int):
        return [self.xy[self.ring_offsets[r]:self.ring_offsets[r + 1]]
                for r in range(int(self.poly_rings[p]), int(self.poly_rings[p + 1]))]


def from_rings(polys) -> RingSet:
    """RingSet from a list of polygons, each a list of (k, 2) rings."""
    rings = [np.asarray(r, dtype=np.int64).reshape(-1, 2) for p in polys for r in p]
    counts = np.array([r.shape[0] for r in rings], dtype=np.int64)
    roff = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=roff[1:])
    proff = np.zeros(len(polys) + 1, dtype=np.int64)
    np.cumsum([len(p) for p in polys], out=proff[1:])
    xy = np.concatenate(rings).astype(np.int32) if rings else np.zeros((0, 2), dtype=np.int32)
    return RingSet(xy, roff, proff)


def _inner_radii(ps: PolySet) -> np.ndarray:
    """Per polygon, the distance from its centre to the nearest point of its
    ring (float)."""
    off, pid = _segments(ps.counts())
    a = ps.xy.astype(np.float64) - ps.centre[pid].astype(np.float64)
    nxt = np.arange(off[-1]) + 1
    nxt[off[1:] - 1] = off[:-1]
    d = a[nxt] - a
    t = np.clip(-(a * d).sum(axis=1) / np.maximum((d * d).sum(axis=1), 1e-30), 0.0, 1.0)
    q = a + t[:, None] * d
    return np.minimum.reduceat(np.sqrt((q * q).sum(axis=1)), off[:-1])


def ring_polygons(rng, n: int, grid_bits: int, count_fn, rfrac_lo: float, rfrac_hi: float,
                  hole_probs=(0.4, 0.35, 0.25), multi_prob: float = 0.25) -> RingSet:
    """``n`` shapes: one or (with probability ``multi_prob``) two star
    components of radius R, each with 0, 1 or 2 star holes (``hole_probs``).
    One hole is centred with radius 0.8 d, two sit at +-0.5 d with radius
    0.4 d, where d is the distance from the component's centre to its outer
    ring (holes under 64 units of radius are left out); holes have 3-12
    vertices and are reversed to clockwise.  Components are 3R apart."""
    w = 1 << grid_bits
    multi = rng.random(n) < multi_prob
    R = rng.uniform(rfrac_lo, rfrac_hi, n) * w
    m = np.ceil(R).astype(np.int64)
    span = np.where(multi, 4 * m, m)
    cx = m + np.floor(rng.random(n) * (w - 1 - span - m + 1)).astype(np.int64)
    cy = m + np.floor(rng.random(n) * (w - 1 - 2 * m + 1)).astype(np.int64)
    # components: shape s has component 0, and component 1 when multi
    comp_shape = np.concatenate([np.arange(n), np.flatnonzero(multi)])
    comp_second = np.concatenate([np.zeros(n, bool), np.ones(int(multi.sum()), bool)])
    order = np.lexsort((comp_second, comp_shape))
    comp_shape, comp_second = comp_shape[order], comp_second[order]
    cc = np.stack([cx[comp_shape] + np.where(comp_second, 3 * m[comp_shape], 0), cy[comp_shape]], axis=1)
    outer = star_polygons(rng, count_fn(rng, comp_shape.shape[0]), cc, R[comp_shape])
    d = _inner_radii(outer)
    nh = rng.choice(3, size=comp_shape.shape[0], p=hole_probs)
    h_comp, h_c, h_r = [], [], []
    for k_, places in ((1, [(0.0, 0.8)]), (2, [(-0.5, 0.4), (0.5, 0.4)])):
        sel = np.flatnonzero(nh == k_)
        for fx, fr in places:
            h_comp.append(sel)
            h_c.append(np.stack([cc[sel, 0] + (fx * d[sel]).astype(np.int64), cc[sel, 1]], axis=1))
            h_r.append(fr * d[sel])
    h_comp, h_c, h_r = np.concatenate(h_comp), np.concatenate(h_c), np.concatenate(h_r)
    keep = h_r >= 64.0
    h_comp, h_c, h_r = h_comp[keep], h_c[keep], h_r[keep]
    h_order = np.lexsort((h_c[:, 0], h_comp))
    h_comp, h_c, h_r = h_comp[h_order], h_c[h_order], h_r[h_order]
    holes = star_polygons(rng, rng.integers(3, 13, h_comp.shape[0]), h_c, h_r)
    # assemble: per component its outer ring, then its holes (clockwise)
    hole_first = np.searchsorted(h_comp, np.arange(comp_shape.shape[0]), side="left")
    hole_last = np.searchsorted(h_comp, np.arange(comp_shape.shape[0]), side="right")
    rings, per_shape = [], np.zeros(n, dtype=np.int64)
    for c in range(comp_shape.shape[0]):
        rings.append(outer.poly(c))
        for h in range(hole_first[c], hole_last[c]):
            rings.append(holes.poly(h)[::-1])
        per_shape[comp_shape[c]] += 1 + hole_last[c] - hole_first[c]
    counts = np.array([r.shape[0] for r in rings], dtype=np.int64)
    roff = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=roff[1:])
    proff = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(per_shape, out=proff[1:])
    return RingSet(np.concatenate(rings).astype(np.int32), roff, proff)


# Table 1: geometries, queries, average vertex count
TABLE1 = {
    "urban": (11_800, 3_000, 95.40),
    "cemetery": (149_000, 3_000, 9.26),
    "parks": (300_000, 3_000, 319.0),
    "sports": (1_000_000, 20_000, 12.0),
}


def table1_standin(name: str, n: int | None = None, n_queries: int | None = None) -> Workload:
    """Synthetic stand-in of Table 1's dataset ``name`` (urban, cemetery,
    parks, sports); ``n`` / ``n_queries`` shrink it.  The signature length,
    tables and cap are the experiment's to choose (k, bands, rows here are
    placeholders for one 3-row table)."""
    N0, Q0, mean = TABLE1[name]
    rng = _rng(100 + list(TABLE1).index(name))
    N = N0 if n is None else n
    Q = Q0 if n_queries is None else n_queries
    gb = 24

    def counts(r, m):
        mu = math.log(mean) - 0.18
        return np.clip(np.rint(np.exp(r.normal(mu, 0.6, m))), 4, 8192).astype(np.int64)
    radii = np.clip(65536.0 * np.exp(rng.normal(0.0, 0.5, N)), 8192.0, 524288.0)
    cnt = counts(rng, N)
    data = star_polygons(rng, cnt, _centres(rng, radii, gb), radii)
    src = rng.integers(0, N, Q)
    q = jittered(rng, data, src, 0.02, gb)
    return Workload(f"table1-{name}", gb, data, q, src, k=3, cap=1 << 22, bands=1, rows=3)


def _rng(cfg: int, stream: int = 0):
    return np.random.default_rng(np.random.SeedSequence([cfg, stream]))


def workload(cfg: int, n: int | None = None, n_queries: int | None = None) -> Workload:
    """Build workload ``cfg`` (1, 2, 3 or 5).  ``n`` / ``n_queries`` shrink it
    (same distributions, fewer polygons) for tests and bounded samples."""
    rng = _rng(cfg)
    if cfg == 1:
        N = 1000 if n is None else n
        Q = 10 if n_queries is None else n_queries
        data = random_polygons(rng, N, 20, lambda r, m: r.integers(8, 33, m), 0.05, 0.20)
        src = rng.integers(0, N, Q)
        q = jittered(rng, data, src, 0.02, 20)
        return Workload("cfg1", 20, data, q, src, k=64, cap=1 << 20, bands=16, rows=4)
    if cfg == 2:
        N = 100_000 if n is None else n
        Q = 10_000 if n_queries is None else n_queries
        data = random_polygons(rng, N, 24, lambda r, m: _lognormal_counts(r, m, 512), 0.02, 0.15)
        src = rng.integers(0, N, Q)
        q = jittered(rng, data, src, 0.02, 24)
        return Workload("cfg2", 24, data, q, src, k=128, cap=1 << 22, bands=32, rows=4)
    if cfg == 3:
        N = 1_000_000 if n is None else n
        Q = 1000 if n_queries is None else n_queries
        n_clu_target = int(round(0.2 * N))
        sizes, total = [], 0
        while total < n_clu_target:
            sizes.append(int(rng.integers(2, 11)))
            total += sizes[-1]
        sizes[-1] -= total - n_clu_target
        if sizes and sizes[-1] < 1:
            sizes.pop()
        sizes = np.asarray(sizes, dtype=np.int64)
        n_base = N - int(sizes.sum()) + sizes.shape[0]
        base = random_polygons(rng, n_base, 20, lambda r, m: _lognormal_counts(r, m, 1024), 0.05, 0.20)
        # the first len(sizes) base polygons seed the clusters
        members = np.repeat(np.arange(sizes.shape[0]), sizes - 1)
        noise = rng.uniform(0.01, 0.05, sizes.shape[0])[members]
        copies = jittered(rng, base, members, noise, 20)
        data = concat([base, copies])
        cluster = np.concatenate([np.where(np.arange(n_base) < sizes.shape[0], np.arange(n_base), -1),
                                  members])
        perm = rng.permutation(data.n)
        data = data.subset(perm)
        cluster = cluster[perm]
        src = rng.integers(0, data.n, Q)
        q = jittered(rng, data, src, 0.02, 20)
        return Workload("cfg3", 20, data, q, src, k=256, cap=1 << 20, bands=32, rows=8, cluster=cluster)
    if cfg == 5:
        N = 4_000_000 if n is None else n
        Q = 10_000 if n_queries is None else n_queries

        def pareto_counts(r, m):
            return np.clip(np.rint(8.0 * (1.0 + r.pareto(1.5, m))), 8, 8192).astype(np.int64)
        data = random_polygons(rng, N, 24, pareto_counts, 0.005, 0.03)
        src = rng.integers(0, N, Q)
        q = jittered(rng, data, src, 0.02, 24)
        return Workload("cfg5", 24, data, q, src, k=256, cap=1 << 26, bands=32, rows=8)
    raise ValueError(f"no workload {cfg}")


def rectangle(x0, y0, x1, y1) -> np.ndarray:
    """Counter-clockwise axis-aligned rectangle with corners (x0,y0), (x1,y1)."""
    return np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]], dtype=np.int32)


def from_list(polys) -> PolySet:
    """CSR PolySet from a list of (n_i, 2) integer arrays."""
    polys = [np.asarray(p, dtype=np.int32).reshape(-1, 2) for p in polys]
    counts = np.array([p.shape[0] for p in polys], dtype=np.int64)
    off = np.zeros(len(polys) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    xy = np.concatenate(polys) if polys else np.zeros((0, 2), dtype=np.int32)
    cen = np.array([p.mean(axis=0) if p.shape[0] else (0, 0) for p in polys], dtype=np.int64).reshape(-1, 2)
    return PolySet(np.ascontiguousarray(xy, dtype=np.int32), off, cen,
                   np.zeros(len(polys), dtype=np.float64))
