"""Pins of the oracle's Alg. 1 signatures (Def. 2, Thm. 1, Thm. 2, Fig. 2)."""
import math

import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

BIG_CAP = 1 << 30


def _rect_set(rects):
    return dg.from_list([dg.rectangle(*r) for r in rects])


def test_geometric_law_thm2(orc):
    # Thm. 2: h is geometric with p = S_p = area(P)/area(B); on the lattice
    # the half-open rectangle covers exactly its area in cells, so p is exact.
    box = (0, 0, 1023, 1023)
    P = _rect_set([(100, 200, 164, 232)])          # 64 x 32 = 2048 cells
    p = 2048 / (1024 * 1024)
    k = 4096
    h = orc.sign(P, box, seed=1, k=k, cap=BIG_CAP)[0].astype(np.float64)
    assert (h > 0).all()
    mean, var = 1 / p, (1 - p) / p ** 2
    assert abs(h.mean() - mean) < 5 * math.sqrt(var / k)
    assert abs(h.var() / var - 1) < 0.25
    # distribution function at a few points: P(h <= t) = 1 - (1-p)^t
    for t in (64, 256, 512, 1024, 2048):
        emp = (h <= t).mean()
        th = 1 - (1 - p) ** t
        assert abs(emp - th) < 5 * math.sqrt(th * (1 - th) / k) + 1e-9


@pytest.mark.parametrize("pair", [
    ((0, 0, 40, 40), (20, 10, 60, 50)),     # J = 600/2600
    ((0, 0, 40, 40), (4, 0, 44, 40)),       # J = 1440/1760
    ((10, 10, 50, 50), (20, 20, 30, 30)),   # nested: J = 100/1600
    ((0, 0, 40, 40), (60, 60, 70, 70)),     # disjoint: J = 0
])
def test_collision_rate_is_jaccard_thm1(orc, pair):
    a, b = pair
    inter = max(0, min(a[2], b[2]) - max(a[0], b[0])) * max(0, min(a[3], b[3]) - max(a[1], b[1]))
    area = lambda r: (r[2] - r[0]) * (r[3] - r[1])
    J = inter / (area(a) + area(b) - inter)
    k = 4096
    sig = orc.sign(_rect_set([a, b]), (0, 0, 255, 255), seed=3, k=k, cap=BIG_CAP)
    assert (sig > 0).all()
    rate = (sig[0] == sig[1]).mean()
    assert abs(rate - J) <= 5 * math.sqrt(max(J * (1 - J), 1e-4) / k)


def _first_hit(orc, box, key, member, cap):
    """1 + first j whose sample lies in the known cell set, else 0."""
    pts = orc.sample_points(box, key, cap)
    hit = np.flatnonzero(member(pts))
    return int(hit[0]) + 1 if hit.size else 0


@pytest.mark.parametrize("rects", [
    [(2, 3, 9, 7)],
    [(0, 0, 6, 2), (0, 2, 2, 5)],            # L-shape as two rectangles
    [(0, 0, 16, 1)],
    [(5, 5, 6, 6)],
])
def test_first_hit_against_known_cells(orc, rects):
    box = (0, 0, 15, 15)
    polys = {1: dg.rectangle(*rects[0]),
             2: np.array([[0, 0], [6, 0], [6, 2], [2, 2], [2, 5], [0, 5]])}
    P = polys[len(rects)] if len(rects) == 2 else dg.rectangle(*rects[0])

    def member(pts):
        m = np.zeros(pts.shape[0], dtype=bool)
        for (x0, y0, x1, y1) in rects:
            m |= (pts[:, 0] >= x0) & (pts[:, 0] < x1) & (pts[:, 1] >= y0) & (pts[:, 1] < y1)
        return m

    k, cap = 24, 3000
    keys = orc.hash_keys(42, k)
    for use_mbr in (True, False):
        sig = orc.sign(dg.from_list([P]), box, seed=42, k=k, cap=cap, use_mbr=use_mbr)[0]
        want = [_first_hit(orc, box, int(keys[i]), member, cap) for i in range(k)]
        assert sig.tolist() == want


def test_fig2_counts_attempts_from_one(orc):
    # Fig. 2: the 6th sampled point is the first inside P, so MinHash(P) = 6.
    box = (0, 0, 1023, 1023)
    key = int(orc.hash_keys(0, 1)[0])
    pts = orc.sample_points(box, key, 6)
    x, y = pts[5]
    assert not any((pts[j] == pts[5]).all() for j in range(5))
    P = dg.from_list([dg.rectangle(x, y, x + 1, y + 1)])
    assert orc.sign(P, box, seed=0, k=1, cap=BIG_CAP)[0, 0] == 6


def test_union_law_and_nesting(orc):
    # Disjoint cell sets A, B with A u B = R: h(R) = min(h(A), h(B)) per hash.
    box = (0, 0, 127, 127)
    R, A, B, C = (10, 20, 50, 40), (10, 20, 27, 40), (27, 20, 50, 40), (15, 25, 20, 30)
    sig = orc.sign(_rect_set([R, A, B, C]), box, seed=9, k=256, cap=BIG_CAP).astype(np.int64)
    assert np.array_equal(sig[0], np.minimum(sig[1], sig[2]))
    assert (sig[0] <= sig[3]).all()       # C inside R hits no earlier than R


def test_mbr_filter_never_changes_result(orc):
    w = dg.workload(1, n=40, n_queries=0)
    a = orc.sign(w.data, w.box, 0, 16, 1 << 20, use_mbr=True)
    b = orc.sign(w.data, w.box, 0, 16, 1 << 20, use_mbr=False)
    assert np.array_equal(a, b)


def test_cap_sentinel_and_prefix(orc):
    w = dg.workload(1, n=30, n_queries=0)
    full = orc.sign(w.data, w.box, 0, 32, 1 << 24)
    assert (full > 0).all()
    for cap in (1, 7, 64):
        s = orc.sign(w.data, w.box, 0, 32, cap)
        assert np.array_equal(s, np.where(full <= cap, full, 0))
    # the first hashes do not depend on how many are asked for
    assert np.array_equal(orc.sign(w.data, w.box, 0, 12, 1 << 24), full[:, :12])


def test_translation_invariance(orc):
    w = dg.workload(1, n=10, n_queries=0)
    box = w.box
    s0 = orc.sign(w.data, box, 5, 16, 1 << 22)
    d = np.array([-123456, 98765], dtype=np.int32)
    moved = dg.PolySet(w.data.xy + d, w.data.offsets, w.data.centre, w.data.radius)
    box2 = (box[0] + d[0], box[1] + d[1], box[2] + d[0], box[3] + d[1])
    assert np.array_equal(orc.sign(moved, box2, 5, 16, 1 << 22), s0)


def test_degenerate_polygons_sign_zero(orc):
    polys = dg.from_list([np.zeros((0, 2)), [[1, 1]], [[1, 1], [5, 5]],
                          [[0, 0], [4, 2], [8, 4], [2, 1]],   # collinear: empty interior
                          dg.rectangle(0, 0, 1, 1)])
    s = orc.sign(polys, (0, 0, 15, 15), 0, 8, 5000)
    assert (s[:4] == 0).all()
    assert (s[4] > 0).all()
