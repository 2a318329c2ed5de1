"""Pins of the oracle's exact Jaccard (Sec. 1: intersection area over union area)."""
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import ConvexHull

from paper_2511_16576_amd import datagen as dg


def _rect(r):
    return dg.rectangle(*r)


@pytest.mark.parametrize("a,b", [
    ((0, 0, 10, 5), (5, 2, 20, 9)),
    ((0, 0, 10, 10), (0, 0, 10, 10)),
    ((0, 0, 10, 10), (10, 0, 20, 10)),     # touching edge: area 0
    ((0, 0, 10, 10), (30, 30, 40, 40)),
    ((0, 0, 100, 100), (20, 30, 40, 90)),  # nested
    ((-5, -5, 5, 5), (-20, -1, 20, 1)),    # cross
])
def test_rectangles_closed_form(orc, a, b):
    inter = max(0, min(a[2], b[2]) - max(a[0], b[0])) * max(0, min(a[3], b[3]) - max(a[1], b[1]))
    ua = (a[2] - a[0]) * (a[3] - a[1]) + (b[2] - b[0]) * (b[3] - b[1]) - inter
    P, Q = _rect(a), _rect(b)
    for PP in (P, P[::-1], np.roll(P, 1, axis=0)):
        for QQ in (Q, Q[::-1], np.roll(Q, 3, axis=0)):
            assert orc.intersection_area(PP, QQ) == pytest.approx(inter, abs=1e-9)
            assert orc.intersection_area_exact(PP, QQ) == inter
            assert orc.jaccard(PP, QQ) == pytest.approx(inter / ua, abs=1e-15)


def test_self_intersection_is_shoelace_and_j_is_one(orc):
    w = dg.workload(1, n=20, n_queries=0)
    for p in range(w.data.n):
        P = w.data.poly(p)
        a = abs(orc.area2(P)) / 2
        assert orc.intersection_area(P, P) == pytest.approx(a, rel=1e-12)
        assert orc.jaccard(P, P) == pytest.approx(1.0, abs=1e-12)


def _convex(rng, n, c, r):
    pts = rng.integers(-r, r + 1, (n, 2)) + c
    h = ConvexHull(pts)
    return pts[h.vertices]            # counter-clockwise hull vertices


def _inside_convex(P, pts):
    n = P.shape[0]
    ok = np.ones(pts.shape[0], dtype=bool)
    for i in range(n):
        a, b = P[i], P[(i + 1) % n]
        ok &= (b[0] - a[0]) * (pts[:, 1] - a[1]) - (b[1] - a[1]) * (pts[:, 0] - a[0]) >= -1e-9
    return ok


def _convex_intersection_area(P, Q):
    """Independent route for convex pairs: the intersection is the convex hull
    of P's vertices in Q, Q's vertices in P and all edge-edge crossings."""
    P = P.astype(np.float64)
    Q = Q.astype(np.float64)
    pts = [P[_inside_convex(Q, P)], Q[_inside_convex(P, Q)]]
    for i in range(P.shape[0]):
        a, b = P[i], P[(i + 1) % P.shape[0]]
        for j in range(Q.shape[0]):
            c, d = Q[j], Q[(j + 1) % Q.shape[0]]
            den = (b[0] - a[0]) * (d[1] - c[1]) - (b[1] - a[1]) * (d[0] - c[0])
            if den == 0:
                continue
            t = ((c[0] - a[0]) * (d[1] - c[1]) - (c[1] - a[1]) * (d[0] - c[0])) / den
            u = ((c[0] - a[0]) * (b[1] - a[1]) - (c[1] - a[1]) * (b[0] - a[0])) / den
            if 0 <= t <= 1 and 0 <= u <= 1:
                pts.append((a + t * (b - a))[None])
    pts = np.concatenate(pts)
    if pts.shape[0] < 3:
        return 0.0
    try:
        return ConvexHull(pts).volume
    except Exception:           # degenerate (collinear) intersection
        return 0.0


def test_convex_pairs_against_scipy_hull(orc):
    rng = np.random.default_rng(5)
    for _ in range(60):
        P = _convex(rng, 12, rng.integers(0, 40, 2), 20)
        Q = _convex(rng, 12, rng.integers(0, 40, 2), 20)
        want = _convex_intersection_area(P, Q)
        assert orc.intersection_area(P, Q) == pytest.approx(want, rel=1e-9, abs=1e-6)


def test_nested_and_disjoint_stars(orc):
    rng = np.random.default_rng(8)
    outer = dg.star_polygons(rng, [12], [[1000, 1000]], [800.0])
    inner = dg.star_polygons(rng, [9], [[1000, 1000]], [150.0])   # radius < 0.5*800: inside
    far = dg.star_polygons(rng, [9], [[5000, 5000]], [100.0])
    O, I, F = outer.xy, inner.xy, far.xy
    ai, ao = abs(orc.area2(I)) / 2, abs(orc.area2(O)) / 2
    assert orc.intersection_area(O, I) == pytest.approx(ai, rel=1e-12)
    assert orc.jaccard(O, I) == pytest.approx(ai / ao, rel=1e-12)
    assert orc.jaccard(O, F) == 0.0


def test_fp64_matches_exact_rationals_on_star_pairs(orc):
    rng = np.random.default_rng(2)
    for _ in range(25):
        c = rng.integers(0, 60, 2)
        P = dg.star_polygons(rng, [int(rng.integers(3, 9))], [c], [float(rng.uniform(10, 40))]).xy
        Q = dg.star_polygons(rng, [int(rng.integers(3, 9))], [c + rng.integers(-20, 21, 2)],
                             [float(rng.uniform(10, 40))]).xy
        ex = orc.intersection_area_exact(P, Q)
        assert isinstance(ex, Fraction)
        assert abs(orc.intersection_area(P, Q) - float(ex)) <= 1e-9 * float(ex) + 1e-6
        # symmetric, orientation-free
        assert orc.intersection_area_exact(Q, P[::-1]) == ex


def test_fp64_matches_exact_rationals_at_grid_scale(orc):
    """The FP64 fan clip serves as the reference of the refinement at the
    workloads' grid sizes, so pin it there too: star pairs centred anywhere
    on 2^20 and 2^24 grids, radii up to 3% of the grid (workload 5) and 20%
    (workloads 1 and 3), against exact rational areas."""
    rng = np.random.default_rng(9)
    for bits in (20, 24):
        W = 1 << bits
        for _ in range(12):
            R = float(rng.uniform(0.005, 0.2)) * W
            c = rng.integers(int(R) + 1, W - int(R) - 1, 2)
            P = dg.star_polygons(rng, [int(rng.integers(4, 10))], [c], [R]).xy
            Q = dg.star_polygons(rng, [int(rng.integers(4, 10))], [c + rng.integers(-int(R // 2), int(R // 2) + 1, 2)],
                                 [float(rng.uniform(0.5, 1.5)) * R]).xy
            assert np.abs(P).max() < W and np.abs(Q).max() < W + 2 * R
            ex = float(orc.intersection_area_exact(P, Q))
            got = orc.intersection_area(P, Q)
            assert abs(got - ex) <= 1e-9 * ex + 1e-6, (bits, got, ex)
            J = orc.jaccard(P, Q)
            ej = float(orc.jaccard_exact(P, Q))
            assert abs(J - ej) <= 1e-9 * ej + 1e-12


def test_additivity_over_a_split(orc):
    # area(P n (A u B)) = area(P n A) + area(P n B) for a rectangle split in two
    rng = np.random.default_rng(4)
    for _ in range(10):
        P = dg.star_polygons(rng, [10], [[50, 50]], [40.0]).xy
        xm = int(rng.integers(20, 80))
        R, A, B = (10, 15, 90, 85), (10, 15, xm, 85), (xm, 15, 90, 85)
        ab = orc.intersection_area_exact(P, _rect(A)) + orc.intersection_area_exact(P, _rect(B))
        assert orc.intersection_area_exact(P, _rect(R)) == ab


def test_degenerate_inputs(orc):
    P = dg.rectangle(0, 0, 4, 4)
    assert orc.jaccard(P, np.array([[0, 0], [2, 2], [4, 4]])) == 0.0
    assert orc.jaccard(P, np.array([[0, 0], [2, 2]])) == 0.0
