"""Pins of the oracle's point-in-polygon test (Alg. 1's PnP, half-open rule).

Pins: exact cell sets of rectangles and rectilinear polygons, Pick's theorem
bounds for lattice polygons, orientation/rotation invariance, and an
independent winding-number computation away from the boundary."""
import math

import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg


def _grid(x0, y0, x1, y1):
    xs, ys = np.meshgrid(np.arange(x0, x1), np.arange(y0, y1), indexing="ij")
    return np.stack([xs.ravel(), ys.ravel()], axis=1)


def _cells(rects, pts):
    """Membership in a disjoint union of half-open rectangles [x0,x1) x [y0,y1)."""
    m = np.zeros(pts.shape[0], dtype=bool)
    for (x0, y0, x1, y1) in rects:
        m |= (pts[:, 0] >= x0) & (pts[:, 0] < x1) & (pts[:, 1] >= y0) & (pts[:, 1] < y1)
    return m


@pytest.mark.parametrize("rect", [(0, 0, 1, 1), (2, 3, 9, 4), (-5, -6, 7, 2), (10, 10, 11, 30)])
def test_rectangle_is_half_open(orc, rect):
    x0, y0, x1, y1 = rect
    P = dg.rectangle(x0, y0, x1, y1)
    pts = _grid(x0 - 3, y0 - 3, x1 + 3, y1 + 3)
    got = orc.inside_points(P, pts)
    assert np.array_equal(got, _cells([rect], pts))
    assert got.sum() == (x1 - x0) * (y1 - y0)
    # clockwise and any starting vertex give the same set
    for s in range(4):
        Q = np.roll(P[::-1], s, axis=0)
        assert np.array_equal(orc.inside_points(Q, pts), got)


RECTILINEAR = [
    # L-shape and its two-rectangle decomposition
    (np.array([[0, 0], [6, 0], [6, 2], [2, 2], [2, 5], [0, 5]]), [(0, 0, 6, 2), (0, 2, 2, 5)]),
    # staircase
    (np.array([[0, 0], [8, 0], [8, 2], [5, 2], [5, 4], [2, 4], [2, 6], [0, 6]]),
     [(0, 0, 8, 2), (0, 2, 5, 4), (0, 4, 2, 6)]),
    # U-shape with a notch from the top
    (np.array([[0, 0], [7, 0], [7, 5], [5, 5], [5, 2], [2, 2], [2, 5], [0, 5]]),
     [(0, 0, 7, 2), (0, 2, 2, 5), (5, 2, 7, 5)]),
]


@pytest.mark.parametrize("case", range(len(RECTILINEAR)))
def test_rectilinear_is_union_of_cells(orc, case):
    P, rects = RECTILINEAR[case]
    pts = _grid(-2, -2, 11, 9)
    want = _cells(rects, pts)
    for s in range(P.shape[0]):
        for Q in (np.roll(P, s, axis=0), np.roll(P[::-1], s, axis=0)):
            assert np.array_equal(orc.inside_points(Q, pts), want)
    area = sum((x1 - x0) * (y1 - y0) for (x0, y0, x1, y1) in rects)
    assert want.sum() == area == abs(orc.area2(P)) // 2


def _boundary_points(P):
    b = 0
    for i in range(P.shape[0]):
        d = P[(i + 1) % P.shape[0]] - P[i]
        b += math.gcd(int(abs(d[0])), int(abs(d[1])))
    return b


def _on_boundary(P, pts):
    on = np.zeros(pts.shape[0], dtype=bool)
    n = P.shape[0]
    for i in range(n):
        a, b = P[i].astype(np.int64), P[(i + 1) % n].astype(np.int64)
        cr = (b[0] - a[0]) * (pts[:, 1] - a[1]) - (b[1] - a[1]) * (pts[:, 0] - a[0])
        inbox = ((pts[:, 0] >= min(a[0], b[0])) & (pts[:, 0] <= max(a[0], b[0])) &
                 (pts[:, 1] >= min(a[1], b[1])) & (pts[:, 1] <= max(a[1], b[1])))
        on |= (cr == 0) & inbox
    return on


def _winding(P, pts):
    """Winding number by summing the signed angles the polygon sweeps about
    each point (valid off the boundary)."""
    a = P[None, :, :].astype(np.float64) - pts[:, None, :]
    b = np.roll(P, -1, axis=0)[None, :, :].astype(np.float64) - pts[:, None, :]
    cr = a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    dt = (a * b).sum(-1)
    return np.rint(np.arctan2(cr, dt).sum(axis=1) / (2 * math.pi)).astype(int)


def test_pick_bounds_and_winding_on_random_polygons(orc):
    rng = np.random.default_rng(3)
    for t in range(40):
        n = int(rng.integers(3, 14))
        ps = dg.star_polygons(rng, [n], [[20, 20]], [float(rng.uniform(4, 18))])
        P = ps.xy.astype(np.int64)
        if t % 2:
            P = P[::-1]
        pts = _grid(0, 0, 41, 41)
        got = orc.inside_points(P, pts)
        A2 = abs(orc.area2(P))
        B = _boundary_points(P)
        I2 = A2 - B + 2            # Pick: A = I + B/2 - 1
        assert I2 % 2 == 0
        I = I2 // 2
        on = _on_boundary(P, pts)
        assert on.sum() == B
        assert I <= got.sum() <= I + B
        off = ~on
        assert np.array_equal(got[off], _winding(P, pts[off]) != 0)
        assert got[off].sum() == I


def test_triangles_pick(orc):
    rng = np.random.default_rng(11)
    for _ in range(60):
        P = rng.integers(-12, 13, (3, 2))
        A2 = abs(orc.area2(P))
        if A2 == 0:
            continue
        pts = _grid(-13, -13, 14, 14)
        got = orc.inside_points(P, pts)
        B = _boundary_points(P)
        I = (A2 - B + 2) // 2
        assert I <= got.sum() <= I + B


def test_collinear_polygon_is_empty(orc):
    P = np.array([[0, 0], [4, 2], [8, 4], [2, 1]])
    pts = _grid(-2, -2, 11, 7)
    assert not orc.inside_points(P, pts).any()
