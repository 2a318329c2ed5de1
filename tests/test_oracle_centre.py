"""Pins of the centring oracle (Sec. 3.1) against closed forms."""
import math

import numpy as np
import pytest

from oracle import centre as oc
from paper_2511_16576_amd import datagen as dg


def _half_up(num, den):
    """floor(num / den + 1/2) for integers (exact)."""
    return math.floor(num / den + 0.5) if abs(num) < 2 ** 40 else (2 * num + den) // (2 * den)


@pytest.mark.parametrize("x0,y0,x1,y1", [(0, 0, 10, 4), (3, -7, 8, 2), (-9, -9, -2, 5), (1, 1, 2, 2),
                                         (-5, 0, 4, 7)])
def test_rectangle_centroid_closed_form(x0, y0, x1, y1):
    r = dg.rectangle(x0, y0, x1, y1)
    want = (_half_up(x0 + x1, 2), _half_up(y0 + y1, 2))
    for ring in (r, r[::-1], np.roll(r, 1, axis=0), np.roll(r[::-1], 2, axis=0)):
        assert oc.centroid_shift(ring) == want


@pytest.mark.parametrize("tri", [[(0, 0), (9, 0), (0, 6)], [(-4, 1), (7, 3), (2, 11)],
                                 [(5, 5), (-3, 8), (1, -6)]])
def test_triangle_centroid_is_vertex_mean(tri):
    sx = sum(v[0] for v in tri)
    sy = sum(v[1] for v in tri)
    want = (_half_up(sx, 3), _half_up(sy, 3))
    assert oc.centroid_shift(np.array(tri)) == want
    assert oc.centroid_shift(np.array(tri[::-1])) == want


def test_l_shape_is_area_weighted_mean_of_rectangles():
    # L = [0,6]x[0,2] union [0,2]x[2,8]: areas 12 and 12, centres (3,1) and (1,5)
    L = np.array([(0, 0), (6, 0), (6, 2), (2, 2), (2, 8), (0, 8)])
    # exact centroid (2, 3); shift it off the lattice by scaling: 3L has centroid (6, 9)
    assert oc.centroid_shift(L) == (2, 3)
    L2 = np.array([(0, 0), (7, 0), (7, 2), (2, 2), (2, 9), (0, 9)])
    # areas 14 (centre (3.5, 1)) and 14 (centre (1, 5.5)): centroid (2.25, 3.25)
    assert oc.centroid_shift(L2) == (2, 3)


def test_translation_equivariance_and_identical_centred_rings():
    rng = np.random.default_rng(0)
    ps = dg.star_polygons(rng, [12, 40, 9], [[500, 700], [-300, 200], [10, -4000]], [120.0, 900.0, 50.0])
    for p in range(ps.n):
        P = ps.poly(p).astype(np.int64)
        s = oc.centroid_shift(P)
        for t in [(1, 0), (-7, 3), (123456, -98765), (-2 ** 20, 2 ** 21 + 1)]:
            st = oc.centroid_shift(P + np.array(t))
            assert st == (s[0] + t[0], s[1] + t[1])
            assert np.array_equal(P - np.array(s), (P + np.array(t)) - np.array(st))


def test_degenerate_polygons_are_not_moved():
    assert oc.centroid_shift(np.array([(1, 1), (5, 5)])) == (0, 0)
    assert oc.centroid_shift(np.array([(0, 0), (4, 2), (8, 4)])) == (0, 0)


def test_translate_has_identical_signatures_after_centring(orc):
    rng = np.random.default_rng(3)
    base = dg.star_polygons(rng, [24, 60], [[2000, 2000], [5000, 3000]], [400.0, 900.0])
    moved = dg.from_list([base.poly(0) + np.array([313, -77]), base.poly(1) + np.array([-1500, 2222])])
    both = dg.concat([base, moved])
    xy, _ = oc.centre(both)
    cen = dg.PolySet(xy, both.offsets, both.centre, both.radius)
    # every centred polygon lies in a box around the origin
    box = np.array([-2048, -2048, 2047, 2047], dtype=np.int32)
    sig = orc.sign(cen, box, 0, 32, 1 << 20)
    assert np.array_equal(sig[0], sig[2]) and np.array_equal(sig[1], sig[3])
    assert np.array_equal(cen.poly(0), cen.poly(2)) and abs(orc.jaccard(cen.poly(0), cen.poly(2)) - 1.0) < 1e-12
    assert orc.jaccard(both.poly(0), both.poly(2)) < 1.0
