"""Pins of the ring-shape oracle (polygons with holes, multipolygons):
closed forms, laws of the paper that hold for any shape, and agreement
with the single-ring oracle where a shape has one ring."""
import numpy as np
import pytest

from oracle import rings as orr
from paper_2511_16576_amd import datagen as dg


def sq(x0, y0, x1, y1, cw=False):
    r = dg.rectangle(x0, y0, x1, y1)
    return r[::-1] if cw else r


HOLED = [sq(0, 0, 10, 10), sq(3, 3, 7, 7, cw=True)]


def test_holed_square_area_and_membership(orc):
    assert orr.area2_rings(HOLED) == 2 * (100 - 16)
    assert not orr.inside_rings(HOLED, 5, 5)        # in the hole
    assert orr.inside_rings(HOLED, 1, 1) and orr.inside_rings(HOLED, 8, 5)
    assert not orr.inside_rings(HOLED, 12, 5)
    g = np.stack(np.meshgrid(np.arange(-2, 13), np.arange(-2, 13)), -1).reshape(-1, 2)
    assert int(orr.inside_points_rings(HOLED, g).sum()) == 100 - 16
    assert int(orr.inside_points_rings([sq(0, 0, 10, 10)], g).sum()) == 100


def test_intersections_closed_form(orc):
    assert orr.intersection_area_rings(HOLED, [sq(5, 0, 15, 10)]) == pytest.approx(50 - 8)
    assert orr.intersection_area_rings(HOLED, [sq(4, 4, 6, 6)]) == pytest.approx(0.0)
    assert orr.intersection_area_rings(HOLED, HOLED) == pytest.approx(84.0)
    # reversing every ring (holes then counter-clockwise) is the same shape
    rev = [r[::-1] for r in HOLED]
    assert orr.intersection_area_rings(rev, [sq(5, 0, 15, 10)]) == pytest.approx(42.0)
    assert orr.jaccard_rings(HOLED, HOLED) == pytest.approx(1.0)
    assert orr.jaccard_rings(HOLED, [sq(0, 0, 10, 10)]) == pytest.approx(84 / 100)
    multi = [sq(0, 0, 10, 10), sq(20, 0, 30, 10)]
    assert orr.jaccard_rings(multi, [sq(0, 0, 10, 10)]) == pytest.approx(0.5)
    assert orr.area2_rings(multi) == 400


def test_centroid_of_off_centre_hole():
    # (1e6 * 500 - 4e4 * 700) / 96e4 = 491.67 -> 492 on both axes
    shape = [sq(0, 0, 1000, 1000), sq(600, 600, 800, 800, cw=True)]
    assert orr.centroid_shift_rings(shape) == (492, 492)
    assert orr.centroid_shift_rings([sq(0, 0, 1000, 1000)]) == (500, 500)
    # two equal squares: the midpoint between their centres
    assert orr.centroid_shift_rings([sq(0, 0, 10, 10), sq(20, 0, 30, 10)]) == (15, 5)


def test_single_ring_shapes_match_the_oracle_walk(orc):
    rng = np.random.default_rng(3)
    ps = dg.star_polygons(rng, [12, 20, 7], [[300, 300], [600, 500], [200, 800]], [150.0, 250.0, 90.0])
    rs = dg.from_rings([[ps.poly(p)] for p in range(ps.n)])
    box = (0, 0, 1023, 1023)
    assert np.array_equal(orr.sign_rings(rs, box, 5, 8, 1 << 14), orc.sign(ps, box, 5, 8, 1 << 14))


def test_union_law_and_holes(orc):
    rng = np.random.default_rng(4)
    a = dg.star_polygons(rng, [10], [[200, 200]], [120.0]).xy
    b = dg.star_polygons(rng, [14], [[700, 650]], [180.0]).xy
    hole = sq(180, 180, 220, 220, cw=True)
    rs = dg.from_rings([[a], [b], [a, b], [a, hole]])
    box, k, cap = (0, 0, 1023, 1023), 24, 1 << 15
    s = orr.sign_rings(rs, box, 9, k, cap).astype(np.int64)
    inf = np.where(s == 0, cap + 1, s)
    # h(A u B) = min(h(A), h(B)) for disjoint components
    assert np.array_equal(inf[2], np.minimum(inf[0], inf[1]))
    # a hole can only delay the first hit, and does so exactly when A's first
    # hit lies in it
    keys = orc.hash_keys(9, k)
    assert (inf[3] >= inf[0]).all()
    for i in range(k):
        pt = orc.sample_points(box, int(keys[i]), int(s[0, i]))[-1]
        in_hole = orc.inside(sq(180, 180, 220, 220), int(pt[0]), int(pt[1]))
        assert (inf[3, i] == inf[0, i]) == (not in_hole)


def test_collision_rate_is_lattice_jaccard(orc):
    # Thm. 1 on a holed shape against its outer ring: in a 16 x 16 box the
    # lattice sets have 84 and 100 points, the first inside the second
    rs = dg.from_rings([HOLED, [sq(0, 0, 10, 10)]])
    s = orr.sign_rings(rs, (0, 0, 15, 15), 1, 2000, 1 << 12)
    rate = float((s[0] == s[1]).mean())
    assert abs(rate - 0.84) < 4 * np.sqrt(0.84 * 0.16 / 2000)


def test_ring_generator_shapes(orc):
    # the generator's shapes meet the ring format's conditions: filled rings
    # counter-clockwise, holes clockwise and strictly inside exactly one
    # filled ring of their shape, components apart
    rng = np.random.default_rng(12)
    rs = dg.ring_polygons(rng, 60, 18, lambda r, m: r.integers(6, 30, m), 0.03, 0.1)
    assert rs.n == 60 and rs.poly_rings[-1] == rs.ring_offsets.shape[0] - 1
    for p in range(rs.n):
        rings = rs.rings(p)
        filled = [r for r in rings if orc.area2(r) > 0]
        holes = [r for r in rings if orc.area2(r) < 0]
        assert 1 <= len(filled) <= 2 and len(filled) + len(holes) == len(rings)
        for h in holes:
            inside = [bool(orc.inside_points(f, h).all()) for f in filled]
            assert sum(inside) == 1
        if len(filled) == 2:
            a, b = filled
            assert a[:, 0].max() < b[:, 0].min() or b[:, 0].max() < a[:, 0].min()
        assert orr.area2_rings(rings) > 0
