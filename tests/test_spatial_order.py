"""The spatial order of a query batch (host side, no GPU): a permutation
along the Z-order curve of the polygons' MBR centres."""
import numpy as np

from paper_2511_16576_amd import datagen as dg
from paper_2511_16576_amd.pipeline import spatial_order


def _grid(nx, ny, step=10, size=2):
    return [dg.rectangle(step * x, step * y, step * x + size, step * y + size) for y in range(ny) for x in range(nx)]


def test_grid_follows_the_z_curve():
    # a 4 x 4 grid of squares, index y * 4 + x: the curve takes the four
    # 2 x 2 quadrants in the order (0,0) (1,0) (0,1) (1,1), x before y at
    # every level
    got = spatial_order(dg.from_list(_grid(4, 4)))
    want = [0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15]
    assert got.tolist() == want


def test_order_is_a_permutation_and_ignores_translation_and_scale():
    rng = np.random.default_rng(5)
    w = dg.workload(2, n=500, n_queries=300)
    o = spatial_order(w.queries)
    assert np.array_equal(np.sort(o), np.arange(300))
    moved = dg.from_list([w.queries.xy[a:b] * 2 + np.array([1000, -700]) for a, b in
                          zip(w.queries.offsets[:-1], w.queries.offsets[1:])])
    assert np.array_equal(spatial_order(moved), o)
    # the curve keeps neighbours together: consecutive queries are far
    # closer than random pairs
    c = np.array([(p[:, 0].min() + p[:, 0].max(), p[:, 1].min() + p[:, 1].max())
                  for p in (w.queries.xy[a:b] for a, b in zip(w.queries.offsets[:-1], w.queries.offsets[1:]))],
                 dtype=np.float64) / 2
    step = np.linalg.norm(np.diff(c[o], axis=0), axis=1).mean()
    rand = np.linalg.norm(c[rng.permutation(300)] - c, axis=1).mean()
    assert step < rand / 4


def test_equal_keys_keep_their_order_and_empty_polygons_come_first():
    sq = dg.rectangle(0, 0, 2, 2)
    polys = [sq, dg.rectangle(100, 100, 102, 102), sq, np.zeros((0, 2), dtype=np.int64), sq]
    assert spatial_order(dg.from_list(polys)).tolist() == [3, 0, 2, 4, 1]
