"""Pins of the oracle's top-k, brute force and recall (Def. 1, Sec. 5.2)."""
import itertools

import numpy as np

from paper_2511_16576_amd import datagen as dg


def test_topk_order_and_ties(orc):
    off = np.array([0, 5, 5, 8], dtype=np.int64)
    ids = np.array([7, 3, 9, 1, 4, 2, 0, 5], dtype=np.int32)
    J = np.array([0.5, 0.9, 0.5, 0.1, 0.9, 0.3, 0.3, 0.7])
    ti, tj = orc.topk(off, ids, J, 3)
    assert ti.tolist() == [[3, 4, 7], [-1, -1, -1], [5, 0, 2]]
    assert tj.tolist() == [[0.9, 0.9, 0.5], [0.0, 0.0, 0.0], [0.7, 0.3, 0.3]]


def test_brute_force_is_exhaustive_ranking(orc):
    w = dg.workload(1, n=25, n_queries=4)
    ids, js = orc.brute_force_topk(w.data, w.queries, 5)
    for q in range(4):
        allj = [orc.jaccard(w.data.poly(p), w.queries.poly(q)) for p in range(25)]
        best = sorted(range(25), key=lambda p: (-allj[p], p))[:5]
        assert ids[q].tolist() == best
        # the jittered source polygon is the nearest neighbour
        assert ids[q, 0] == w.query_source[q]


def test_recall(orc):
    bf_ids = np.array([[1, 2, 3], [4, 5, 6]])
    bf_j = np.array([[0.9, 0.8, 0.7], [0.6, 0.5, 0.4]])
    assert orc.recall_at_k(bf_ids, bf_j, bf_ids, bf_j, 3) == 1.0
    ann = np.array([[1, 9, 3], [-1, -1, -1]])
    annj = np.array([[0.9, 0.2, 0.7], [0, 0, 0]])
    assert abs(orc.recall_at_k(ann, annj, bf_ids, bf_j, 3) - (2 / 3) / 2) < 1e-12
    # a tie with the k-th value counts
    annt = np.array([[1, 2, 8], [4, 5, 6]])
    anntj = np.array([[0.9, 0.8, 0.7], [0.6, 0.5, 0.4]])
    assert orc.recall_at_k(annt, anntj, bf_ids, bf_j, 3) == 1.0


def test_all_pairs_candidates_give_full_recall(orc):
    w = dg.workload(1, n=30, n_queries=3)
    off = np.arange(4, dtype=np.int64) * 30
    ids = np.tile(np.arange(30, dtype=np.int32), 3)
    J = orc.jaccard_candidates(w.data, w.queries, off, ids)
    ti, tj = orc.topk(off, ids, J, 10)
    bi, bj = orc.brute_force_topk(w.data, w.queries, 10)
    assert np.array_equal(ti, bi)
    assert orc.recall_at_k(ti, tj, bi, bj, 10) == 1.0
