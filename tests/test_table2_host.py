"""Host pieces of Table 2's experiment: the stand-ins of Table 1's datasets
(sizes and mean vertex counts) and recall@k for k = 10, 50, 100 (the
package's metric against the oracle's independent one, plus fixed cases)."""
import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg
from paper_2511_16576_amd import metrics


@pytest.mark.parametrize("name", list(dg.TABLE1))
def test_standin_shape(name):
    N, Q, mean = dg.TABLE1[name]
    n = 3000 if name != "parks" else 600
    w = dg.table1_standin(name, n=n, n_queries=40)
    c = w.data.counts()
    assert w.data.n == n and w.queries.n == 40
    assert c.min() >= 4
    assert abs(c.mean() - mean) < 0.05 * mean, (c.mean(), mean)
    # queries are jittered copies: same vertex counts as their sources
    assert np.array_equal(w.queries.counts(), c[w.query_source])


def test_recall_fixed_cases():
    bf_i = np.array([[3, 1, 2, 0]], dtype=np.int32)
    bf_j = np.array([[0.9, 0.8, 0.7, 0.7]])
    assert metrics.recall_at_k(bf_i, bf_j, bf_i, bf_j, 3) == 1.0
    assert metrics.recall_at_k(np.array([[5, 6, 7, -1]]), np.array([[0.1, 0.1, 0.1, 0.0]]), bf_i, bf_j, 3) == 0.0
    # id 0 ties the third value (0.7): counts as a hit
    assert metrics.recall_at_k(np.array([[3, 1, 0, 2]]), np.array([[0.9, 0.8, 0.7, 0.7]]), bf_i, bf_j, 3) == 1.0
    assert metrics.recall_at_k(np.array([[3, 9, 8, 2]]), np.array([[0.9, 0.5, 0.4, 0.7]]), bf_i, bf_j, 3) == 1 / 3


@pytest.mark.parametrize("k", [10, 50, 100])
def test_recall_matches_oracle(orc, k):
    rng = np.random.default_rng(k)
    nq, width = 30, 120
    bf_j = -np.sort(-np.round(rng.random((nq, width)), 1), axis=1)      # many ties
    bf_i = np.stack([rng.permutation(400)[:width] for _ in range(nq)]).astype(np.int32)
    ann_i = bf_i.copy()
    ann_j = bf_j.copy()
    # replace a random share of the answers by other ids with random values
    swap = rng.random((nq, width)) < 0.4
    ann_i[swap] = rng.integers(400, 800, swap.sum())
    ann_j[swap] = np.round(rng.random(swap.sum()), 1)
    o = np.argsort(-ann_j, axis=1, kind="stable")
    ann_i, ann_j = np.take_along_axis(ann_i, o, 1), np.take_along_axis(ann_j, o, 1)
    got = metrics.recall_at_k(ann_i, ann_j, bf_i, bf_j, k)
    want = orc.recall_at_k(ann_i, ann_j, bf_i, bf_j, k)
    assert got == pytest.approx(want, abs=1e-12)
