"""Search-quality measures (Sec. 5.2): recall@k against a brute-force answer."""
from __future__ import annotations

import numpy as np


def recall_at_k(ann_ids, ann_j, bf_ids, bf_j, k: int, tie_eps: float = 1e-12) -> float:
    """Mean over queries of |ANN_k n BF_k| / |BF_k|, where an ANN answer whose
    exact J ties the brute-force k-th value also counts."""
    ann_ids, ann_j = np.asarray(ann_ids), np.asarray(ann_j)
    bf_ids, bf_j = np.asarray(bf_ids), np.asarray(bf_j)
    nq = ann_ids.shape[0]
    if nq == 0:
        return 1.0
    total = 0.0
    for q in range(nq):
        truth = bf_ids[q, :k]
        truth = truth[truth >= 0]
        if truth.size == 0:
            total += 1.0
            continue
        kth = bf_j[q, truth.size - 1]
        a, aj = ann_ids[q, :k], ann_j[q, :k]
        ok = (a >= 0) & (np.isin(a, truth) | (aj >= kth - tie_eps))
        total += min(int(ok.sum()), truth.size) / truth.size
    return total / nq
