"""The MBR-prefiltered brute force used to measure recall on large sets
(exact J of each query against every polygon whose MBR meets its MBR) gives
the oracle's all-pairs top-k: same ids (J descending, id ascending, J = 0
ranked by id over the whole set), J within the refinement tolerance."""
import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu

REL, ABS = 1e-9, 1e-12


@pytest.mark.parametrize("cfg,n,nq,k", [(5, 3000, 8, 10), (1, 600, 6, 25)])
def test_mbr_brute_force_equals_all_pairs(orc, cfg, n, nq, k):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import metrics
    from paper_2511_16576_amd import polymh as pm
    w = dg.workload(cfg, n=n, n_queries=nq)
    gi, gj = metrics.brute_force_topk_mbr(pm.to_device(w.data), pm.to_device(w.queries), k, chunk=3)
    wi, wj = orc.brute_force_topk(w.data, w.queries, k)
    assert np.allclose(gj, wj, rtol=REL, atol=ABS)
    J = orc.jaccard_all(w.data, w.queries)
    for q in range(nq):
        for a, b, ja in zip(gi[q], wi[q], wj[q]):
            if a != b:   # only where exact J values tie
                assert np.isclose(J[q, a], ja, rtol=REL, atol=ABS), (q, a, b)
