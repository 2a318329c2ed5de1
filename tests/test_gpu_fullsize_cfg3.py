"""Workload 3 at full size (1,000,000 polygons, 20% in near-duplicate
clusters, k = 256, cap 2^20, 32 bands x 8 rows, 1,000 queries) through the
whole search path in one pass.  The oracle recomputes, one by one: the
signature rows and band keys of sampled polygons (bit-exact); for sampled
queries, the band keys of every GPU candidate (each must share a key with
the query in the same band) and of a random sample of non-candidates (none
may), the exact J of every candidate (1e-9 relative) and the top-10."""
import time

import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu

REL, ABS = 1e-9, 1e-12
BANDS, ROWS = 32, 8


def test_search_path_workload3_full_size(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh as pm
    pm.check_device()
    t0 = time.time()
    w = dg.workload(3)
    print(f"workload 3: {w.data.n} polygons, {w.data.xy.shape[0]} vertices, {w.queries.n} queries, "
          f"generated in {time.time() - t0:.1f}s", flush=True)
    D, Q = pm.to_device(w.data), pm.to_device(w.queries)
    sig = pm.sign(D, w.box, w.seed, w.k, w.cap)
    qsig = pm.sign(Q, w.box, w.seed, w.k, w.cap)
    keys = pm.band(sig, BANDS, ROWS, w.seed)
    qkeys = pm.band(qsig, BANDS, ROWS, w.seed)
    sk, si = pm.index_build(keys)
    off, ids = pm.query(sk, si, D.n, qkeys)
    J = pm.refine(D, Q, off, ids)
    ti, tj = pm.topk(off, ids, J, 10)
    torch.cuda.synchronize()
    off, ids, J = off.cpu().numpy(), ids.cpu().numpy(), J.cpu().numpy()
    ti, tj = ti.cpu().numpy(), tj.cpu().numpy()
    print(f"{ids.size} candidates", flush=True)
    rng = np.random.default_rng(31)
    # signature rows and band keys of sampled polygons
    rows = np.sort(rng.choice(w.data.n, 64, replace=False))
    osig = orc.sign(w.data.subset(rows), w.box, w.seed, w.k, w.cap)
    assert np.array_equal(sig.cpu().numpy().view(np.uint32)[rows], osig)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64)[rows], orc.band(osig, BANDS, ROWS, w.seed))
    # sampled queries: candidates sound and (on a sample) complete, J and top-10
    for q in rng.choice(w.queries.n, 6, replace=False):
        oq = orc.band(orc.sign(w.queries.subset([q]), w.box, w.seed, w.k, w.cap), BANDS, ROWS, w.seed)[0]
        cand = ids[off[q]:off[q + 1]]
        ck = orc.band(orc.sign(w.data.subset(cand), w.box, w.seed, w.k, w.cap), BANDS, ROWS, w.seed)
        assert (ck == oq[None, :]).any(axis=1).all(), q
        others = np.setdiff1d(rng.choice(w.data.n, 1500, replace=False), cand)
        nk = orc.band(orc.sign(w.data.subset(others), w.box, w.seed, w.k, w.cap), BANDS, ROWS, w.seed)
        assert not (nk == oq[None, :]).any(), q
        want = orc.jaccard_candidates(w.data, w.queries.subset([q]), np.array([0, cand.size]), cand)
        got = J[off[q]:off[q + 1]]
        assert np.all(np.abs(got - want) <= REL * np.abs(want) + ABS), (q, np.abs(got - want).max())
        wi, wj = orc.topk(np.array([0, cand.size]), cand, want, 10)
        assert np.allclose(tj[q], wj[0], rtol=REL, atol=ABS)
        for a, b, ja in zip(ti[q], wi[0], wj[0]):
            if a != b:    # only where exact J values tie
                assert np.isclose(want[cand == a][0], ja, rtol=REL, atol=ABS), (q, a, b)
        print(f"query {q}: {cand.size} candidates checked", flush=True)
