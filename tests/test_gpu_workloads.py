"""Parity of the whole search path on seeded subsets of workloads 3 and 5:
signatures and band keys bit-exact, candidate sets equal to the brute-force
definition, exact Jaccard of every candidate pair within 1e-9 relative, and
the top-10.  Workload 3 brings near-duplicate clusters (1-5% jitter: pairs
with many boundary crossings), k = 256 and 32 x 8 bands; workload 5 brings
heavy-tailed vertex counts (up to 8,192) and small polygons in a 2^24 grid
(long first-hit walks), here with k = 64 and cap 2^22 so the oracle stays
within seconds."""
import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu

REL, ABS = 1e-9, 1e-12


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh
    polymh.check_device()
    return polymh


@pytest.mark.parametrize("cfg,n,nq,k,cap,bands,rows", [
    (3, 4000, 40, 256, 1 << 20, 32, 8),
    (5, 4000, 30, 64, 1 << 22, 16, 4),
])
def test_search_path_subset(pm, orc, cfg, n, nq, k, cap, bands, rows):
    import torch
    w = dg.workload(cfg, n=n, n_queries=nq)
    print(f"workload {cfg}: {w.data.n} polygons ({w.data.xy.shape[0]} vertices), {w.queries.n} queries",
          flush=True)
    D, Q = pm.to_device(w.data), pm.to_device(w.queries)
    sd = pm.sign(D, w.box, w.seed, k, cap)
    sq = pm.sign(Q, w.box, w.seed, k, cap)
    osd = orc.sign(w.data, w.box, w.seed, k, cap)
    osq = orc.sign(w.queries, w.box, w.seed, k, cap)
    assert np.array_equal(sd.cpu().numpy().view(np.uint32), osd)
    assert np.array_equal(sq.cpu().numpy().view(np.uint32), osq)
    kd, kq = pm.band(sd, bands, rows, w.seed), pm.band(sq, bands, rows, w.seed)
    okd, okq = orc.band(osd, bands, rows, w.seed), orc.band(osq, bands, rows, w.seed)
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), okd)
    assert np.array_equal(kq.cpu().numpy().view(np.uint64), okq)
    sk, si = pm.index_build(kd)
    off, ids = pm.query(sk, si, D.n, kq)
    ooff, oids = orc.candidates(okd, okq)
    assert np.array_equal(off.cpu().numpy(), ooff)
    assert np.array_equal(ids.cpu().numpy(), oids)
    J, stats = pm.refine_stats(D, Q, off, ids)
    torch.cuda.synchronize()
    got = J.cpu().numpy()
    want = orc.jaccard_candidates(w.data, w.queries, ooff, oids)
    err = np.abs(got - want)
    assert np.all(err <= REL * np.abs(want) + ABS), (err.max(), int(np.argmax(err)))
    print(f"{oids.size} candidate pairs; refinement work counts {stats}")
    ti, tj = pm.topk(off, ids, J, 10)
    wi, wj = orc.topk(ooff, oids, want, 10)
    ti, tj = ti.cpu().numpy(), tj.cpu().numpy()
    assert np.allclose(tj, wj, rtol=REL, atol=ABS)
    for q in range(Q.n):
        for a, b, ja in zip(ti[q], wi[q], wj[q]):
            if a != b:   # only where exact J values tie
                jg = want[ooff[q]:ooff[q + 1]][oids[ooff[q]:ooff[q + 1]] == a]
                assert jg.size == 1 and np.isclose(jg[0], ja, rtol=REL, atol=ABS), (q, a, b)
