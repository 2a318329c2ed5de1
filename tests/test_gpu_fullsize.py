"""Parity of the whole search step at workload 2's full size (100,000 data
polygons, 10,000 queries, k = 128, 32 bands x 4 rows) in the launch
configuration the benchmark times.  The oracle recomputes, from its own
signatures: band keys of sampled polygons (bit-exact), the candidate sets of
sampled queries by brute-force key comparison against all 100,000 polygons
(bit-exact), exact Jaccard of sampled candidate pairs (1e-9 relative) and the
top-10 of sampled queries (ids exact, J within 1e-9)."""
import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu

REL, ABS = 1e-9, 1e-12
BANDS, ROWS = 32, 4


@pytest.fixture(scope="module")
def run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh as pm
    pm.check_device()
    w = dg.workload(2)
    D, Q = pm.to_device(w.data), pm.to_device(w.queries)
    cfg = pm.default_sign_config()
    sig = pm.sign(D, w.box, w.seed, w.k, w.cap, config=cfg)
    qsig = pm.sign(Q, w.box, w.seed, w.k, w.cap, config=cfg)
    keys = pm.band(sig, BANDS, ROWS, w.seed)
    qkeys = pm.band(qsig, BANDS, ROWS, w.seed)
    sk, si = pm.index_build(keys)
    off, ids = pm.query(sk, si, D.n, qkeys)
    J = pm.refine(D, Q, off, ids)
    ti, tj = pm.topk(off, ids, J, 10)
    torch.cuda.synchronize()
    print(f"workload 2: {ids.numel()} candidates for {Q.n} queries", flush=True)
    return dict(w=w, keys=keys.cpu().numpy().view(np.uint64), qkeys=qkeys.cpu().numpy().view(np.uint64),
                off=off.cpu().numpy(), ids=ids.cpu().numpy(), J=J.cpu().numpy(),
                ti=ti.cpu().numpy(), tj=tj.cpu().numpy())


@pytest.fixture(scope="module")
def oracle_keys(run, orc):
    w = run["w"]
    sd = orc.sign(w.data, w.box, w.seed, w.k, w.cap)
    return orc.band(sd, BANDS, ROWS, w.seed)


def _sample_queries(run, n=24):
    rng = np.random.default_rng(5)
    return np.sort(rng.choice(run["w"].queries.n, n, replace=False))


def test_band_keys_full_size(run, oracle_keys):
    rng = np.random.default_rng(3)
    s = rng.choice(run["w"].data.n, 2000, replace=False)
    assert np.array_equal(run["keys"][s], oracle_keys[s])


def test_candidates_full_size(run, orc, oracle_keys):
    w = run["w"]
    qs = _sample_queries(run)
    qsig = orc.sign(w.queries.subset(qs), w.box, w.seed, w.k, w.cap)
    qk = orc.band(qsig, BANDS, ROWS, w.seed)
    assert np.array_equal(run["qkeys"][qs], qk)
    ooff, oids = orc.candidates(oracle_keys, qk)
    off, ids = run["off"], run["ids"]
    for i, q in enumerate(qs):
        got = ids[off[q]:off[q + 1]]
        want = oids[ooff[i]:ooff[i + 1]]
        assert np.array_equal(got, want), (q, got.size, want.size)


def test_refine_full_size_sampled(run, orc):
    w = run["w"]
    off, ids, J = run["off"], run["ids"], run["J"]
    rng = np.random.default_rng(7)
    c = np.sort(rng.choice(ids.size, 3000, replace=False))
    q_of = np.searchsorted(off, c, side="right") - 1
    for q in np.unique(q_of):
        sel = c[q_of == q]
        Qp = w.queries.poly(q)
        for cc in sel:
            want = orc.jaccard(w.data.poly(ids[cc]), Qp)
            assert abs(J[cc] - want) <= REL * abs(want) + ABS, (q, ids[cc], J[cc], want)


def test_topk_full_size_sampled(run, orc):
    w = run["w"]
    off, ids = run["off"], run["ids"]
    for q in _sample_queries(run, 12):
        cand = ids[off[q]:off[q + 1]]
        Js = np.array([orc.jaccard(w.data.poly(p), w.queries.poly(q)) for p in cand])
        wi, wj = orc.topk(np.array([0, cand.size], dtype=np.int64), cand, Js, 10)
        want_ids, want_j = wi[0], wj[0]
        got_i, got_j = run["ti"][q], run["tj"][q]
        kk = min(10, cand.size)
        assert np.allclose(got_j[:kk], want_j[:kk], rtol=REL, atol=ABS), q
        # ids must agree except where exact J ties make several orders valid
        for a, b, ja in zip(got_i[:kk], want_ids[:kk], want_j[:kk]):
            if a != b:
                assert np.isclose(Js[np.where(cand == a)[0][0]], ja, rtol=REL, atol=ABS), q
        assert (got_i[kk:] == -1).all()


def test_scorer_inference_full_size_sampled(run, orc):
    """The learned scorer's inference path at full size: workload 2 signed at
    k = 256, pair rows of sampled (query, data) pairs and the network output
    against the FP64 oracle on the same BF16-rounded weights."""
    import torch
    from oracle import mlp as om
    from paper_2511_16576_amd import polymh as pm
    from paper_2511_16576_amd import scorer as sc
    w = run["w"]
    D, Q = pm.to_device(w.data), pm.to_device(w.queries)
    dsig = pm.sign(D, w.box, w.seed, 256, w.cap)
    qsig = pm.sign(Q, w.box, w.seed, 256, w.cap)
    dfe, qfe = pm.poly_features(D, w.box), pm.poly_features(Q, w.box)
    rng = np.random.default_rng(11)
    li = rng.integers(0, Q.n, 4096).astype(np.int32)
    ri = rng.integers(0, D.n, 4096).astype(np.int32)
    ri[::4] = w.query_source[li[::4]]                      # near-duplicate pairs too
    s = sc.init_scorer(3)
    y = sc.predict_pairs(s, qsig, qfe, dsig, dfe, torch.from_numpy(li).cuda(),
                         torch.from_numpy(ri).cuda()).cpu().numpy()
    p = s.params.cpu().numpy()
    # the products use the BF16 copies of W1 and W2
    p[om.OFF_W1:om.OFF_B1] = om.bf16_round(p[om.OFF_W1:om.OFF_B1])
    p[om.OFF_W2:om.OFF_B2] = om.bf16_round(p[om.OFF_W2:om.OFF_B2])
    p = p.astype(np.float64)
    samp = rng.choice(4096, 256, replace=False)
    osig_q = orc.sign(w.queries.subset(li[samp]), w.box, w.seed, 256, w.cap)
    osig_d = orc.sign(w.data.subset(ri[samp]), w.box, w.seed, 256, w.cap)
    rows = np.stack([
        om.pair_features(osig_q[i], om.poly_features(w.queries.poly(li[j]), w.box),
                         osig_d[i], om.poly_features(w.data.poly(ri[j]), w.box))
        for i, j in enumerate(samp)])
    X = om.bf16_round(rows.astype(np.float32)).astype(np.float64)
    want = om.forward(X, p)["y"]
    # inputs agree up to the BF16 rounding of the shape features; hidden
    # activations are rounded to BF16 between layers on the GPU
    assert np.abs(y[samp] - want).max() < 2 ** -6
