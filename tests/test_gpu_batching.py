"""Batching form: graph-captured query batches equal eager runs and the
unfused calls; the autotuner's chosen shape gives the same bits."""
import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh
    polymh.check_device()
    return polymh


def test_graph_replays_match_eager_and_plain_calls(pm, orc):
    import torch
    from paper_2511_16576_amd.pipeline import QueryBatch
    w = dg.workload(1, n=600, n_queries=60)
    D = pm.to_device(w.data)
    sig = pm.sign(D, w.box, w.seed, w.k, w.cap)
    keys = pm.band(sig, w.bands, w.rows, w.seed)
    sk, se = pm.index_build(keys)
    nb = 20
    batches = [w.queries.subset(np.arange(i, i + nb)) for i in range(0, 60, nb)]
    maxv = max(b.xy.shape[0] for b in batches)
    qb = QueryBatch(D, sk, se, w.box, w.seed, w.k, w.cap, w.bands, w.rows, nb, maxv, cand_cap=nb * 600)
    qb.load(batches[0])
    qb.capture()
    for rep in range(2):
        for b in batches:
            # eager reference through the plain calls
            Q = pm.to_device(b)
            qs = pm.sign(Q, w.box, w.seed, w.k, w.cap)
            qk = pm.band(qs, w.bands, w.rows, w.seed)
            off, ids = pm.query(sk, se, D.n, qk)
            J = pm.refine(D, Q, off, ids)
            ti, tj = pm.topk(off, ids, J, 10)
            # graph replay on the loaded batch
            qb.load(b)
            torch.cuda.synchronize()
            qb.run_graph()
            gi, gj = qb.result()
            assert torch.equal(gi, ti) and torch.equal(gj, tj)
            # eager run of the same batch object
            qb.run_eager()
            ei, ej = qb.result()
            assert torch.equal(ei, ti) and torch.equal(ej, tj)


def test_capacity_overflow_flag(pm):
    import torch
    from paper_2511_16576_amd.pipeline import QueryBatch
    w = dg.workload(1, n=300, n_queries=10)
    D = pm.to_device(w.data)
    sig = pm.sign(D, w.box, w.seed, w.k, w.cap)
    sk, se = pm.index_build(pm.band(sig, w.bands, w.rows, w.seed))
    qb = QueryBatch(D, sk, se, w.box, w.seed, w.k, w.cap, w.bands, w.rows, 10,
                    w.queries.xy.shape[0], cand_cap=1)
    qb.load(w.queries)
    qb.run_eager()
    with pytest.raises(RuntimeError):
        qb.result()
    assert int(qb.cand_off.abs().sum().item()) == 0


def test_autotuner_choice_is_bit_identical(pm, tmp_path, monkeypatch):
    import torch
    from paper_2511_16576_amd import autotune
    monkeypatch.setenv("POLYMH_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = dg.workload(2, n=3000, n_queries=0)
    space = {"persistent": [1, 0], "block_threads": [64, 256], "hash_block": [0, 16],
             "lds_edges": [256], "samples_per_lane": [1, 2], "blocks_per_cu": [8]}
    cfg, rep = autotune.tune_sign(w.data, w.box, w.seed, 64, w.cap, sample=3000, reps=1, space=space)
    assert rep["tried"] == 16
    D = pm.to_device(w.data)
    a = pm.sign(D, w.box, w.seed, 64, w.cap)
    b = pm.sign(D, w.box, w.seed, 64, w.cap, config=cfg)
    assert torch.equal(a, b)
    cfg2, rep2 = autotune.tune_sign(w.data, w.box, w.seed, 64, w.cap, sample=3000, reps=1, space=space)
    assert rep2 == rep and cfg2.as_dict() == cfg.as_dict()   # served from the cache


def test_graph_replays_binned_signing_and_split_pairs(pm, orc):
    # the batch pipeline with binned query signing, over polygons large
    # enough that refinement defers pairs to its windowed launches (a pair
    # of two 1,510-vertex polygons split over two windows): graph replays
    # and eager runs equal the plain calls (walked signatures, refinement),
    # and the batch's top-10 equals the oracle's for one batch
    import torch
    from paper_2511_16576_amd.pipeline import QueryBatch
    rng = np.random.default_rng(17)
    w = dg.workload(5, n=2500, n_queries=0)
    big = np.argsort(-w.data.counts())[:20]
    src = np.concatenate([big, rng.choice(w.data.n, 20, replace=False)])
    queries = dg.jittered(rng, w.data, src, 0.02, w.grid_bits)
    k, cap, bands, rows = 32, 1 << 22, 8, 4
    D = pm.to_device(w.data)
    sig = pm.sign(D, w.box, w.seed, k, cap)
    sk, se = pm.index_build(pm.band(sig, bands, rows, w.seed))
    h, b = pm.binned_params(D, w.box, k, cap)
    nb = 20
    batches = [queries.subset(np.arange(i, i + nb)) for i in range(0, 40, nb)]
    maxv = max(x.xy.shape[0] for x in batches)
    qb = QueryBatch(D, sk, se, w.box, w.seed, k, cap, bands, rows, nb, maxv, cand_cap=nb * 2500,
                    binned={"horizon": h, "bin_bits": b, "walk_ratio": 300.0})
    qb.load(batches[0])
    qb.capture()
    deferred_seen = split_seen = 0
    dcount = w.data.counts()
    for rep in range(2):
        for x in batches:
            Q = pm.to_device(x)
            qk = pm.band(pm.sign(Q, w.box, w.seed, k, cap), bands, rows, w.seed)
            off, ids = pm.query(sk, se, D.n, qk)
            J, st = pm.refine_stats(D, Q, off, ids)
            n = dcount[ids.cpu().numpy()]
            m = np.repeat(x.counts(), np.diff(off.cpu().numpy()))
            deferred_seen += int((np.maximum(n, m) > 512).sum())
            split_seen += int(((n > 1024) & (m > 1024)).sum())
            assert st[0] == ids.numel() and st[2] == 0     # all on the tiled forms
            ti, tj = pm.topk(off, ids, J, 10)
            qb.load(x)
            torch.cuda.synchronize()
            qb.run_graph()
            gi, gj = qb.result()
            assert torch.equal(gi, ti) and torch.equal(gj, tj)
            qb.run_eager()
            ei, ej = qb.result()
            assert torch.equal(ei, ti) and torch.equal(ej, tj)
    assert deferred_seen > 0 and split_seen > 0
    # the oracle's top-10 of the first batch over the same candidates
    x = batches[0]
    oq = orc.band(orc.sign(x, w.box, w.seed, k, cap), bands, rows, w.seed)
    od = orc.band(orc.sign(w.data, w.box, w.seed, k, cap), bands, rows, w.seed)
    ooff, oids = orc.candidates(od, oq)
    wj = orc.jaccard_candidates(w.data, x, ooff, oids)
    wi, wjt = orc.topk(ooff, oids, wj, 10)
    qb.load(x)
    torch.cuda.synchronize()
    qb.run_graph()
    gi, gj = (t.cpu().numpy() for t in qb.result())
    assert np.allclose(gj, wjt, rtol=1e-9, atol=1e-12)
