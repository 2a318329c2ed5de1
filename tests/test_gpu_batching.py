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
