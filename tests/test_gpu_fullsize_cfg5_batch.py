"""Workload 5's query batch at full size, in the launch configuration the
benchmark times: 4,000,000 polygons signed from binned samples, 64 x 4
bands, 10,000 queries in the Morton order of their MBR centres signed from
binned samples, looked up and refined as four sub-batches (stretches of the
curve) on streams forked inside one captured graph, ordered by
the collision fraction (read from the saturated signature table) with early
stop (first rounds of 16, 4 rounds, margin 0.01), and beside it the plain
batch (every candidate refined, one graph, the same order).  For five
sampled queries of every sub-batch (its first and last among them, and one
of 257 to 2,048 vertices) the oracle recomputes, one by one: the query's signature and
band keys; the signatures of all its candidates (bit-exact against the
indexed rows and their rows of the saturated table; each shares a band key
with the query, the list is ascending and free of repeats, and none of
2,000 random other polygons shares a key); every candidate's collision
fraction and the best-first order; the early stop's top-10 from its own
exact J of the candidates it refines; and the plain batch's top-10 from the
exact J of the whole list."""
import time

import numpy as np
import pytest

import oracle
from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu

BANDS, ROWS, PARTS = 64, 4, 4
F, ROUNDS, MARGIN = 16, 4, 0.01
REL, ABS = 1e-9, 1e-12


def _assert_top_equal(got_ids, got_j, want_ids, want_j, ctx):
    """One top-k row: J within the refinement tolerance, ids exactly except
    where exact J values tie within it (either order is correct then)."""
    assert np.allclose(got_j, want_j, rtol=REL, atol=ABS), ctx
    live = got_ids[got_ids >= 0]
    assert np.unique(live).size == live.size, ctx
    for t in np.flatnonzero(got_ids != want_ids):
        tied = np.isclose(want_j, want_j[t], rtol=REL, atol=ABS).sum()
        assert want_ids[t] >= 0 and (tied >= 2 or t == want_ids.size - 1), (ctx, t)


@pytest.fixture(scope="module")
def state(orc):
    """Workload 5 in full: the indexed data set and the batch's setup."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh as pm
    pm.check_device()
    t0 = time.time()
    w = dg.workload(5, n_queries=10000)
    nq, k, cap = w.queries.n, w.k, w.cap
    print(f"workload 5: {w.data.n} polygons, {nq} queries, generated in {time.time() - t0:.1f}s", flush=True)
    D = pm.to_device(w.data)
    h, bb = pm.binned_params(D, w.box, k, cap)
    sig = pm.sign_binned(D, w.box, w.seed, k, cap, horizon=h, bin_bits=bb, config=pm.binned_config(D))
    sk, se = pm.index_build(pm.band(sig, BANDS, ROWS, w.seed))
    Qd = pm.to_device(w.queries)
    binned = {"horizon": h, "bin_bits": bb, "walk_ratio": 300.0}
    qs = pm.sign_binned(Qd, w.box, w.seed, k, cap, horizon=h, bin_bits=bb)
    off, _ = pm.query(sk, se, D.n, pm.band(qs, BANDS, ROWS, w.seed))
    cand_cap = int(1.25 * int(off[-1].item())) + 65536
    del qs, off
    common = dict(sign_config=pm.binned_config(Qd), binned=binned, dsig=sig)
    args = (D, sk, se, w.box, w.seed, k, cap, BANDS, ROWS, nq, w.queries.xy.shape[0], cand_cap)
    packed = pm.sig_pack(sig)
    yield dict(w=w, D=D, sig=sig, packed=packed, common=common, args=args, cand_cap=cand_cap)
    torch.cuda.empty_cache()


def test_query_batch_workload5_full_size(orc, state):
    from paper_2511_16576_amd.pipeline import SplitBatch
    w, sig, packed, common, args = state["w"], state["sig"], state["packed"], state["common"], state["args"]
    nq, k, cap = w.queries.n, w.k, w.cap
    cand_cap = state["cand_cap"]
    jb = SplitBatch(*args, parts=PARTS, method="jhat", F=F, rounds=ROUNDS, margin=MARGIN, dpacked=packed,
                    query_order="morton", **common)
    jb.load(w.queries)
    jb.capture()
    pb = SplitBatch(*args, parts=1, method="plain", query_order="morton", **common)
    pb.load(w.queries)
    pb.capture()
    # both batches hold query perm[r] in row r; results come back in the given order
    perm = jb.perm
    assert np.array_equal(pb.perm, perm) and np.array_equal(np.sort(perm), np.arange(nq))
    for _ in range(2):
        jb.run_graph()
        pb.run_graph()
    j_ids, j_j = (x.cpu().numpy() for x in jb.result())
    p_ids, p_j = (x.cpu().numpy() for x in pb.result())
    print(f"batches replayed: {cand_cap} candidate slots a part", flush=True)

    rng = np.random.default_rng(51)
    nv = np.diff(w.queries.offsets)
    # rows of each sub-batch: its first and last, two at random and one at
    # random among queries of 257 to 2,048 vertices (the longest rings are
    # left out so the oracle's fan clipping of whole lists stays short; they
    # have refinement tests of their own)
    sample = []
    for a, b in jb.bounds:
        pool = np.arange(a + 1, b - 1)
        sample += [a, b - 1] + rng.choice(pool, 2, replace=False).tolist()
        long_ = pool[(nv[perm[pool]] > 256) & (nv[perm[pool]] <= 2048)]
        if long_.size:
            sample.append(int(rng.choice(long_)))
    others = np.sort(rng.choice(w.data.n, 2000, replace=False))
    okeys = orc.band(orc.sign(w.data.subset(others), w.box, w.seed, k, cap), BANDS, ROWS, w.seed)
    gsig = sig.cpu().numpy().view(np.uint32)
    gpk = packed.cpu().numpy().view(np.uint16)
    assert (gsig >= 65535).any(), "values of 65535 and more: the comparison reads full values"
    for row in sample:
        t1 = time.time()
        q = int(perm[row])
        p = int(np.searchsorted([b for _, b in jb.bounds], row, side="right"))
        part, lq = jb.parts[p], row - jb.bounds[p][0]
        o = part.cand_off.cpu().numpy()
        a, b = int(o[lq]), int(o[lq + 1])
        cand = part.cand_ids[a:b].cpu().numpy()
        oq = orc.sign(w.queries.subset([q]), w.box, w.seed, k, cap)
        assert np.array_equal(part.sig[lq].cpu().numpy().view(np.uint32), oq[0]), q
        oqk = orc.band(oq, BANDS, ROWS, w.seed)[0]
        assert np.array_equal(part.keys[lq].cpu().numpy().view(np.uint64), oqk), q
        # the candidate list: sound, ascending without repeats, sampled complete
        assert cand.size > 0 and np.all(np.diff(cand) > 0), q
        osig = orc.sign(w.data.subset(cand), w.box, w.seed, k, cap)
        assert np.array_equal(gsig[cand], osig), q
        # their rows of the saturated table
        assert np.array_equal(gpk[cand], np.minimum(osig, 65535).astype(np.uint16)), q
        assert (orc.band(osig, BANDS, ROWS, w.seed) == oqk[None, :]).any(axis=1).all(), q
        outside = ~np.isin(others, cand)
        assert not (okeys[outside] == oqk[None, :]).any(), q
        pl = pb.parts[0]
        po = pl.cand_off.cpu().numpy()
        assert np.array_equal(pl.cand_ids[int(po[row]):int(po[row + 1])].cpu().numpy(), cand), q
        # collision fractions and the best-first order
        pred = oracle.collision_fraction(oq[0], osig).astype(np.float32)
        assert np.array_equal(part.score[a:b].cpu().numpy(), pred), q
        order, is_sorted = oracle.best_first(pred)
        assert bool(part.sorted_ok[lq].item()) == is_sorted, q
        assert np.array_equal(part.order[a:b].cpu().numpy(), order), q
        # the early stop from the oracle's exact J of the candidates it refines
        one = w.queries.subset([q])
        jf = lambda pos: orc.jaccard_candidates(w.data, one, np.array([0, pos.size]), cand[pos])
        r = oracle.early_stop_query(cand, pred, jf, 10, F, ROUNDS, MARGIN)
        assert min(r["gaps"], default=1.0) > 1e-6, q
        _assert_top_equal(j_ids[q], j_j[q], r["top_ids"], r["top_j"], ("early stop", q))
        # the plain batch: the top-10 of the whole list
        Jall = orc.jaccard_candidates(w.data, one, np.array([0, cand.size]), cand)
        ti, tj = oracle.topk(np.array([0, cand.size]), cand, Jall, 10)
        _assert_top_equal(p_ids[q], p_j[q], ti[0], tj[0], ("plain", q))
        print(f"query {q} (row {row}, sub-batch {p}, {nv[q]} vertices): {cand.size} candidates, {r['refined']} refined by "
              f"the early stop; checked in {time.time() - t1:.1f}s", flush=True)
    del jb, pb


# the learned batch as the benchmark runs it: the network re-scores each
# query's first 8 candidates by collision fraction, the order is rebuilt,
# then one round of 22 (margin -0.3) and the finishing pass
HEAD, F_L, ROUNDS_L, MARGIN_L = 8, 22, 1, -0.3


def test_learned_batch_workload5_full_size(orc, state):
    """The learned batch in the benchmark's launch configuration (queries in
    Morton order; a seeded network: its arithmetic, not its training, is
    under test).  For sampled queries: the head slots are the
    collision-fraction order's first 8; their
    new scores are the oracle's FP64 network on the oracle's feature rows
    (within the BF16 rounding between the layers), the other scores the
    oracle's collision fractions exactly; the rebuilt order sorts the final
    scores (desc, position asc); and the top-10 is the exact top-10 (the
    oracle's J) of the first 22 candidates of that order (every query that
    stops after its round), or of the whole list (the finishing pass)."""
    import torch
    from oracle import mlp as om
    from paper_2511_16576_amd import polymh as pm
    from paper_2511_16576_amd import scorer as sc
    from paper_2511_16576_amd.pipeline import SplitBatch
    w, D, sig, packed = state["w"], state["D"], state["sig"], state["packed"]
    k, cap = w.k, w.cap
    net = sc.init_scorer(5)
    dfeat = pm.poly_features(D, w.box)
    lb = SplitBatch(*state["args"], parts=PARTS, method="scorer", scorer=net, dfeat=dfeat, head=HEAD, F=F_L,
                    rounds=ROUNDS_L, margin=MARGIN_L, dpacked=packed, query_order="morton", **state["common"])
    lb.load(w.queries)
    perm = lb.perm
    lb.capture()
    for _ in range(2):
        lb.run_graph()
    l_ids, l_j = (x.cpu().numpy() for x in lb.result())
    p = net.params.cpu().numpy()
    p[om.OFF_W1:om.OFF_B1] = om.bf16_round(p[om.OFF_W1:om.OFF_B1])
    p[om.OFF_W2:om.OFF_B2] = om.bf16_round(p[om.OFF_W2:om.OFF_B2])
    p = p.astype(np.float64)
    rng = np.random.default_rng(61)
    sample = []
    for a, b in lb.bounds:
        sample += [a, b - 1] + rng.choice(np.arange(a + 1, b - 1), 2, replace=False).tolist()
    for row in sample:
        t1 = time.time()
        q = int(perm[row])
        pi = int(np.searchsorted([b for _, b in lb.bounds], row, side="right"))
        part, lq = lb.parts[pi], row - lb.bounds[pi][0]
        o = part.cand_off.cpu().numpy()
        a, b = int(o[lq]), int(o[lq + 1])
        cand = part.cand_ids[a:b].cpu().numpy()
        oq = orc.sign(w.queries.subset([q]), w.box, w.seed, k, cap)
        osig = orc.sign(w.data.subset(cand), w.box, w.seed, k, cap)
        pred = oracle.collision_fraction(oq[0], osig).astype(np.float32)
        jorder, _ = oracle.best_first(pred)
        assert np.array_equal(part.order[a:b].cpu().numpy(), jorder), q
        # the head slots: the first 8 of the collision-fraction order
        nh = min(HEAD, cand.size)
        hc = part.hc[lq * HEAD:(lq + 1) * HEAD].cpu().numpy()
        hid = part.hid[lq * HEAD:(lq + 1) * HEAD].cpu().numpy()
        assert np.array_equal(hc[:nh], a + jorder[:nh]) and (hc[nh:] == -1).all(), q
        assert np.array_equal(hid[:nh], cand[jorder[:nh]]), q
        # final scores: the network on the head, the collision fraction elsewhere
        score = part.score[a:b].cpu().numpy()
        rest = np.setdiff1d(np.arange(cand.size), jorder[:nh])
        assert np.array_equal(score[rest], pred[rest]), q
        qf = om.poly_features(w.queries.poly(q), w.box)
        rows = np.stack([om.pair_features(oq[0], qf, osig[j], om.poly_features(w.data.poly(cand[j]), w.box))
                         for j in jorder[:nh]])
        want = om.forward(om.bf16_round(rows.astype(np.float32)).astype(np.float64), p)["y"]
        assert np.abs(score[jorder[:nh]] - want).max() < 2 ** -6, q
        # the rebuilt order sorts the final scores
        forder, srt = oracle.best_first(score)
        assert srt and np.array_equal(part.order2[a:b].cpu().numpy(), forder), q
        # the top-10: the exact top-10 of the candidates a round reached
        one = w.queries.subset([q])
        Jall = orc.jaccard_candidates(w.data, one, np.array([0, cand.size]), cand)
        fits = []
        # candidates refined after each round (F, then F 2^(r-1)), or all
        reach = np.cumsum([F_L if r < 2 else F_L << (r - 1) for r in range(ROUNDS_L)]).tolist()
        for r in reach + [cand.size]:
            sel = forder[:r]
            ti, tj = oracle.topk(np.array([0, sel.size]), cand[sel], Jall[sel], 10)
            if np.allclose(l_j[q], tj[0], rtol=REL, atol=ABS):
                fits.append(r)
                _assert_top_equal(l_ids[q], l_j[q], ti[0], tj[0], ("learned", q, r))
        assert fits, q
        print(f"query {q} (row {row}, sub-batch {pi}): {cand.size} candidates, top-10 of the first {fits[0]} refined; "
              f"checked in {time.time() - t1:.1f}s", flush=True)
    del lb
