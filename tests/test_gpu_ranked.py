"""Ranked refinement without host reads (the form a captured query batch
uses): collision-fraction scores and orders, fixed head slots, the ordered
early-stop refinement with its finishing pass, and whole query batches of
each method replayed as graphs against their eager runs."""
import numpy as np
import pytest

import oracle
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


@pytest.fixture(scope="module")
def setup(pm):
    """A 3,000-polygon workload-2 subset signed at k = 256 (bit-exact with the
    oracle, checked here), 64 x 4 bands, 48 queries and their candidates."""
    import torch
    w = dg.workload(2, n=3000, n_queries=48)
    D, Q = pm.to_device(w.data), pm.to_device(w.queries)
    k = 256
    sig = pm.sign(D, w.box, 0, k, w.cap)
    qsig = pm.sign(Q, w.box, 0, k, w.cap)
    osig = oracle.sign(w.data, w.box, 0, k, w.cap)
    oqsig = oracle.sign(w.queries, w.box, 0, k, w.cap)
    assert np.array_equal(sig.cpu().numpy().view(np.uint32), osig)
    assert np.array_equal(qsig.cpu().numpy().view(np.uint32), oqsig)
    sk, se = pm.index_build(pm.band(sig, 64, 4, 0))
    off, ids = pm.query(sk, se, D.n, pm.band(qsig, 64, 4, 0))
    torch.cuda.synchronize()
    return dict(w=w, D=D, Q=Q, sig=sig, qsig=qsig, osig=osig, oqsig=oqsig, sk=sk, se=se, off=off, ids=ids)


def _check_order(score, off, order):
    """Within each query, positions sorted by (score desc, position asc)."""
    for q in range(off.size - 1):
        a, b = off[q], off[q + 1]
        pos = order[a:b]
        assert np.array_equal(np.sort(pos), np.arange(b - a)), q
        s = score[a + pos]
        key = np.lexsort((pos, -s))
        assert np.array_equal(key, np.arange(b - a)), q


def test_jhat_order_matches_definition(pm, setup):
    off, ids = setup["off"], setup["ids"]
    score, order, ok = pm.rank_jhat_order(setup["qsig"], setup["sig"], off, ids)
    o, i = off.cpu().numpy(), ids.cpu().numpy()
    sc, od = score.cpu().numpy()[:i.size], order.cpu().numpy()[:i.size]
    # the share of the 256 oracle hashes on which query and candidate agree
    rows = np.repeat(np.arange(o.size - 1), np.diff(o))
    want = (setup["oqsig"][rows] == setup["osig"][i]).mean(axis=1).astype(np.float32)
    assert np.array_equal(sc, want)
    assert (ok.cpu().numpy() == 1).all()
    _check_order(sc, o, od)
    # rank_order on the same scores gives the same order
    order2 = order.clone()
    pm.rank_order(off, score, order2, ok)
    assert np.array_equal(order2.cpu().numpy()[:i.size], od)


@pytest.mark.parametrize("k", [1, 37, 64, 100, 300])
def test_jhat_order_other_k(pm, k):
    """Signature lengths off the vector path (not a multiple of 4, or beyond
    256) and tiny ones."""
    import torch
    rng = np.random.default_rng(k)
    qs = rng.integers(1, 4, (5, k)).astype(np.uint32)
    ds = rng.integers(1, 4, (40, k)).astype(np.uint32)
    counts = np.array([0, 7, 40, 1, 13])
    off = np.zeros(6, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    ids = np.concatenate([rng.choice(40, c, replace=False) for c in counts]).astype(np.int32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    score, order, ok = pm.rank_jhat_order(t(qs.view(np.int32)), t(ds.view(np.int32)), t(off), t(ids))
    rows = np.repeat(np.arange(5), counts)
    want = (qs[rows] == ds[ids]).sum(axis=1).astype(np.float32) * np.float32(1.0 / k)
    assert np.array_equal(score.cpu().numpy()[:ids.size], want)
    _check_order(want, off, order.cpu().numpy()[:ids.size])


def test_sig_pack_layout(pm, setup):
    """The saturated table: every value as min(value, 65535) in 16 bits."""
    osig = setup["osig"]
    got = pm.sig_pack(setup["sig"]).cpu().numpy().view(np.uint16)
    assert got.shape == osig.shape
    assert np.array_equal(got, np.minimum(osig, 65535).astype(np.uint16))


def test_jhat_order_packed_equals_unpacked(pm, setup):
    off, ids = setup["off"], setup["ids"]
    packed = pm.sig_pack(setup["sig"])
    a = pm.rank_jhat_order(setup["qsig"], setup["sig"], off, ids)
    b = pm.rank_jhat_order(setup["qsig"], setup["sig"], off, ids, packed=packed)
    C = int(off[-1].item())
    assert np.array_equal(a[0].cpu().numpy()[:C], b[0].cpu().numpy()[:C])
    assert np.array_equal(a[1].cpu().numpy()[:C], b[1].cpu().numpy()[:C])
    assert np.array_equal(a[2].cpu().numpy(), b[2].cpu().numpy())


@pytest.mark.parametrize("k", [4, 64, 100, 192, 256])
def test_jhat_order_packed_saturated_values(pm, k):
    """Values around the saturation point (equal and different values that
    both saturate, one that saturates against one that does not, equal low
    halves with different high halves), so that every branch of the
    comparison is taken: scores equal the oracle's share of equal values,
    the order is the oracle's."""
    import torch
    rng = np.random.default_rng(k)
    vals = np.array([7, 7 + (1 << 16), 65534, 65535, 65536, 65537, 1 << 20, (1 << 20) + 7, 70000, 3, 65535 + 7,
                     1 << 26], dtype=np.uint32)
    qs = vals[rng.integers(0, vals.size, (6, k))]
    ds = vals[rng.integers(0, vals.size, (120, k))]
    ds[:6] = qs                                  # candidates equal to their query
    counts = np.array([0, 3, 120, 1, 40, 77])
    off = np.zeros(7, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    ids = np.concatenate([rng.choice(120, c, replace=False) for c in counts]).astype(np.int32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    dsig = t(ds.view(np.int32))
    packed = pm.sig_pack(dsig)
    assert np.array_equal(packed.cpu().numpy().view(np.uint16), np.minimum(ds, 65535).astype(np.uint16))
    score, order, ok = pm.rank_jhat_order(t(qs.view(np.int32)), dsig, t(off), t(ids), packed=packed)
    cnt = np.concatenate([oracle.collision_counts(qs[q], ds[ids[off[q]:off[q + 1]]]) for q in range(6)])
    assert np.array_equal(score.cpu().numpy()[:ids.size], cnt.astype(np.float32) * np.float32(1.0 / k))
    for q in range(6):
        a, b = off[q], off[q + 1]
        od, srt = oracle.best_first(score.cpu().numpy()[a:b])
        assert srt and np.array_equal(order.cpu().numpy()[a:b], od), q
    assert (ok.cpu().numpy() == 1).all()


def test_head_fixed(pm, setup):
    off, ids = setup["off"], setup["ids"]
    score, order, ok = pm.rank_jhat_order(setup["qsig"], setup["sig"], off, ids)
    M = 20
    hq, hc, hid = (x.cpu().numpy() for x in pm.rank_head_fixed(off, ids, order, M))
    o, i, od = off.cpu().numpy(), ids.cpu().numpy(), order.cpu().numpy()
    for q in range(o.size - 1):
        n = o[q + 1] - o[q]
        for t in range(M):
            s = q * M + t
            assert hq[s] == q
            if t < n:
                c = o[q] + od[o[q] + t]
                assert hc[s] == c and hid[s] == i[c]
            else:
                assert hc[s] == -1 and hid[s] == -1


@pytest.mark.parametrize("M", [1, 7, 32, 64])
def test_reorder_head_equals_full_sort(pm, setup, M):
    """New scores for the first M of each order (a query with fewer
    candidates re-scores all of them; one list left unsorted is copied):
    the merge equals a sort of all candidates by the new scores."""
    import torch
    off, ids = setup["off"], setup["ids"]
    score, order, ok = pm.rank_jhat_order(setup["qsig"], setup["sig"], off, ids)
    hq, hc, hid = pm.rank_head_fixed(off, ids, order, M)
    rng = np.random.default_rng(M)
    new = torch.from_numpy(rng.random(hc.numel()).astype(np.float32)).cuda()
    new[::5] = 0.25                             # ties, broken by position
    pm.scatter_scores(hc, new, score)
    ok[3] = 0                                   # an unsorted list: copied as it is
    out = torch.empty_like(order)
    pm.rank_reorder_head(off, score, order, M, ok, out)
    want = order.clone()
    pm.rank_order(off, score, want, torch.empty_like(ok))
    o = off.cpu().numpy()
    got, exp, src = out.cpu().numpy(), want.cpu().numpy(), order.cpu().numpy()
    for q in range(o.size - 1):
        a, b = o[q], o[q + 1]
        if q == 3:
            assert np.array_equal(got[a:b], src[a:b])
        else:
            assert np.array_equal(got[a:b], exp[a:b]), q


def test_ordered_refine_inf_margin_is_full(pm, setup):
    D, Q, off, ids = setup["D"], setup["Q"], setup["off"], setup["ids"]
    J = pm.refine(D, Q, off, ids)
    ti, tj = pm.topk(off, ids, J, 10)
    score, order, ok = pm.rank_jhat_order(setup["qsig"], setup["sig"], off, ids)
    for rounds in (0, 1, 3):
        a_ids, a_j, cnt = pm.rank_refine_ordered(D, Q, off, ids, score, order, ok, topk=10, F=8, rounds=rounds,
                                                 margin=float("inf"))
        assert bool((a_ids == ti).all()), rounds
        assert bool((a_j == tj).all()), rounds
        c = cnt.cpu().numpy()
        assert c[0] == ids.numel(), rounds
        # rounds of 8, 8, 16, 32, ...: queries with more than 8 2^(rounds - 1)
        # candidates (none visited without a round) are completed by the
        # finishing pass
        seen = 8 * 2 ** (rounds - 1) if rounds else 0
        want_fin = int((np.diff(off.cpu().numpy()) > seen).sum())
        assert c[1] == want_fin, (rounds, c[1], want_fin)


def test_ordered_refine_exact_scores(pm, setup):
    """With the exact J as scores and margin 0 the early stop returns the
    exact top-10 (every candidate it skips has a J at most the 10th best)
    and refines fewer pairs; one round plus the finishing pass equals the
    host-driven rank_refine with one round."""
    D, Q, off, ids = setup["D"], setup["Q"], setup["off"], setup["ids"]
    J = pm.refine(D, Q, off, ids)
    ti, tj = pm.topk(off, ids, J, 10)
    score = J.float()
    order = torch_empty_like_int(ids)
    ok = torch_empty_u8(Q.n)
    pm.rank_order(off, score, order, ok)
    # rounds of 4, 8, ..., 512 candidates: every list ends inside them
    b_ids, b_j, cnt = pm.rank_refine_ordered(D, Q, off, ids, score, order, ok, topk=10, F=4, rounds=8, margin=0.0)
    assert np.allclose(b_j.cpu().numpy(), tj.cpu().numpy(), rtol=0, atol=1e-6)
    c = cnt.cpu().numpy()
    assert c[0] < ids.numel() and c[1] == 0
    # one round of 3 per query, then the finishing pass
    f_ids, f_j, cnt1 = pm.rank_refine_ordered(D, Q, off, ids, score, order, ok, topk=10, F=3, rounds=1,
                                              margin=0.0)
    assert np.allclose(f_j.cpu().numpy(), tj.cpu().numpy(), rtol=0, atol=1e-6)
    assert cnt1.cpu().numpy()[1] > 0
    # the host-driven call with its one round exhausted finishes the same way
    g_ids, g_j, nref1, r1 = pm.rank_refine(D, Q, off, ids, score, topk=10, F=3, margin=0.0, max_rounds=1)
    assert r1 == 1
    assert bool((g_ids == f_ids).all()) and bool((g_j == f_j).all())
    assert nref1 == int(cnt1.cpu().numpy()[0])
    # the schedule F, F, 2F, 4F, ...: three rounds of F = 1 visit 4 candidates
    # of each query before the finishing pass
    h_ids, h_j, cnt2 = pm.rank_refine_ordered(D, Q, off, ids, score, order, ok, topk=10, F=1, rounds=3,
                                              margin=float("inf"))
    nc = np.diff(off.cpu().numpy())
    assert int(cnt2.cpu().numpy()[1]) == int((nc > 4).sum())


def _assert_top_equal(got_ids, got_j, want_ids, want_j, ctx):
    """Top-k rows equal: J within the refinement tolerance, ids exactly
    except where two candidates' exact J tie within it (either order is
    correct then)."""
    assert np.allclose(got_j, want_j, rtol=1e-9, atol=1e-12), ctx
    k = want_ids.shape[1]
    for q in range(want_ids.shape[0]):
        live = got_ids[q][got_ids[q] >= 0]
        assert np.unique(live).size == live.size, (ctx, q)
        for t in np.flatnonzero(got_ids[q] != want_ids[q]):
            tied = np.isclose(want_j[q], want_j[q, t], rtol=1e-9, atol=1e-12).sum()
            assert want_ids[q, t] >= 0 and (tied >= 2 or t == k - 1), (ctx, q, t)


@pytest.fixture(scope="module")
def oracle_j(setup):
    """The oracle's exact J of every candidate, its collision fractions (from
    its own signatures) as FP32 predictions."""
    o, i = setup["off"].cpu().numpy(), setup["ids"].cpu().numpy()
    i = i[:o[-1]]
    w = setup["w"]
    J = oracle.jaccard_candidates(w.data, w.queries, o, i)
    pred = np.concatenate([oracle.collision_fraction(setup["oqsig"][q], setup["osig"][i[o[q]:o[q + 1]]])
                           for q in range(o.size - 1)]).astype(np.float32)
    return o, i, J, pred


@pytest.mark.parametrize("F,rounds,margin", [(4, 3, 0.01), (8, 4, 0.0), (2, 5, -0.02), (16, 2, 0.05),
                                             (3, 1, 0.0), (1, 0, 0.0)])
def test_ordered_refine_equals_oracle_early_stop(pm, setup, oracle_j, F, rounds, margin):
    """The device-driven early stop, ordered by the fused collision fraction,
    against the oracle's best-first refinement with early stop on its own
    collision fractions and exact J: top-10 ids and J, pairs refined and
    queries the finishing pass completed.  Every stop decision of the oracle
    is at least 1e-6 from the other outcome, so the refinement tolerance
    cannot flip one."""
    o, i, J, pred = oracle_j
    off, ids = setup["off"], setup["ids"]
    score, order, ok = pm.rank_jhat_order(setup["qsig"], setup["sig"], off, ids)
    assert np.array_equal(score.cpu().numpy()[:i.size], pred)
    want = oracle.early_stop_topk(o, i, pred, J, 10, F, rounds, margin)
    assert want["min_gap"] > 1e-6
    t_ids, t_j, cnt = pm.rank_refine_ordered(setup["D"], setup["Q"], off, ids, score, order, ok, topk=10, F=F,
                                             rounds=rounds, margin=margin)
    _assert_top_equal(t_ids.cpu().numpy(), t_j.cpu().numpy(), want["top_ids"], want["top_j"], (F, rounds, margin))
    c = cnt.cpu().numpy()
    assert c[0] == want["refined"] and c[1] == want["finished"], (c, want["refined"], want["finished"])


@pytest.mark.parametrize("seed", [0, 1])
def test_ordered_refine_other_predictions_equals_oracle(pm, setup, oracle_j, seed):
    """Predictions that are not collision fractions (as the scorer writes
    them; coarse values, so many ties broken by position): ordered by
    polymh_rank_order, refined with early stop, against the oracle."""
    import torch
    o, i, J, _ = oracle_j
    off, ids = setup["off"], setup["ids"]
    rng = np.random.default_rng(seed)
    pred = (rng.integers(0, 48, i.size) / 64).astype(np.float32)
    score = torch.from_numpy(pred).cuda()
    order = torch_empty_like_int(ids)
    ok = torch_empty_u8(setup["Q"].n)
    pm.rank_order(off, score, order, ok)
    for F, rounds, margin in ((4, 3, 0.05), (6, 4, -0.1)):
        want = oracle.early_stop_topk(o, i, pred, J, 10, F, rounds, margin)
        assert want["min_gap"] > 1e-6
        t_ids, t_j, cnt = pm.rank_refine_ordered(setup["D"], setup["Q"], off, ids, score, order, ok, topk=10, F=F,
                                                 rounds=rounds, margin=margin)
        _assert_top_equal(t_ids.cpu().numpy(), t_j.cpu().numpy(), want["top_ids"], want["top_j"], (seed, F))
        c = cnt.cpu().numpy()
        assert c[0] == want["refined"] and c[1] == want["finished"], (seed, F)


def torch_empty_like_int(t):
    import torch
    return torch.empty(max(t.numel(), 1), dtype=torch.int32, device=t.device)


def torch_empty_u8(n):
    import torch
    return torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("method", ["jhat", "scorer"])
def test_ranked_batch_graph_equals_eager(pm, setup, method):
    """A whole batch (sign, band, capped lookup, ranking, early-stop
    refinement) captured as one graph: every replay equals the eager run,
    with eager work between replays; margin +inf equals the plain batch."""
    import torch
    from paper_2511_16576_amd import scorer as sc
    from paper_2511_16576_amd.pipeline import QueryBatch
    w, D = setup["w"], setup["D"]
    feats = pm.poly_features(D, w.box)
    s = sc.init_scorer(0)
    cap = int(setup["ids"].numel()) * 2 + 1024
    common = dict(box=w.box, seed=0, k=256, cap=w.cap, bands=64, rows=4, n_queries=w.queries.n,
                  max_vertices=w.queries.xy.shape[0], cand_cap=cap)
    plain = QueryBatch(D, setup["sk"], setup["se"], **common)
    plain.load(w.queries)
    plain.run_eager()
    p_ids, p_j = (x.clone() for x in plain.result())
    for margin in (0.02, float("inf")):
        qb = QueryBatch(D, setup["sk"], setup["se"], **common, method=method, dsig=setup["sig"], scorer=s,
                        dfeat=feats, head=16, F=4, rounds=3, margin=margin)
        qb.load(w.queries)
        qb.run_eager()
        e_ids, e_j = (x.clone() for x in qb.result())
        e_cnt = qb.counts.clone()
        qb.capture()
        for rep in range(3):
            qb.top_ids.fill_(-7)
            torch.cuda.synchronize()
            qb.run_graph()
            g_ids, g_j = qb.result()
            assert torch.equal(g_ids, e_ids) and torch.equal(g_j, e_j), (margin, rep)
            assert torch.equal(qb.counts, e_cnt)
            # eager work of the program between replays
            pm.refine(D, plain.Q, plain.cand_off, plain.cand_ids, n_cand=plain.cand_ids.numel())
            torch.cuda.synchronize()
        if margin == float("inf"):
            assert torch.equal(e_ids, p_ids) and torch.equal(e_j, p_j)
        else:
            # every answer is an exact J of its pair, in (J desc, id asc) order
            J = pm.refine(D, qb.Q, qb.cand_off, qb.cand_ids).cpu().numpy()
            o, i = qb.cand_off.cpu().numpy(), qb.cand_ids.cpu().numpy()
            ei, ej = e_ids.cpu().numpy(), e_j.cpu().numpy()
            for q in range(o.size - 1):
                lst = dict(zip(i[o[q]:o[q + 1]].tolist(), J[o[q]:o[q + 1]].tolist()))
                got = [(x, y) for x, y in zip(ei[q], ej[q]) if x >= 0]
                assert all(lst[x] == y for x, y in got), q
                assert got == sorted(got, key=lambda t: (-t[1], t[0])), q
        del qb


@pytest.mark.parametrize("method,parts", [("plain", 1), ("jhat", 4), ("scorer", 2)])
def test_split_batch_morton_order_equals_given(pm, setup, method, parts):
    """The batch run in the Morton order of its queries (the parts hold
    stretches of the curve) returns every query's top-10 in the given order,
    equal to the given-order batch's, eagerly and on graph replays, and the
    early stop's counts are the same."""
    import torch
    from paper_2511_16576_amd import scorer as sc
    from paper_2511_16576_amd.pipeline import SplitBatch, spatial_order
    w, D = setup["w"], setup["D"]
    feats = pm.poly_features(D, w.box)
    s = sc.init_scorer(0)
    cap = int(setup["ids"].numel()) * 2 + 1024
    packed = pm.sig_pack(setup["sig"]) if method != "plain" else None
    common = dict(box=w.box, seed=0, k=256, cap=w.cap, bands=64, rows=4, n_queries=w.queries.n,
                  max_vertices=w.queries.xy.shape[0], cand_cap=cap, method=method, dsig=setup["sig"], scorer=s,
                  dfeat=feats, head=8, F=4, rounds=3, margin=float("inf") if method == "plain" else 0.02,
                  dpacked=packed, parts=parts)
    given = SplitBatch(D, setup["sk"], setup["se"], **common)
    given.load(w.queries)
    given.run_eager()
    w_ids, w_j = (x.clone() for x in given.result())
    z = SplitBatch(D, setup["sk"], setup["se"], query_order="morton", **common)
    z.load(w.queries)
    perm = spatial_order(w.queries)
    assert np.array_equal(z.perm, perm) and not np.array_equal(perm, np.arange(w.queries.n))
    # the first part holds the queries the curve visits first
    first = w.queries.subset(perm[:z.bounds[0][1]])
    assert np.array_equal(z.parts[0].off.cpu().numpy(), first.offsets)
    z.run_eager()
    e_ids, e_j = z.result()
    assert torch.equal(e_ids, w_ids) and torch.equal(e_j, w_j)
    if method != "plain":
        assert torch.equal(z.counts, given.counts)
    z.capture()
    for rep in range(2):
        for p in z.parts:
            p.top_ids.fill_(-7)
        torch.cuda.synchronize()
        z.run_graph()
        g_ids, g_j = z.result()
        assert torch.equal(g_ids, w_ids) and torch.equal(g_j, w_j), rep


@pytest.mark.parametrize("method,parts", [("plain", 3), ("jhat", 4), ("scorer", 2)])
def test_split_batch_equals_whole(pm, setup, method, parts):
    """The batch run as sub-batches of consecutive queries on their own
    streams, forked inside one captured graph: every replay (eager work of
    the program between them) and the eager run give the whole batch's
    top-10, and the early stop's counts add up to the whole batch's."""
    import torch
    from paper_2511_16576_amd import scorer as sc
    from paper_2511_16576_amd.pipeline import QueryBatch, SplitBatch
    w, D = setup["w"], setup["D"]
    feats = pm.poly_features(D, w.box)
    s = sc.init_scorer(0)
    cap = int(setup["ids"].numel()) * 2 + 1024
    common = dict(box=w.box, seed=0, k=256, cap=w.cap, bands=64, rows=4, n_queries=w.queries.n,
                  max_vertices=w.queries.xy.shape[0], cand_cap=cap, method=method, dsig=setup["sig"], scorer=s,
                  dfeat=feats, head=16, F=4, rounds=3, margin=float("inf") if method == "plain" else 0.02)
    whole = QueryBatch(D, setup["sk"], setup["se"], **common)
    whole.load(w.queries)
    whole.run_eager()
    w_ids, w_j = (x.clone() for x in whole.result())
    # the collision fraction of the sub-batches reads the saturated table
    packed = pm.sig_pack(setup["sig"]) if method == "jhat" else None
    split = SplitBatch(D, setup["sk"], setup["se"], parts=parts, dpacked=packed, **common)
    sizes = [b - a for a, b in split.bounds]
    assert split.bounds[0][0] == 0 and split.bounds[-1][1] == w.queries.n and max(sizes) - min(sizes) <= 1
    assert all(split.bounds[i][1] == split.bounds[i + 1][0] for i in range(parts - 1))
    split.load(w.queries)
    split.run_eager()
    e_ids, e_j = split.result()
    assert torch.equal(e_ids, w_ids) and torch.equal(e_j, w_j)
    if method != "plain":
        assert torch.equal(split.counts, whole.counts)
    split.capture()
    for rep in range(3):
        for p in split.parts:
            p.top_ids.fill_(-7)
        torch.cuda.synchronize()
        split.run_graph()
        g_ids, g_j = split.result()
        assert torch.equal(g_ids, w_ids) and torch.equal(g_j, w_j), rep
        pm.refine(D, whole.Q, whole.cand_off, whole.cand_ids, n_cand=whole.cand_ids.numel())
        torch.cuda.synchronize()
