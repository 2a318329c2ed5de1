"""GPU parity of the search path: bucket table, candidates (bit-exact),
refinement (within 1e-9 relative of the FP64 oracle; exact rationals on
small pairs) and top-k (exact)."""
from fractions import Fraction

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


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.cuda() if dtype is None else t.to(dtype).cuda()


def test_index_build_is_stable_sort(pm):
    rng = np.random.default_rng(0)
    for n, b in [(1, 1), (3, 5), (1000, 16), (40000, 32)]:
        keys = rng.integers(0, 2**63, (n, b), dtype=np.int64).view(np.uint64)
        keys[: n // 3] = keys[0]            # many duplicates
        keys[-1, -1] = 2**64 - 1
        sk, si = pm.index_build(_t(keys.view(np.int64)))
        sk = sk.cpu().numpy().view(np.uint64)
        si = si.cpu().numpy()
        flat = keys.reshape(-1)
        order = np.argsort(flat, kind="stable")
        assert np.array_equal(sk, flat[order]), (n, b)
        assert np.array_equal(si, order.astype(np.int32)), (n, b)


def test_query_matches_brute_force(pm, orc):
    rng = np.random.default_rng(1)
    for nd, nq, b, vals in [(500, 40, 6, 5), (3000, 17, 16, 50), (64, 3, 2, 2), (5, 0, 3, 4), (0, 4, 3, 4)]:
        dk = rng.integers(0, vals, (nd, b)).astype(np.uint64)
        qk = rng.integers(0, vals, (nq, b)).astype(np.uint64)
        qk[:, 0] += 10 ** 6                 # band 0 never matches
        sk, si = pm.index_build(_t(dk.view(np.int64)))
        off, ids = pm.query(sk, si, nd, _t(qk.view(np.int64)))
        ooff, oids = orc.candidates(dk, qk)
        assert np.array_equal(off.cpu().numpy(), ooff), (nd, nq, b)
        assert np.array_equal(ids.cpu().numpy(), oids), (nd, nq, b)



def test_query_large_data_set_sparse_lists(pm, orc):
    # 600,000 data polygons and 15,000 queries (bitmap rows of 18,750 words,
    # 1.1 GB in all): a query's bucket entries are gathered and sorted on
    # chip, and a query whose buckets hold more than 4,096 entries (5,000
    # polygons sharing every key) falls back to its bitmap row; on sampled
    # queries both lookup phases and the capped lookup equal the oracle's
    # candidates, and a capacity one short raises the flag and leaves
    # cand_ids untouched
    import torch
    rng = np.random.default_rng(21)
    nd, b, nq0 = 600_000, 8, 14_998
    dk = rng.integers(0, 200_000, (nd, b)).astype(np.uint64)
    popular = np.arange(b, dtype=np.uint64) + np.uint64(10 ** 9)
    dk[rng.choice(nd, 5000, replace=False)] = popular
    qk = dk[rng.integers(0, nd, nq0)].copy()
    qk[::2, :b // 2] += np.uint64(10 ** 7)        # half the bands never match on even queries
    qk = np.concatenate([qk, popular[None, :], popular[None, :] + np.uint64(10 ** 8)])
    nq = qk.shape[0]
    sample = np.concatenate([np.sort(rng.choice(nq0, 62, replace=False)), [nq - 2, nq - 1]])
    ooff, oids = orc.candidates(dk, qk[sample])
    want = [oids[ooff[i]:ooff[i + 1]] for i in range(sample.size)]
    assert want[-2].size == 5000 and want[-1].size == 0
    sk, si = pm.index_build(_t(dk.view(np.int64)))
    qkd = _t(qk.view(np.int64))

    def check(off, ids):
        for i, q in enumerate(sample):
            assert np.array_equal(ids[off[q]:off[q + 1]], want[i]), q
    off, ids = pm.query(sk, si, nd, qkd)
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    check(off, ids)
    total = int(off[-1])
    ws = torch.empty(int(pm.lib().polymh_query_workspace_size(nd, nq)), dtype=torch.uint8, device="cuda")
    assert ws.numel() > (1 << 30)
    coff = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    flag = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    cids = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    pm.query_capped(sk, si, nd, qkd, coff, cids, flag, ws)
    assert int(flag.item()) == 0
    assert np.array_equal(coff.cpu().numpy(), off) and np.array_equal(cids.cpu().numpy(), ids)
    short = torch.full((total - 1,), -7, dtype=torch.int32, device="cuda")
    pm.query_capped(sk, si, nd, qkd, coff, short, flag, ws)
    assert int(flag.item()) == 1
    assert (coff.cpu().numpy() == 0).all() and (short.cpu().numpy() == -7).all()

def test_query_sparse_lists_band_chunks_and_shared_keys(pm, orc):
    # the on-chip lists with 80 bands (two chunks of lanes), buckets of about
    # 1, 50 and 200 entries whose key values recur in other bands (the
    # band of every entry is checked), and a few queries whose one bucket
    # holds more than 4,096 entries (the bitmap takes those): sampled lists
    # equal the oracle's candidates
    rng = np.random.default_rng(22)
    nd, b, nq0 = 600_000, 80, 14_996
    dk = np.empty((nd, b), dtype=np.uint64)
    dk[:, :60] = rng.integers(0, 600_000, (nd, 60))
    dk[:, 60:70] = rng.integers(0, 12_000, (nd, 10))
    dk[:, 70:] = rng.integers(0, 3_000, (nd, 10))
    big = rng.choice(nd, 5000, replace=False)
    dk[big, 3] = np.uint64(10 ** 9)
    qk = dk[rng.integers(0, nd, nq0)].copy()
    qk = np.concatenate([qk, dk[big[:4]]])
    nq = qk.shape[0]
    sample = np.concatenate([np.sort(rng.choice(nq0, 60, replace=False)), np.arange(nq0, nq)])
    ooff, oids = orc.candidates(dk, qk[sample])
    sk, si = pm.index_build(_t(dk.view(np.int64)))
    off, ids = pm.query(sk, si, nd, _t(qk.view(np.int64)))
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    for i, q in enumerate(sample):
        assert np.array_equal(ids[off[q]:off[q + 1]], oids[ooff[i]:ooff[i + 1]]), q
    assert np.diff(off)[nq0:].min() > 5000 > np.median(np.diff(off)[:nq0])


def test_query_sparse_lists_every_sort_branch(pm, orc):
    # queries built to reach each way a gathered list is sorted: on a
    # wavefront (hash set with 1,024 / 1,025 / 2,048 / 2,049 members, raw
    # lists of exactly 4,096 entries, more than 3,008 distinct ids: sorted
    # whole), on a block (4,096 and 4,097 distinct ids, 2,000 ids met in
    # eight bands, 7,000 ids, 12,500 distinct ids and 12,200 with repeats:
    # sorted whole), a list past 16,384 entries (bitmap) and an empty one;
    # each list equals the oracle's candidates
    rng = np.random.default_rng(23)
    nd, b = 600_000, 64
    dk = rng.integers(0, 600_000, (nd, b)).astype(np.uint64)
    perm = rng.permutation(nd)
    groups = [(1024, 2), (1025, 3), (2048, 2), (2049, 1), (3100, 1), (4096, 2), (4097, 2), (2000, 8),
              (12_500, 1), (7000, 2), (9000, 2)]
    qrows = []
    at = 0
    for g, (size, bands) in enumerate(groups):
        members = perm[at:at + size]
        at += size
        q = np.uint64(2 * 10 ** 12) + np.uint64(100 * g) + np.arange(b, dtype=np.uint64)
        for t in range(bands):
            key = np.uint64(10 ** 12 + 1000 * g + t)
            dk[members, t] = key
            q[t] = key
        qrows.append(q)
    # 6,000 ids in band 0 and 6,500 in band 1, 300 of them in both
    a_set, b_set = perm[at:at + 6000], np.concatenate([perm[at:at + 300], perm[at + 6000:at + 12_200]])
    q = np.uint64(3 * 10 ** 12) + np.arange(b, dtype=np.uint64)
    dk[a_set, 0] = q[0] = np.uint64(4 * 10 ** 12)
    dk[b_set, 1] = q[1] = np.uint64(4 * 10 ** 12 + 1)
    qrows.append(q)
    qrows.append(np.uint64(5 * 10 ** 12) + np.arange(b, dtype=np.uint64))   # matches nothing
    nq0 = 14_990
    qk = np.concatenate([dk[rng.integers(0, nd, nq0)], np.stack(qrows)])
    nq = qk.shape[0]
    sample = np.concatenate([np.sort(rng.choice(nq0, 20, replace=False)), np.arange(nq0, nq)])
    ooff, oids = orc.candidates(dk, qk[sample])
    sizes = np.diff(ooff)[20:]
    assert list(sizes) == [1024, 1025, 2048, 2049, 3100, 4096, 4097, 2000, 12_500, 7000, 9000, 12_200, 0]
    sk, si = pm.index_build(_t(dk.view(np.int64)))
    off, ids = pm.query(sk, si, nd, _t(qk.view(np.int64)))
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    for i, q in enumerate(sample):
        assert np.array_equal(ids[off[q]:off[q + 1]], oids[ooff[i]:ooff[i + 1]]), (q, i)

def _pairs_all(nd, nq):
    off = np.arange(nq + 1, dtype=np.int64) * nd
    ids = np.tile(np.arange(nd, dtype=np.int32), nq)
    return off, ids


def _refine(pm, data, queries, off, ids):
    import torch
    D, Q = pm.to_device(data), pm.to_device(queries)
    J = pm.refine(D, Q, _t(off), _t(ids))
    torch.cuda.synchronize()
    return J.cpu().numpy()


def test_refine_workload1_against_oracle(pm, orc):
    w = dg.workload(1, n=300, n_queries=8)
    off, ids = _pairs_all(w.data.n, w.queries.n)
    got = _refine(pm, w.data, w.queries, off, ids)
    want = orc.jaccard_candidates(w.data, w.queries, off, ids)
    err = np.abs(got - want)
    assert np.all(err <= REL * np.abs(want) + ABS), (err.max(), np.argmax(err))
    assert (want > 0).sum() > 20


def test_refine_exact_rationals(pm, orc):
    rng = np.random.default_rng(3)
    data, queries = [], []
    for _ in range(30):
        c = rng.integers(0, 60, 2)
        data.append(dg.star_polygons(rng, [int(rng.integers(3, 10))], [c], [float(rng.uniform(8, 40))]).xy)
        queries.append(dg.star_polygons(rng, [int(rng.integers(3, 10))], [c + rng.integers(-15, 16, 2)],
                                        [float(rng.uniform(8, 40))]).xy)
    D, Q = dg.from_list(data), dg.from_list(queries)
    off = np.arange(31, dtype=np.int64)
    ids = np.arange(30, dtype=np.int32)
    got = _refine(pm, D, Q, off, ids)
    for i in range(30):
        ex = orc.jaccard_exact(data[i], queries[i])
        assert abs(got[i] - float(ex)) <= REL * float(ex) + ABS, (i, got[i], float(ex))


def test_refine_degenerate_contacts(pm, orc):
    sq = dg.rectangle(0, 0, 10, 10)
    tri = np.array([[0, 0], [10, 0], [0, 10]])
    cases = [
        (sq, sq, Fraction(1)),                                   # identical
        (sq, sq[::-1], Fraction(1)),                             # opposite orientation
        (sq, np.roll(sq, 2, axis=0), Fraction(1)),               # rotated start
        (sq, dg.rectangle(10, 0, 20, 10), Fraction(0)),          # shared edge
        (sq, dg.rectangle(10, 10, 20, 20), Fraction(0)),         # shared corner
        (sq, dg.rectangle(5, 0, 15, 10), Fraction(50, 150)),     # collinear overlapping edges
        (sq, dg.rectangle(0, 0, 5, 5), Fraction(25, 100)),       # nested, shared corner
        (sq, dg.rectangle(2, 0, 8, 10), Fraction(60, 100)),      # T-junctions
        (sq, tri, Fraction(50, 100)),                            # shared diagonal endpoints
        (tri, np.array([[0, 0], [10, 0], [10, 10]]), Fraction(25, 75)),
        (sq, np.array([[5, 0], [10, 5], [5, 10], [0, 5]]), Fraction(50, 100)),  # vertices on edges
        (sq, np.array([[0, 0], [4, 4], [10, 0]]), Fraction(20, 100)),
        (sq, np.array([[0, 0], [0, 0], [10, 0], [10, 10]]), Fraction(50, 100)),  # repeated vertex
    ]
    D = dg.from_list([c[0] for c in cases])
    Q = dg.from_list([c[1] for c in cases])
    off = np.arange(len(cases) + 1, dtype=np.int64)
    ids = np.arange(len(cases), dtype=np.int32)
    got = _refine(pm, D, Q, off, ids)
    for i, (_, _, want) in enumerate(cases):
        assert abs(got[i] - float(want)) <= 1e-12, (i, got[i], want)
        assert orc.jaccard_exact(cases[i][0], cases[i][1]) == want, i


def test_refine_wide_coordinates(pm, orc):
    # MBR spans beyond 2^26: the 128-bit orientation path
    a = dg.rectangle(-(1 << 27), -(1 << 27), 1 << 27, 1 << 27)
    b = dg.rectangle(0, -(1 << 26), 1 << 28, 1 << 26)
    rng = np.random.default_rng(4)
    s = dg.star_polygons(rng, [20], [[0, 0]], [float(1 << 27)]).xy
    D, Q = dg.from_list([a, s, s]), dg.from_list([b, a, s])
    got = _refine(pm, D, Q, np.arange(4, dtype=np.int64), np.arange(3, dtype=np.int32))
    for i, (P, R) in enumerate([(a, b), (s, a), (s, s)]):
        want = float(orc.jaccard_exact(P, R))
        assert abs(got[i] - want) <= 1e-9 * want + ABS, (i, got[i], want)


def test_topk_exact(pm, orc):
    import torch
    rng = np.random.default_rng(5)
    nq = 50
    counts = rng.integers(0, 300, nq)
    counts[3] = 0
    counts[7] = 4
    off = np.zeros(nq + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    ids = np.concatenate([np.sort(rng.choice(10000, c, replace=False)) for c in counts]).astype(np.int32)
    J = np.round(rng.random(ids.shape[0]), 2)        # many ties
    for k in (1, 10, 64):
        ti, tj = pm.topk(_t(off), _t(ids), _t(J), k)
        torch.cuda.synchronize()
        oi, oj = orc.topk(off, ids, J, k)
        assert np.array_equal(ti.cpu().numpy(), oi), k
        assert np.array_equal(tj.cpu().numpy(), oj), k


def test_pipeline_workload1_recall(pm, orc):
    """Sign, band, index, query, refine and top-10 on workload 1; every stage
    equals the oracle and recall@10 is computed against brute force."""
    import torch
    w = dg.workload(1)
    D, Q = pm.to_device(w.data), pm.to_device(w.queries)
    sig = pm.sign(D, w.box, w.seed, w.k, w.cap)
    qsig = pm.sign(Q, w.box, w.seed, w.k, w.cap)
    keys = pm.band(sig, w.bands, w.rows, w.seed)
    qkeys = pm.band(qsig, w.bands, w.rows, w.seed)
    sk, si = pm.index_build(keys)
    off, ids = pm.query(sk, si, D.n, qkeys)
    J = pm.refine(D, Q, off, ids)
    ti, tj = pm.topk(off, ids, J, 10)
    torch.cuda.synchronize()
    okeys = orc.band(orc.sign(w.data, w.box, w.seed, w.k, w.cap), w.bands, w.rows, w.seed)
    oqkeys = orc.band(orc.sign(w.queries, w.box, w.seed, w.k, w.cap), w.bands, w.rows, w.seed)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), okeys)
    ooff, oids = orc.candidates(okeys, oqkeys)
    assert np.array_equal(off.cpu().numpy(), ooff)
    assert np.array_equal(ids.cpu().numpy(), oids)
    oJ = orc.jaccard_candidates(w.data, w.queries, ooff, oids)
    gJ = J.cpu().numpy()
    assert np.all(np.abs(gJ - oJ) <= REL * np.abs(oJ) + ABS)
    oti, otj = orc.topk(ooff, oids, gJ, 10)
    assert np.array_equal(ti.cpu().numpy(), oti)
    bi, bj = orc.brute_force_topk(w.data, w.queries, 10)
    rec = orc.recall_at_k(ti.cpu().numpy(), tj.cpu().numpy(), bi, bj, 10)
    print(f"workload 1: recall@10 = {rec:.3f}, {ids.numel()} candidates for {Q.n} queries")
    assert 0.0 < rec <= 1.0
    # the jittered source is found for every query
    assert all(int(w.query_source[q]) in set(oids[ooff[q]:ooff[q + 1]].tolist()) for q in range(Q.n))


def test_refine_lattice_degeneracies(pm, orc):
    # small stars on a 7 x 7 grid share many vertices, T-junctions and
    # collinear edge overlaps: every area must equal the exact rational one
    rng = np.random.default_rng(6)
    data, queries = [], []
    for _ in range(150):
        data.append(dg.star_polygons(rng, [int(rng.integers(3, 7))], [[3, 3]], [3.0]).xy)
        q = dg.star_polygons(rng, [int(rng.integers(3, 7))], [[3, 3]], [3.0]).xy
        queries.append(q if rng.random() < 0.5 else q[::-1])
    D, Q = dg.from_list(data), dg.from_list(queries)
    got = _refine(pm, D, Q, np.arange(151, dtype=np.int64), np.arange(150, dtype=np.int32))
    for i in range(150):
        want = float(orc.jaccard_exact(data[i], queries[i]))
        assert abs(got[i] - want) <= 1e-12, (i, got[i], want)


def test_refine_large_polygons_general_path(pm, orc):
    # polygons beyond the tiled form's 512-edge staging cap
    rng = np.random.default_rng(7)
    data = dg.star_polygons(rng, [600, 1500, 40, 2000], [[50000, 50000]] * 4, [40000.0] * 4)
    queries = dg.star_polygons(rng, [1200, 30, 900], [[52000, 49000]] * 3, [38000.0] * 3)
    off = np.array([0, 4, 8, 12], dtype=np.int64)
    ids = np.tile(np.arange(4, dtype=np.int32), 3)
    got = _refine(pm, data, queries, off, ids)
    want = orc.jaccard_candidates(data, queries, off, ids)
    assert np.all(np.abs(got - want) <= REL * np.abs(want) + ABS), np.abs(got - want).max()


def test_refine_heavy_pairs_split(pm, orc):
    # with the workspace, every pair with coordinate spans below 2^26 takes
    # the tiled form (in windows beyond 1024 edges) where the in-place call
    # takes the general form beyond 512 edges: the values equal the oracle's
    # and the in-place form's, and the work counts move by exactly those
    # pairs
    import torch
    rng = np.random.default_rng(8)
    data = dg.star_polygons(rng, [600, 1500, 40, 2000, 3000], [[50000, 50000]] * 5, [40000.0] * 5)
    queries = dg.star_polygons(rng, [1200, 30, 900, 2500], [[52000, 49000]] * 4, [38000.0] * 4)
    D, Q = pm.to_device(data), pm.to_device(queries)
    off = torch.tensor([0, 5, 10, 15, 20], dtype=torch.int64, device="cuda")
    ids = torch.arange(5, dtype=torch.int32, device="cuda").repeat(4)
    split, st_split = pm.refine_stats(D, Q, off, ids)
    inplace, st_inplace = pm.refine_stats(D, Q, off, ids, split_heavy=False)
    want = orc.jaccard_candidates(data, queries, off.cpu().numpy(), ids.cpu().numpy())
    got = split.cpu().numpy()
    assert np.all(np.abs(got - want) <= REL * np.abs(want) + ABS), np.abs(got - want).max()
    assert np.all(np.abs(got - inplace.cpu().numpy()) <= REL * np.abs(want) + ABS)
    n = data.counts()[ids.cpu().numpy()]
    m = np.repeat(queries.counts(), 5)
    moved = np.maximum(n, m) > 512
    assert moved.sum() == 19 and ((n > 1024) & (m > 1024)).sum() == 6
    assert st_split[0] == 20 and st_split[2] == 0
    assert st_split[0] == st_inplace[0] + moved.sum()
    assert st_inplace[2] == int((2 * n * m)[moved].sum())
    assert st_split[3] == st_inplace[3]


def test_refine_more_heavy_pairs_than_the_split_list(pm):
    # 8,400 heavy pairs (400 x 400 edges, n m >= 2^17, coordinate spans
    # beyond 2^26, so the general form with 128-bit signs): the first 8,192
    # are split, the rest run in place; every value equals the in-place
    # form's
    import torch
    rng = np.random.default_rng(9)
    big = float(1 << 26)
    data = dg.star_polygons(rng, [400] * 120, [[50000 * i, 0] for i in range(120)], [big] * 120)
    queries = dg.star_polygons(rng, [400] * 70, [[0, 40000 * i] for i in range(70)], [big] * 70)
    D, Q = pm.to_device(data), pm.to_device(queries)
    off = torch.arange(71, dtype=torch.int64, device="cuda") * 120
    ids = torch.arange(120, dtype=torch.int32, device="cuda").repeat(70)
    split = pm.refine(D, Q, off, ids).cpu().numpy()
    inplace = pm.refine(D, Q, off, ids, split_heavy=False).cpu().numpy()
    assert (inplace > 0.2).all()
    assert np.all(np.abs(split - inplace) <= 1e-12 + 1e-12 * np.abs(inplace))


def test_refine_more_split_pairs_than_the_split_list(pm):
    # 8,400 pairs of two 1,100-edge polygons: each is split into five P
    # windows of 256 edges (one wavefront each, added up by the finish)
    # while split slots last (4,096), the rest take both windows on one
    # wavefront;
    # every value equals the general form's (the call without workspace)
    import torch
    rng = np.random.default_rng(14)
    data = dg.star_polygons(rng, [1100] * 120, [[50000 + 50 * i, 50000] for i in range(120)], [30000.0] * 120)
    queries = dg.star_polygons(rng, [1100] * 70, [[51000, 49000 + 30 * i] for i in range(70)], [30000.0] * 70)
    D, Q = pm.to_device(data), pm.to_device(queries)
    off = torch.arange(71, dtype=torch.int64, device="cuda") * 120
    ids = torch.arange(120, dtype=torch.int32, device="cuda").repeat(70)
    split, st = pm.refine_stats(D, Q, off, ids)
    split = split.cpu().numpy()
    inplace = pm.refine(D, Q, off, ids, split_heavy=False).cpu().numpy()
    assert (inplace > 0.2).all()
    assert np.all(np.abs(split - inplace) <= REL * np.abs(inplace) + ABS), np.abs(split - inplace).max()
    assert st[0] == 8400 and st[2] == 0

def test_refine_heavy_pairs_wide_coordinates(pm, orc):
    # large pairs whose coordinate span needs the 128-bit orientation form,
    # split over wavefronts like the others
    import torch
    rng = np.random.default_rng(10)
    big = float(1 << 27)
    data = dg.star_polygons(rng, [700, 900], [[0, 0], [1 << 20, 0]], [big, big])
    queries = dg.star_polygons(rng, [800, 650], [[1 << 19, 1 << 19], [0, 1 << 21]], [big, big])
    D, Q = pm.to_device(data), pm.to_device(queries)
    off = torch.tensor([0, 2, 4], dtype=torch.int64, device="cuda")
    ids = torch.tensor([0, 1, 0, 1], dtype=torch.int32, device="cuda")
    got, st = pm.refine_stats(D, Q, off, ids)
    want = orc.jaccard_candidates(data, queries, off.cpu().numpy(), ids.cpu().numpy())
    got = got.cpu().numpy()
    assert st[2] > 0 and (want > 0.3).all()
    assert np.all(np.abs(got - want) <= REL * np.abs(want) + ABS), np.abs(got - want).max()
    inplace = pm.refine(D, Q, off, ids, split_heavy=False).cpu().numpy()
    assert np.all(np.abs(got - inplace) <= 1e-12 + 1e-12 * np.abs(want))


def test_refine_wide_tiled_pairs(pm, orc):
    # pairs with a polygon of 513 to 1024 edges (none beyond) take the tiled
    # form in a second launch, one wavefront staging both rings: the values
    # equal the oracle's and the general form's, and every pair is counted as
    # tiled
    import torch
    rng = np.random.default_rng(11)
    data = dg.star_polygons(rng, [513, 1024, 700, 40, 900, 8], [[50000, 50000]] * 6, [40000.0] * 6)
    queries = dg.star_polygons(rng, [1000, 30, 513, 800, 1024], [[52000, 49000]] * 5, [38000.0] * 5)
    D, Q = pm.to_device(data), pm.to_device(queries)
    off = torch.arange(6, dtype=torch.int64, device="cuda") * 6
    ids = torch.arange(6, dtype=torch.int32, device="cuda").repeat(5)
    got, st = pm.refine_stats(D, Q, off, ids)
    inplace, st0 = pm.refine_stats(D, Q, off, ids, split_heavy=False)
    want = orc.jaccard_candidates(data, queries, off.cpu().numpy(), ids.cpu().numpy())
    got, inplace = got.cpu().numpy(), inplace.cpu().numpy()
    assert (want > 0.2).sum() >= 25
    assert np.all(np.abs(got - want) <= REL * np.abs(want) + ABS), np.abs(got - want).max()
    assert np.all(np.abs(inplace - want) <= REL * np.abs(want) + ABS)
    assert st[0] == 30 and st[2] == 0 and st[1] > 0
    assert st0[2] > 0


def _subdivided_rect(x0, y0, x1, y1, k):
    """Counter-clockwise rectangle with k vertices per side (all on its edges)."""
    i = np.arange(k)
    w, h = x1 - x0, y1 - y0
    return np.concatenate([np.stack([x0 + w * i // k, np.full(k, y0)], 1),
                           np.stack([np.full(k, x1), y0 + h * i // k], 1),
                           np.stack([x1 - w * i // k, np.full(k, y1)], 1),
                           np.stack([np.full(k, x0), y1 - h * i // k], 1)]).astype(np.int64)


def test_ranked_rounds_split_large_pairs(pm):
    """The early-stop rounds' refinement splits pairs with very large
    polygons as refine does (P windows of 128 edges for a staged polygon of
    4,096 edges or more, up to 512 units a pair): 6,000-vertex squares
    (128-edge P windows, each with one of the 6 Q windows), 9,000-vertex
    squares (256-edge windows) and 20,000-vertex squares (1,024-edge
    windows, each with one of the 20 Q windows) give the exact J through
    the ranked rounds, equal to refine's."""
    import torch
    L6, L9, L20 = 6000, 9000, 20000
    a6 = _subdivided_rect(0, 0, L6, L6, 1500)
    a9 = _subdivided_rect(0, 0, L9, L9, 2250)
    a20 = _subdivided_rect(0, 0, L20, L20, 5000)
    cases = [
        (a6, a6, Fraction(1)), (a6, _subdivided_rect(L6 // 2, 0, L6 // 2 + L6, L6, 1500), Fraction(1, 3)),
        (a6[::-1], a6, Fraction(1)),
        (a9, a9, Fraction(1)), (a9, _subdivided_rect(L9 // 2, 0, L9 // 2 + L9, L9, 2250), Fraction(1, 3)),
        (a20, _subdivided_rect(L20 // 2, 0, L20 // 2 + L20, L20, 5000), Fraction(1, 3)),
    ]
    D = pm.to_device(dg.from_list([c[0] for c in cases]))
    Q = pm.to_device(dg.from_list([c[1] for c in cases]))
    n = len(cases)
    off = torch.arange(n + 1, dtype=torch.int64, device="cuda")
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    score = torch.zeros(n, dtype=torch.float32, device="cuda")
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    ok = torch.empty(n, dtype=torch.uint8, device="cuda")
    pm.rank_order(off, score, order, ok)
    t_ids, t_j, cnt = pm.rank_refine_ordered(D, Q, off, ids, score, order, ok, topk=1, F=1, rounds=1,
                                             margin=float("inf"))
    got = t_j.cpu().numpy()[:, 0]
    for j, (_, _, want) in enumerate(cases):
        assert abs(got[j] - float(want)) <= 1e-12, (j, got[j], want)
    assert (t_ids.cpu().numpy()[:, 0] == np.arange(n)).all()
    coarse = pm.refine(D, Q, off, ids).cpu().numpy()
    assert np.allclose(got, coarse, rtol=1e-12, atol=1e-12)


def test_refine_wide_tiled_degenerate_contacts(pm, orc):
    # the degenerate contacts of the small cases at 513 to 1024 edges: every
    # side of a 400 x 400 square carries 200 (or 150) vertices, so edges
    # overlap collinearly, vertices lie on edges and shapes share corners
    L = 400
    sq = _subdivided_rect(0, 0, L, L, 200)                     # 800 vertices
    sq6 = _subdivided_rect(0, 0, L, L, 150)                    # 600 vertices, every third shared
    k = 200
    i = np.arange(k)
    tri = np.concatenate([np.stack([L * i // k, np.zeros(k, np.int64)], 1),
                          np.stack([L - L * i // k, L * i // k], 1),
                          np.stack([np.zeros(k, np.int64), L - L * i // k], 1)])   # 600 vertices
    cases = [
        (sq, sq, Fraction(1)),                                   # identical
        (sq, sq[::-1], Fraction(1)),                             # opposite orientation
        (sq, np.roll(sq, 337, axis=0), Fraction(1)),             # rotated start
        (sq, sq6, Fraction(1)),                                  # same square, other subdivision
        (sq, dg.rectangle(0, 0, L, L), Fraction(1)),
        (sq, _subdivided_rect(L, 0, 2 * L, L, 200), Fraction(0)),               # shared edge
        (sq, _subdivided_rect(L, L, 2 * L, 2 * L, 200), Fraction(0)),           # shared corner
        (sq, _subdivided_rect(L // 2, 0, L // 2 + L, L, 200), Fraction(1, 3)),  # collinear overlaps
        (sq, dg.rectangle(0, 0, L // 2, L // 2), Fraction(1, 4)),               # nested, shared corner
        (sq, dg.rectangle(80, 0, 320, L), Fraction(60, 100)),                   # T-junctions
        (sq, tri, Fraction(1, 2)),                               # shared diagonal endpoints
        (tri, sq6, Fraction(1, 2)),
        (sq, np.array([[L // 2, 0], [L, L // 2], [L // 2, L], [0, L // 2]]), Fraction(1, 2)),  # vertices on edges
    ]
    D = dg.from_list([c[0] for c in cases])
    Q = dg.from_list([c[1] for c in cases])
    off = np.arange(len(cases) + 1, dtype=np.int64)
    ids = np.arange(len(cases), dtype=np.int32)
    got = _refine(pm, D, Q, off, ids)
    for j, (_, _, want) in enumerate(cases):
        assert abs(got[j] - float(want)) <= 1e-12, (j, got[j], want)
    want = orc.jaccard_candidates(D, Q, off, ids)
    assert np.all(np.abs(want - np.array([float(c[2]) for c in cases])) <= 1e-9)


def test_refine_windowed_pairs(pm, orc):
    # a polygon of at most 1024 edges against one of any length: the small
    # one is staged whole (the query when the data polygon is the larger),
    # the other passes in windows of 1024 edges (2,048: two full windows;
    # 1,025: a last window of one edge); pairs with both beyond 1024 edges
    # stay on the general form
    import torch
    rng = np.random.default_rng(13)
    data = dg.star_polygons(rng, [3000, 20, 1025, 2048, 700, 8], [[50000, 50000]] * 6, [40000.0] * 6)
    queries = dg.star_polygons(rng, [40, 5000, 1100, 300, 1025], [[52000, 49000]] * 5, [38000.0] * 5)
    D, Q = pm.to_device(data), pm.to_device(queries)
    off = torch.arange(6, dtype=torch.int64, device="cuda") * 6
    ids = torch.arange(6, dtype=torch.int32, device="cuda").repeat(5)
    got, st = pm.refine_stats(D, Q, off, ids)
    inplace = pm.refine(D, Q, off, ids, split_heavy=False).cpu().numpy()
    want = orc.jaccard_candidates(data, queries, off.cpu().numpy(), ids.cpu().numpy())
    got = got.cpu().numpy()
    assert (want > 0.2).sum() >= 25
    assert np.all(np.abs(got - want) <= REL * np.abs(want) + ABS), np.abs(got - want).max()
    assert np.all(np.abs(inplace - want) <= REL * np.abs(want) + ABS)
    n = data.counts()[ids.cpu().numpy()]
    m = np.repeat(queries.counts(), 6)
    assert ((n > 1024) & (m > 1024)).sum() == 9     # windows on both sides
    assert st[0] == 30 and st[2] == 0


def test_refine_windowed_degenerate_contacts(pm, orc):
    # exact J with a 3,200-vertex square (800 collinear vertices a side, four
    # windows) on either side of the pair: shared and collinear edges,
    # corners, T-junctions, vertices on edges, a small square inside it (no
    # vertex of the small polygon outside the other's MBR) and a square
    # around it (no vertex of the large one outside the other's MBR)
    L = 1600
    big = _subdivided_rect(0, 0, L, L, 800)
    others = [
        (dg.rectangle(0, 0, L, L), Fraction(1)),
        (_subdivided_rect(0, 0, L, L, 200), Fraction(1)),
        (_subdivided_rect(L, 0, 2 * L, L, 200), Fraction(0)),                   # shared edge
        (dg.rectangle(L, L, 2 * L, 2 * L), Fraction(0)),                        # shared corner
        (_subdivided_rect(L // 2, 0, L // 2 + L, L, 200), Fraction(1, 3)),      # collinear overlaps
        (dg.rectangle(0, 0, L // 2, L // 2), Fraction(1, 4)),                   # nested, shared corner
        (dg.rectangle(320, 0, 1280, L), Fraction(60, 100)),                     # T-junctions
        (np.array([[L // 2, 0], [L, L // 2], [L // 2, L], [0, L // 2]]), Fraction(1, 2)),  # vertices on edges
        (dg.rectangle(400, 400, 800, 800), Fraction(1, 16)),                    # inside, away from the edges
        (dg.rectangle(-10, -10, L + 10, L + 10), Fraction(L * L, (L + 20) ** 2)),  # around it
    ]
    # the large square as the query, then as the data polygon; then both
    # large (windows on both sides)
    cases = [(o, big, j) for o, j in others] + [(big, o, j) for o, j in others] + [
        (big, big, Fraction(1)), (big, big[::-1], Fraction(1)), (big, np.roll(big, 1234, axis=0), Fraction(1)),
        (big, _subdivided_rect(L // 2, 0, L // 2 + L, L, 800), Fraction(1, 3)),
        (big, _subdivided_rect(L, 0, 2 * L, L, 800), Fraction(0))]
    D = dg.from_list([c[0] for c in cases])
    Q = dg.from_list([c[1] for c in cases])
    off = np.arange(len(cases) + 1, dtype=np.int64)
    ids = np.arange(len(cases), dtype=np.int32)
    got = _refine(pm, D, Q, off, ids)
    for j, (_, _, want) in enumerate(cases):
        assert abs(got[j] - float(want)) <= 1e-12, (j, got[j], want)
    want = orc.jaccard_candidates(D, Q, off, ids)
    assert np.all(np.abs(want - np.array([float(c[2]) for c in cases])) <= 1e-9)


def test_refine_split_units_exact(pm):
    # exact J for pairs split into units of each shape: 6,000-vertex squares
    # (P windows of 128 edges, each with one of the 6 Q windows), 9,000-vertex
    # squares (P windows of 256 edges, each with one of the 9 Q windows:
    # windows of 128 would give more than 512 units), 20,000-vertex squares
    # (P windows of 1,024 edges, each with one of the 20 Q windows),
    # 30,000-vertex squares (P windows of 128 edges walking all 30 Q windows:
    # a unit per Q window would exceed the cap at any window length) and a
    # 4-vertex rectangle against a 20,000-vertex square, either way round
    # (one P window, each of the 20 Q windows a unit of its own); collinear
    # overlaps, shared edges and a reversed ring included; and flat chains
    # (zero area, J = 0) of 6,000 and 9,000 vertices inside a square's MBR,
    # the data polygon staged as P in the first and as Q in the second
    import torch
    L6, L9, L20, L30 = 6000, 9000, 20000, 30000
    a6 = _subdivided_rect(0, 0, L6, L6, 1500)
    a9 = _subdivided_rect(0, 0, L9, L9, 2250)
    a20 = _subdivided_rect(0, 0, L20, L20, 5000)
    a30 = _subdivided_rect(0, 0, L30, L30, 7500)
    small = dg.rectangle(1000, 1000, 3000, 5000)

    def flat(n):
        x = np.concatenate([2 * np.arange(n // 2), 2 * (n // 2) - 1 - 2 * np.arange(n // 2)])
        return np.stack([x, np.full(n, 3000)], 1).astype(np.int64)
    cases = [
        (a6, a6, Fraction(1)), (a6, _subdivided_rect(L6 // 2, 0, L6 // 2 + L6, L6, 1500), Fraction(1, 3)),
        (a9, a9, Fraction(1)), (a9, a9[::-1], Fraction(1)),
        (a9, _subdivided_rect(L9 // 2, 0, L9 // 2 + L9, L9, 2250), Fraction(1, 3)),
        (a9, _subdivided_rect(L9, 0, 2 * L9, L9, 2250), Fraction(0)),
        (a20, a20, Fraction(1)),
        (a20, _subdivided_rect(L20 // 2, 0, L20 // 2 + L20, L20, 5000), Fraction(1, 3)),
        (a30, _subdivided_rect(L30 // 2, 0, L30 // 2 + L30, L30, 7500), Fraction(1, 3)),
        (small, a20, Fraction(2000 * 4000, L20 * L20)),
        (a20, small, Fraction(2000 * 4000, L20 * L20)),
        (flat(6000), a6, Fraction(0)), (flat(9000), a6, Fraction(0)),
    ]
    D = pm.to_device(dg.from_list([c[0] for c in cases]))
    Q = pm.to_device(dg.from_list([c[1] for c in cases]))
    off = torch.arange(len(cases) + 1, dtype=torch.int64, device="cuda")
    ids = torch.arange(len(cases), dtype=torch.int32, device="cuda")
    got, st = pm.refine_stats(D, Q, off, ids)
    got = got.cpu().numpy()
    for j, (_, _, want) in enumerate(cases):
        assert abs(got[j] - float(want)) <= 1e-12, (j, got[j], want)
    # the pair sharing an edge has MBRs that only touch: counted disjoint
    assert st[0] == len(cases) - 1 and st[3] == 1 and st[2] == 0
