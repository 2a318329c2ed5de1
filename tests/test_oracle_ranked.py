"""Pins of the oracle's best-first refinement with early stop and of the
collision fraction that orders it (Thm. 1, Def. 1)."""
import math
import os

import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "early_stop_cases.txt")


def _golden():
    cand, cases = {}, []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("cand "):
                _, pos, i, s, j = line.split()
                cand[int(pos)] = (int(i), float(s), float(j))
            else:
                head, ids, js, tail = (x.strip() for x in line[len("case "):].split("|"))
                k, F, rounds, margin, limit = head.split()
                refined, fin = tail.split()
                cases.append(dict(k=int(k), F=int(F), rounds=int(rounds), margin=float(margin), limit=int(limit),
                                  ids=[int(x) for x in ids.split()], j=[float(x) for x in js.split()],
                                  refined=int(refined), finished=bool(int(fin))))
    n = len(cand)
    ids = np.array([cand[p][0] for p in range(n)])
    score = np.array([cand[p][1] for p in range(n)], dtype=np.float32)
    J = np.array([cand[p][2] for p in range(n)])
    return ids, score, J, cases


def test_golden_cases():
    import oracle
    ids, score, J, cases = _golden()
    assert len(cases) >= 10
    order, ok = oracle.best_first(score)
    assert ok and order.tolist() == [1, 2, 4, 7, 9, 0, 5, 8, 3, 6]
    for c in cases:
        seen = []
        r = oracle.early_stop_query(ids, score, lambda pos: (seen.extend(pos.tolist()), J[pos])[1], c["k"], c["F"],
                                    c["rounds"], c["margin"], sort_limit=c["limit"])
        assert r["top_ids"].tolist() == c["ids"], c
        assert r["top_j"].tolist() == c["j"], c
        assert r["refined"] == c["refined"] and r["finished"] == c["finished"], c
        # every candidate refined exactly once, and only those
        assert len(seen) == len(set(seen)) == c["refined"], c


def _random_lists(seed, nq=40, max_n=70, tie_levels=24):
    """Candidate CSR with unique ids per query, J and predictions on coarse
    dyadic grids (many ties, every value exact in FP32)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, max_n, nq)
    counts[:3] = (0, 1, 9)
    off = np.zeros(nq + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    ids = np.concatenate([rng.choice(500, c, replace=False) for c in counts]).astype(np.int32)
    J = rng.integers(0, tie_levels + 1, ids.size) / tie_levels
    J = np.round(J * 1024) / 1024
    score = (rng.integers(0, 64, ids.size) / 64).astype(np.float32)
    return off, ids, J, score


@pytest.mark.parametrize("F,rounds", [(1, 0), (1, 1), (3, 2), (8, 4), (5, 6)])
def test_infinite_margin_refines_everything(F, rounds):
    """m = +inf never stops: the result is Def. 1's top-k of the whole list,
    every pair is refined, and the finishing pass completes exactly the
    queries whose lists outlast the rounds (F 2^(r-1) candidates after r >= 1
    rounds)."""
    import oracle
    off, ids, J, score = _random_lists(F * 10 + rounds)
    r = oracle.early_stop_topk(off, ids, score, J, 10, F, rounds, float("inf"))
    ti, tj = oracle.topk(off, ids, J, 10)
    assert np.array_equal(r["top_ids"], ti) and np.array_equal(r["top_j"], tj)
    assert r["refined"] == ids.size
    seen = F * 2 ** (rounds - 1) if rounds else 0
    assert r["finished"] == int((np.diff(off) > seen).sum())
    assert r["min_gap"] == float("inf")


@pytest.mark.parametrize("F,rounds", [(4, 3), (8, 4), (2, 6)])
def test_exact_predictions_give_exact_topk(F, rounds):
    """With the exact J as the prediction and margin 0 the stop is exact:
    the next candidate has the largest J left, so nothing unrefined can beat
    the k-th; the top-k J values equal the full top-k's (ids too, except
    among candidates tied with the k-th J), with fewer pairs refined."""
    import oracle
    off, ids, J, _ = _random_lists(100 + F, nq=60, max_n=120)
    r = oracle.early_stop_topk(off, ids, J.astype(np.float32), J, 10, F, rounds, 0.0)
    ti, tj = oracle.topk(off, ids, J, 10)
    assert np.array_equal(r["top_j"], tj)
    for q in range(off.size - 1):
        kth = tj[q, -1]
        assert set(r["top_ids"][q][tj[q] > kth]) == set(ti[q][tj[q] > kth]), q
    assert r["refined"] < ids.size


def test_margin_trades_pairs_for_exactness():
    """A larger margin never refines fewer pairs (each stop test only gets
    harder), and at a margin above the largest possible J the early stop
    never fires."""
    import oracle
    off, ids, J, score = _random_lists(7, nq=50, max_n=100)
    prev = -1
    for m in (-0.5, -0.1, 0.0, 0.05, 0.2, 0.6):
        r = oracle.early_stop_topk(off, ids, score, J, 10, 2, 4, m)
        assert r["refined"] >= prev
        prev = r["refined"]
    r = oracle.early_stop_topk(off, ids, score, J, 10, 2, 4, 1.5)
    full = oracle.early_stop_topk(off, ids, score, J, 10, 2, 4, float("inf"))
    assert r["refined"] == full["refined"] and np.array_equal(r["top_ids"], full["top_ids"])


def test_best_first_is_the_sort():
    import oracle
    rng = np.random.default_rng(3)
    for n in (0, 1, 2, 17, 300):
        s = (rng.integers(0, 5, n) / 4).astype(np.float32)
        order, ok = oracle.best_first(s)
        assert ok and sorted(order.tolist()) == list(range(n))
        for a, b in zip(order[:-1], order[1:]):
            assert s[a] > s[b] or (s[a] == s[b] and a < b)
    s = rng.random(20).astype(np.float32)
    order, ok = oracle.best_first(s, sort_limit=19)
    assert not ok and order.tolist() == list(range(20))


@pytest.mark.parametrize("pair", [
    ((0, 0, 40, 40), (20, 10, 60, 50)),     # J = 600/2600
    ((0, 0, 40, 40), (4, 0, 44, 40)),       # J = 1440/1760
    ((10, 10, 50, 50), (20, 20, 30, 30)),   # nested: J = 100/1600
    ((0, 0, 40, 40), (60, 60, 70, 70)),     # disjoint: J = 0
])
def test_collision_fraction_estimates_jaccard(orc, pair):
    """Thm. 1 on rectangle pairs of closed-form J: the share of agreeing
    hashes concentrates at J; a polygon against itself agrees everywhere."""
    import oracle
    a, b = pair
    inter = max(0, min(a[2], b[2]) - max(a[0], b[0])) * max(0, min(a[3], b[3]) - max(a[1], b[1]))
    area = lambda r: (r[2] - r[0]) * (r[3] - r[1])
    Jc = inter / (area(a) + area(b) - inter)
    k = 4096
    sig = orc.sign(dg.from_list([dg.rectangle(*a), dg.rectangle(*b)]), (0, 0, 255, 255), seed=5, k=k, cap=1 << 30)
    est = oracle.collision_fraction(sig[0], sig[1:])[0]
    assert abs(est - Jc) <= 5 * math.sqrt(max(Jc * (1 - Jc), 1e-4) / k)
    assert oracle.collision_fraction(sig[0], sig)[0] == 1.0
    assert oracle.collision_counts(sig[0], sig[0] + 1)[0] == 0
