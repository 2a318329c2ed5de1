"""Best-first refinement with early stop -- CPU oracle, TEST INFRASTRUCTURE ONLY.

Not a step of the paper's own method: the learned-scorer form orders each
query's LSH candidates by a predicted J and refines them best first, so that
refinement can end before the list does, with full refinement of every
candidate as the fallback.  This module states plainly, one query at a time,
what that computes.  Only the test suite, the package's smoke check and the
CPU baseline leg of the benchmark use it; it shares no code with the GPU
library.

- ``collision_counts`` / ``collision_fraction``: Thm. 1.  For one hash, the
  probability that two polygons' values agree is their Jaccard J, so the
  share of agreeing values among k hashes is an unbiased estimate of J.
  Pinned by Thm. 1 on rectangle pairs whose J has a closed form (the share
  concentrates at J), by share(P, P) = 1, and by share 0 for signatures
  that have no value in common.
- ``best_first``: a query's candidate positions by decreasing predicted J,
  equal predictions by list position; a list longer than the sort limit
  keeps its given order (and is then never stopped early).  Pinned by the
  defining properties of that sort on random lists with many ties.
- ``early_stop_query`` / ``early_stop_topk``: the candidates are refined in
  that order in rounds (rounds 0 and 1 take up to F more candidates, round
  r >= 2 up to F * 2^(r-1), so after r >= 1 rounds F * 2^(r-1) have been
  refined); after each round a query stops when it holds k exact results
  and its k-th best exact J is at least the next candidate's prediction
  plus a margin (in FP64, of the FP32 prediction and FP32 margin), or when
  its list is exhausted.  A query still active after the last round has
  every remaining candidate refined (the finishing pass), so the result is
  always a full top-k of Def. 1 over the refined set.  Pinned by: margin
  +inf gives the top-k of all candidates (``oracle.topk``); exact J as the
  prediction with margin 0 gives the exact top-k while refining fewer
  pairs; the number of queries the finishing pass completes in closed
  form; and hand-worked cases (``tests/golden/early_stop_cases.txt``).
"""
from __future__ import annotations

import numpy as np

__all__ = ["collision_counts", "collision_fraction", "best_first", "early_stop_query", "early_stop_topk",
           "SORT_LIMIT"]

# lists longer than this are refined in their given order without early stop
SORT_LIMIT = 8192


def collision_counts(qsig_row, dsig_rows) -> np.ndarray:
    """Per data row, the number of hashes on which it agrees with the query."""
    q = np.asarray(qsig_row, dtype=np.uint32).reshape(-1)
    d = np.asarray(dsig_rows, dtype=np.uint32).reshape(-1, q.shape[0])
    counts = np.zeros(d.shape[0], dtype=np.int64)
    for i in range(q.shape[0]):
        counts += d[:, i] == q[i]
    return counts


def collision_fraction(qsig_row, dsig_rows) -> np.ndarray:
    """Thm. 1's estimate of J: agreeing hashes over k (FP64)."""
    q = np.asarray(qsig_row).reshape(-1)
    return collision_counts(q, dsig_rows) / float(q.shape[0])


def best_first(scores, sort_limit: int = SORT_LIMIT):
    """(order, sorted): positions by (score desc, position asc), or the given
    order with sorted False when the list is longer than ``sort_limit``."""
    s = np.asarray(scores, dtype=np.float32).reshape(-1)
    n = s.shape[0]
    if n > sort_limit:
        return np.arange(n, dtype=np.int64), False
    keyed = sorted(range(n), key=lambda i: (-float(s[i]), i))
    return np.array(keyed, dtype=np.int64), True


def _top(refined, k):
    """Def. 1's order over (J, id) pairs: J descending, then id ascending."""
    return sorted(refined, key=lambda t: (-t[0], t[1]))[:k]


def early_stop_query(ids, scores, exact_j, k: int, F: int, rounds: int, margin: float,
                     sort_limit: int = SORT_LIMIT) -> dict:
    """One query.  ``ids``: its candidates' data polygon ids; ``scores``: their
    predictions (FP32); ``exact_j(positions)``: the exact J of the candidates
    at those list positions (called only for candidates refined).

    Returns top_ids / top_j (k entries, -1 / 0.0 padded), ``refined`` (pairs
    refined), ``finished`` (True when the finishing pass refined anything)
    and ``gaps``: |k-th J - (prediction + margin)| at every stop test taken,
    how far each decision was from the other outcome."""
    ids = np.asarray(ids).reshape(-1)
    order, is_sorted = best_first(scores, sort_limit)
    pred = np.asarray(scores, dtype=np.float32).reshape(-1)
    n = order.shape[0]
    m32 = float(np.float32(margin))
    refined = []
    gaps = []
    visited = 0

    def visit(count):
        nonlocal visited
        pos = order[visited:visited + count]
        if pos.size:
            js = np.asarray(exact_j(pos), dtype=np.float64).reshape(-1)
            refined.extend((float(j), int(ids[p])) for p, j in zip(pos, js))
        visited += pos.size

    active = n > 0
    for r in range(rounds):
        if not active:
            break
        visit(F if r < 2 else F * 2 ** (r - 1))
        if visited >= n:
            active = False
            break
        if is_sorted and len(refined) >= k:
            kth = _top(refined, k)[-1][0]
            bound = float(pred[order[visited]]) + m32
            gaps.append(abs(kth - bound))
            if kth >= bound:
                active = False
    finished = False
    if active and visited < n:
        visit(n - visited)
        finished = True
    top = _top(refined, k)
    top_ids = np.full(k, -1, dtype=np.int32)
    top_j = np.zeros(k, dtype=np.float64)
    for t, (j, i) in enumerate(top):
        top_ids[t] = i
        top_j[t] = j
    return {"top_ids": top_ids, "top_j": top_j, "refined": visited, "finished": finished, "gaps": gaps}


def early_stop_topk(cand_off, cand_ids, scores, exact_j, k: int, F: int, rounds: int, margin: float,
                    sort_limit: int = SORT_LIMIT, queries=None) -> dict:
    """``early_stop_query`` over a candidate CSR.  ``exact_j`` is either the
    exact J of every candidate ([C] FP64, CSR order) or a callable
    ``exact_j(q, positions)``.  ``queries`` (optional) limits the work to
    those query indices; the outputs then have one row per listed query.

    Returns top_ids [nq][k], top_j [nq][k], ``refined`` (pairs, summed),
    ``finished`` (queries the finishing pass completed) and ``min_gap`` (the
    smallest decision gap of any stop test, +inf without one)."""
    cand_off = np.asarray(cand_off, dtype=np.int64)
    cand_ids = np.asarray(cand_ids)
    scores = np.asarray(scores, dtype=np.float32)
    qs = np.arange(cand_off.shape[0] - 1) if queries is None else np.asarray(queries, dtype=np.int64)
    if callable(exact_j):
        jf = exact_j
    else:
        jall = np.asarray(exact_j, dtype=np.float64)
        jf = lambda q, pos: jall[cand_off[q] + pos]
    top_ids = np.full((qs.shape[0], k), -1, dtype=np.int32)
    top_j = np.zeros((qs.shape[0], k), dtype=np.float64)
    refined = finished = 0
    min_gap = float("inf")
    for row, q in enumerate(qs):
        a, b = int(cand_off[q]), int(cand_off[q + 1])
        r = early_stop_query(cand_ids[a:b], scores[a:b], lambda pos, q=q: jf(q, pos), k, F, rounds, margin,
                             sort_limit)
        top_ids[row], top_j[row] = r["top_ids"], r["top_j"]
        refined += r["refined"]
        finished += int(r["finished"])
        if r["gaps"]:
            min_gap = min(min_gap, min(r["gaps"]))
    return {"top_ids": top_ids, "top_j": top_j, "refined": refined, "finished": finished, "min_gap": min_gap}
