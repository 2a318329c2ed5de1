"""Search-quality measures (Sec. 5.2): recall@k against a brute-force answer."""
from __future__ import annotations

import numpy as np


def recall_at_k(ann_ids, ann_j, bf_ids, bf_j, k: int, tie_eps: float = 1e-12) -> float:
    """Mean over queries of |ANN_k n BF_k| / |BF_k|, where an ANN answer whose
    exact J ties the brute-force k-th value also counts."""
    ann_ids, ann_j = np.asarray(ann_ids), np.asarray(ann_j)
    bf_ids, bf_j = np.asarray(bf_ids), np.asarray(bf_j)
    nq = ann_ids.shape[0]
    if nq == 0:
        return 1.0
    total = 0.0
    for q in range(nq):
        truth = bf_ids[q, :k]
        truth = truth[truth >= 0]
        if truth.size == 0:
            total += 1.0
            continue
        kth = bf_j[q, truth.size - 1]
        a, aj = ann_ids[q, :k], ann_j[q, :k]
        ok = (a >= 0) & (np.isin(a, truth) | (aj >= kth - tie_eps))
        total += min(int(ok.sum()), truth.size) / truth.size
    return total / nq


def brute_force_topk_mbr(D, Q, k: int, chunk: int = 16):
    """Def. 1 by brute force on the device for sets too large to refine every
    pair: exact J (the refinement kernel) of each query against every dataset
    polygon whose MBR meets the query's, since a pair with disjoint MBRs has
    J = 0; those rank after every positive J (ties by id), which the tie rule
    of ``recall_at_k`` counts as equal.  Returns (ids int32 [nq, k], J [nq, k])
    as numpy arrays."""
    import torch
    from . import polymh as pm
    dm, _, _ = pm.prepare(D)
    qm, _, _ = pm.prepare(Q)
    ids_out = np.full((Q.n, k), -1, dtype=np.int32)
    j_out = np.zeros((Q.n, k))
    for a in range(0, Q.n, chunk):
        b = min(Q.n, a + chunk)
        q = qm[a:b]
        hit = ((dm[None, :, 0] <= q[:, None, 2]) & (dm[None, :, 2] >= q[:, None, 0]) &
               (dm[None, :, 1] <= q[:, None, 3]) & (dm[None, :, 3] >= q[:, None, 1]))
        cnt = hit.sum(dim=1)
        off = torch.zeros(b - a + 1, dtype=torch.int64, device=dm.device)
        off[1:] = torch.cumsum(cnt, 0)
        ids = torch.nonzero(hit, as_tuple=False)[:, 1].to(torch.int32).contiguous()
        Qs = pm.DevicePolys(*_slice_polys(Q, a, b))
        if ids.numel():
            J = pm.refine(D, Qs, off, ids)
            ti, tj = pm.topk(off, ids, J, k)
            ti, tj = ti.cpu().numpy(), tj.cpu().numpy()
            ti[tj <= 0.0] = -1                  # J = 0 ranks by id over the whole set
            ids_out[a:b], j_out[a:b] = ti, np.maximum(tj, 0.0)
        # fewer than k positive: the smallest ids not listed, J = 0, as the
        # all-pairs ranking (J desc, id asc) would give
        for q_ in range(a, b):
            row = ids_out[q_]
            free = np.flatnonzero(row < 0)
            if free.size:
                taken = set(int(x) for x in row if x >= 0)
                fill = [i for i in range(min(D.n, k + len(taken))) if i not in taken][:free.size]
                row[free[:len(fill)]] = fill          # fewer than k polygons: -1 pads the rest
                j_out[q_, free] = 0.0
    return ids_out, j_out


def _slice_polys(P, a: int, b: int):
    off = P.offsets[a:b + 1]
    lo, hi = int(off[0].item()), int(off[-1].item())
    return P.xy[lo:max(hi, lo + 1)].contiguous(), (off - lo).contiguous()
