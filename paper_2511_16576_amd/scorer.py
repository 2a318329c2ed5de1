"""Learned candidate scorer: training and the ranked query path.

Every numeric step runs in libpolymh's kernels (features, MFMA forward and
backward, Adam, ordered refinement); this module sequences the calls, mines
training pairs (input preparation) and initialises the weights.

Training data (the learned-scorer workload): pairs of workload-2 polygons
signed at k = 256, half sharing at least one 32 x 8 LSH bucket and half drawn
uniformly, labelled with their exact Jaccard by the refinement kernel.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import polymh as pm

K_SCORER = 256
BATCH = 8192


@dataclasses.dataclass
class Scorer:
    params: torch.Tensor   # float32 [P] master weights
    wbf16: torch.Tensor    # int16 [W1 + W2] BF16 copy
    m: torch.Tensor
    v: torch.Tensor
    step: int = 0


def init_scorer(seed: int = 0, device="cuda") -> Scorer:
    """Uniform fan-in scaled weights (He-like for GELU), zero biases."""
    rng = np.random.default_rng(seed)
    P = pm.mlp_param_count()
    p = np.zeros(P, dtype=np.float32)
    n_in, n_hid = 288, 256
    o_w1, o_b1 = 0, n_hid * n_in
    o_w2 = o_b1 + n_hid
    o_b2 = o_w2 + n_hid * n_hid
    o_w3 = o_b2 + n_hid
    p[o_w1:o_b1] = rng.uniform(-1, 1, n_hid * n_in) * math.sqrt(6.0 / n_in)
    p[o_w2:o_b2] = rng.uniform(-1, 1, n_hid * n_hid) * math.sqrt(6.0 / n_hid)
    p[o_w3:o_w3 + n_hid] = rng.uniform(-1, 1, n_hid) * math.sqrt(1.0 / n_hid)
    params = torch.from_numpy(p).to(device)
    wbf16 = torch.empty(pm.mlp_bf16_count(), dtype=torch.int16, device=device)
    pm.mlp_sync_bf16(params, wbf16)
    z = torch.zeros_like(params)
    return Scorer(params, wbf16, z.clone(), z.clone())


def mine_pairs(sorted_keys: torch.Tensor, sorted_ent: torch.Tensor, n: int, bands: int,
               n_pairs: int, seed: int = 0):
    """(left, right) polygon ids: half from shared buckets, half uniform."""
    rng = np.random.default_rng(seed)
    sk = sorted_keys.cpu().numpy()
    se = sorted_ent.cpu().numpy() // bands
    half = n_pairs // 2
    same_next = sk[1:] == sk[:-1]
    cand = np.flatnonzero(same_next & (se[1:] != se[:-1]))   # entry i pairs with i + 1
    pick = rng.choice(cand, half, replace=cand.shape[0] < half)
    left_b, right_b = se[pick], se[pick + 1]
    left_r = rng.integers(0, n, n_pairs - half)
    right_r = rng.integers(0, n, n_pairs - half)
    keep = left_r != right_r
    left = np.concatenate([left_b, left_r[keep]]).astype(np.int32)
    right = np.concatenate([right_b, right_r[keep]]).astype(np.int32)
    perm = rng.permutation(left.shape[0])
    return left[perm], right[perm]


def mine_head_pairs(D: pm.DevicePolys, sig, sorted_keys, sorted_ent, bands: int, rows: int, band_seed: int,
                    n_pairs: int, head: int, seed: int = 0, chunk: int = 10_000):
    """(left, right) polygon ids of the pairs the ranked search scores: a
    seeded sample of data polygons, each looked up as a query in the bucket
    table (sorted_keys, sorted_ent) of `bands` x `rows` bands, gives the
    first `head` of its candidates by collision fraction, itself excluded.
    Polygons are drawn until n_pairs pairs are found."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(D.n)
    dev = sig.device
    left, right, got, at = [], [], 0, 0
    while got < n_pairs and at < D.n:
        ids = torch.from_numpy(np.sort(perm[at:at + chunk])).to(dev)
        at += chunk
        qs = sig[ids.long()].contiguous()
        off, cand = pm.query(sorted_keys, sorted_ent, D.n, pm.band(qs, bands, rows, band_seed))
        _, order, _ = pm.rank_jhat_order(qs, sig, off, cand)
        hq, _, hid = pm.rank_head_fixed(off, cand, order, head)
        lq = ids[hq.long()].to(torch.int32)
        keep = (hid >= 0) & (hid != lq)
        lq, hid = lq[keep].cpu().numpy(), hid[keep].cpu().numpy()
        left.append(lq)
        right.append(hid)
        got += lq.size
    left, right = np.concatenate(left)[:n_pairs], np.concatenate(right)[:n_pairs]
    p = rng.permutation(left.size)
    return left[p].astype(np.int32), right[p].astype(np.int32)


def exact_pair_j(D: pm.DevicePolys, left: np.ndarray, right: np.ndarray) -> torch.Tensor:
    """Exact J of (left[i], right[i]) by the refinement kernel: pairs grouped
    by left polygon as the 'query', so no polygon is copied."""
    order = np.argsort(left, kind="stable")
    lo = left[order]
    counts = np.bincount(lo, minlength=D.n)
    off = np.zeros(D.n + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    dev = D.offsets.device
    J = pm.refine(D, D, torch.from_numpy(off).to(dev), torch.from_numpy(right[order]).to(dev))
    out = torch.empty_like(J)
    out[torch.from_numpy(order).to(dev)] = J
    return out


class Trainer:
    def __init__(self, scorer: Scorer, batch: int = BATCH, lr: float = 1e-3):
        self.s = scorer
        self.batch = batch
        self.lr = lr
        dev = scorer.params.device
        self.X = torch.empty((batch, 288), dtype=torch.int16, device=dev)
        self.acts, self.scratch = pm.mlp_buffers(batch, dev)
        self.grad = torch.empty_like(scorer.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)

    def step(self, sig, feats, li, ri, label):
        """One Adam step on pairs (li, ri) of the table (sig, feats)."""
        pm.pair_features(sig, feats, sig, feats, li, ri, R_pad=self.batch, out=self.X)
        pm.mlp_forward(self.X, self.s.params, self.s.wbf16, self.acts)
        lab = torch.zeros(self.batch, dtype=torch.float32, device=label.device)
        lab[:label.numel()] = label
        pm.mlp_backward(self.X, self.s.params, self.s.wbf16, self.acts, lab, self.grad, self.loss,
                        self.scratch)
        self.s.step += 1
        pm.mlp_adam(self.s.params, self.grad, self.s.m, self.s.v, self.s.step, self.s.wbf16, lr=self.lr)
        return self.loss


def train(scorer: Scorer, sig, feats, left, right, label, epochs: int = 3, batch: int = BATCH,
          lr: float = 1e-3, seed: int = 0, log=None):
    """Mini-batch Adam over the pair set; batches are whole (the remainder of
    an epoch is dropped)."""
    tr = Trainer(scorer, batch, lr)
    n = left.shape[0]
    rng = np.random.default_rng(seed)
    dev = sig.device
    L = torch.from_numpy(left).to(dev)
    R = torch.from_numpy(right).to(dev)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        tot, cnt = 0.0, 0
        t0 = time.perf_counter()
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            loss = tr.step(sig, feats, L[idx].contiguous(), R[idx].contiguous(), label[idx].contiguous())
            if (b0 // batch) % 16 == 0:
                tot += float(loss.item())
                cnt += 1
        torch.cuda.synchronize()
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.5f} ({time.perf_counter() - t0:.2f} s)")
    return hist


def predict_pairs(scorer: Scorer, lsig, lfeat, rsig, rfeat, li, ri, chunk: int = 1 << 18):
    """Predicted J of every (li, ri) pair, in chunks of `chunk` rows."""
    R = li.numel()
    dev = lsig.device
    R32 = max(((R + 31) // 32) * 32, 32)
    out = torch.empty(R32, dtype=torch.float32, device=dev)   # padded: chunks write whole tiles
    rows = min(chunk, R32)
    X = torch.empty((rows, 288), dtype=torch.int16, device=dev)
    acts, _ = pm.mlp_buffers(rows, dev)
    for c0 in range(0, R, rows):
        c1 = min(R, c0 + rows)
        pad = ((c1 - c0 + 31) // 32) * 32
        pm.pair_features(lsig, lfeat, rsig, rfeat, li[c0:c1], ri[c0:c1], R_pad=pad, out=X)
        pm.mlp_forward(X[:pad], scorer.params, scorer.wbf16, acts, y=out[c0:c0 + pad])
    return out[:R]


HEAD = 64


def candidate_scores(kind: str, scorer, qsig, qfeat, dsig, dfeat, cand_off, cand_ids, head: int = HEAD):
    """Per-candidate predicted J.  'jhat': the collision fraction of the
    signatures (Thm. 1's estimate).  'mlp': a cascade -- the collision
    fraction orders every candidate, then the scorer re-predicts the first
    `head` candidates of each query (one fused launch writes into their
    scores)."""
    C = cand_ids.numel()
    score, order, _ = pm.rank_jhat_order(qsig, dsig, cand_off, cand_ids)
    if kind == "jhat":
        return score[:C]
    hq, hc, hid = pm.rank_head_fixed(cand_off, cand_ids, order, head)
    pm.mlp_score_pairs(qsig, qfeat, dsig, dfeat, hq, hid, scorer.params, scorer.wbf16, out=score, out_idx=hc)
    return score[:C]


# ------------------------------------------------------------ measurement --

def brute_force_top10(D: pm.DevicePolys, Q: pm.DevicePolys):
    """Exact top-10 of every query against the whole dataset (all pairs
    refined by the refinement kernel)."""
    dev = D.offsets.device
    off = torch.arange(Q.n + 1, device=dev, dtype=torch.int64) * D.n
    ids = torch.arange(D.n, device=dev, dtype=torch.int32).repeat(Q.n)
    J = pm.refine(D, Q, off, ids)
    return pm.topk(off, ids, J, 10)


def _prefix(off, ids, n):
    """CSR of the first n queries."""
    o = off[:n + 1]
    return o, ids[:int(o[-1].item())]


def learned_comparison(w, D, Q, log, n_pairs=2_000_000, epochs=3, bands=64, rows=4, n_calib=1000,
                       n_eval=1000, reps=3, F=16, target=0.95, sig=None, brute=None):
    """Plain full refinement vs best-first refinement with early stop ordered
    by the collision fraction or by the trained scorer: the learned-scorer
    workload (workload-2 polygons signed at k = 256), or another one given
    its dataset signatures at k = 256 (``sig``) and a brute-force top-10
    (``brute(D, Q) -> (ids, J)``; default: every pair refined).  The early
    stop is calibrated to recall@10 >= ``target`` on the calibration
    queries."""
    from .metrics import recall_at_k
    k, cap = K_SCORER, w.cap
    dev = D.offsets.device
    brute = brute_force_top10 if brute is None else brute
    out = {"k": k, "bands": bands, "rows": rows, "train_pairs": n_pairs, "epochs": epochs}
    t0 = time.perf_counter()
    if sig is None:
        sig = pm.sign(D, w.box, w.seed, k, cap)
    elif sig.shape[1] != k:
        raise ValueError(f"learned_comparison: signatures of {k} hashes expected")
    feats = pm.poly_features(D, w.box)
    keys8 = pm.band(sig, 32, 8, w.seed)
    sk8, se8 = pm.index_build(keys8)
    left, right = mine_pairs(sk8, se8, D.n, 32, n_pairs, seed=1)
    J = exact_pair_j(D, left, right).float()
    torch.cuda.synchronize()
    out["label_s"] = time.perf_counter() - t0
    n_val = max(len(left) // 50, 1024)
    s = init_scorer(0)
    t0 = time.perf_counter()
    hist = train(s, sig, feats, left[n_val:], right[n_val:], J[n_val:], epochs=epochs, log=log)
    out["train_s"] = time.perf_counter() - t0
    out["train_loss"] = hist
    Lv, Rv = torch.from_numpy(left[:n_val]).to(dev), torch.from_numpy(right[:n_val]).to(dev)
    pv = predict_pairs(s, sig, feats, sig, feats, Lv, Rv)
    jv = pm.jhat(sig, sig, Lv, Rv)
    out["val_mse_scorer"] = float(((pv - J[:n_val]) ** 2).mean())
    out["val_mse_collision_fraction"] = float(((jv - J[:n_val]) ** 2).mean())
    log(f"held-out MSE: scorer {out['val_mse_scorer']:.5f}, collision fraction {out['val_mse_collision_fraction']:.5f}")

    keys = pm.band(sig, bands, rows, w.seed)
    sk, se = pm.index_build(keys)
    qfeats = pm.poly_features(Q, w.box)

    def candidates(Qp):
        qs = pm.sign(Qp, w.box, w.seed, k, cap)
        qk = pm.band(qs, bands, rows, w.seed)
        off, ids = pm.query(sk, se, D.n, qk)
        return qs, off, ids

    def run(method, Qp, qf, margin, timed=False):
        qs, off, ids = candidates(Qp)
        if method == "plain":
            Jc = pm.refine(D, Qp, off, ids)
            ti, tj = pm.topk(off, ids, Jc, 10)
            return ti, tj, ids.numel()
        score = candidate_scores("mlp" if method == "scorer" else "jhat", s, qs, qf, sig, feats, off, ids)
        ti, tj, nref, _ = pm.rank_refine(D, Qp, off, ids, score, topk=10, F=F, margin=margin)
        return ti, tj, nref

    # calibration and evaluation query samples, with brute-force answers
    import numpy as np_
    cal = pm.to_device(w.queries.subset(np_.arange(n_calib)))
    ev = pm.to_device(w.queries.subset(np_.arange(n_calib, n_calib + n_eval)))
    cal_f, ev_f = qfeats[:n_calib].contiguous(), qfeats[n_calib:n_calib + n_eval].contiguous()
    bci, bcj = brute(D, cal)
    bei, bej = brute(D, ev)
    bci, bcj, bei, bej = (x.cpu().numpy() if torch.is_tensor(x) else x for x in (bci, bcj, bei, bej))
    grid = [0.0, 0.005, 0.01, 0.015, 0.02, 0.025, 0.03, 0.04, 0.05, 0.06, 0.08, 0.1, 0.15, 0.2, 0.3, 0.5]
    res = {}
    for method in ("plain", "collision_fraction", "scorer"):
        margin = float("inf")
        if method != "plain":
            for m in grid:
                ti, tj, _ = run(method, cal, cal_f, m)
                # calibrate with a small safety margin over the target
                if recall_at_k(ti.cpu().numpy(), tj.cpu().numpy(), bci, bcj, 10) >= target + 0.005:
                    margin = m
                    break
        ti, tj, nref = run(method, ev, ev_f, margin)
        rec = recall_at_k(ti.cpu().numpy(), tj.cpu().numpy(), bei, bej, 10)
        # throughput over all queries
        run(method, Q, qfeats, margin)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            _, _, nref_all = run(method, Q, qfeats, margin)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        res[method] = {"margin": margin, "recall_at_10": rec, "queries_per_s": Q.n / dt,
                       "ms_per_batch": 1e3 * dt, "refined_pairs_per_query": nref_all / Q.n}
        log(f"{method}: margin {margin}, recall@10 {rec:.3f}, {Q.n / dt:.0f} q/s, "
            f"{nref_all / Q.n:.1f} refined pairs/query")
    out["methods"] = res
    return out
