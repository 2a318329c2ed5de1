"""Table 2's experiment (Sec. 5.2-5.3) on synthetic stand-ins of Table 1's
datasets, on the GPU path.

The paper's index is one hashmap keyed by a polygon's whole m-long MinHash
code (Sec. 5.2.1, MinHash length m = 1..5); a query's candidates are the
polygons in its bucket.  That is banding with one band of m rows, and the
"2 hashmaps" system of Sec. 5.3 is two independent such tables OR-ed (two
bands of m rows, 2m hashes).  Following Sec. 3.1, every polygon (dataset
and query) is centred first and B is the lattice box of the centred
dataset; the queries are signed in that B.

Per configuration the run reports, like Table 2: recall@10/50/100 against
brute force (exact J of a query against every dataset polygon, the same
refinement kernel), MinHashing time (signing dataset and queries),
hashmap lookup + refinement time (band keys, bucket table, candidates,
exact J, top-100), brute-force time, the speedup BF / total, and pruning
(100 (1 - candidates / N), averaged over queries).  Brute force runs on a
seeded query sample and its time is scaled to all queries; recall is
measured on that sample.  When ``--queries`` is below the table's query
count, PolyMinHash times are scaled the same way.

Run: ``python -m paper_2511_16576_amd.table2 --dataset cemetery [--m 1 2 3]
[--tables 1 2] [--bf-queries B] [--queries Q] [--n N] [--json out.json]``
(``--dataset all`` runs the four).  Defaults per dataset: Table 2's m
values, and for Parks (319 vertices on average, about 0.9 us per exact J
once centred) and Sports (20,000 queries) a timed query subset of 300 and
2,000 queries with brute force on 50 and 100 of them."""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import datagen as dg
from . import metrics
from . import polymh as pm

KS = (10, 50, 100)
# Table 2's MinHash lengths per dataset; query subset and brute-force sample
PAPER_M = {"urban": (1, 2, 3), "cemetery": (1, 3, 5), "parks": (1, 2, 3), "sports": (1, 3)}
QUERIES = {"urban": None, "cemetery": None, "parks": 300, "sports": 2000}
BF_QUERIES = {"urban": 200, "cemetery": 200, "parks": 50, "sports": 100}
# queries per lookup batch (bounded by candidate memory and by progress lines)
BATCH = {"urban": 1000, "cemetery": 1000, "parks": 100, "sports": 250}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _slice(P: pm.DevicePolys, a: int, b: int) -> pm.DevicePolys:
    off = P.offsets[a:b + 1]
    lo, hi = int(off[0].item()), int(off[-1].item())
    return pm.DevicePolys(P.xy[lo:max(hi, lo + 1)].contiguous(), (off - lo).contiguous())


class _Timer:
    """Milliseconds of GPU work between start and stop on the current stream."""

    def __init__(self):
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def start(self):
        self.e0.record()

    def stop(self) -> float:
        self.e1.record()
        self.e1.synchronize()
        return self.e0.elapsed_time(self.e1)


def brute_force(D: pm.DevicePolys, Q: pm.DevicePolys, kmax: int, chunk_pairs: int = 1 << 25, log=None):
    """Exact top-kmax of every query of Q against all of D: (ids, J, ms)."""
    n, nq = D.n, Q.n
    per = max(1, chunk_pairs // max(n, 1))
    ids_all = torch.arange(n, dtype=torch.int32, device="cuda")
    top_i, top_j, ms = [], [], 0.0
    t = _Timer()
    for a in range(0, nq, per):
        b = min(nq, a + per)
        Qs = _slice(Q, a, b)
        off = torch.arange(b - a + 1, dtype=torch.int64, device="cuda") * n
        ids = ids_all.repeat(b - a)
        t.start()
        J = pm.refine(D, Qs, off, ids)
        ti, tj = pm.topk(off, ids, J, kmax)
        ms += t.stop()
        top_i.append(ti.cpu().numpy())
        top_j.append(tj.cpu().numpy())
        del J, ids
        if log is not None and nq > per:
            log(f"  brute force: queries {a}-{b} of {nq}, {ms:.0f} ms")
    return np.concatenate(top_i), np.concatenate(top_j), ms


def run_config(D, Q, box, seed, m, tables, cap, sample, bf_i, bf_j, batch=100):
    """One (m, tables) configuration over all of Q's queries.  Times in ms,
    dataset-side (once) and query-side (proportional to the query count)."""
    k = m * tables
    t = _Timer()
    t.start()
    sd = pm.sign(D, box, seed, k, cap)
    ms_sign_d = t.stop()
    t.start()
    sq = pm.sign(Q, box, seed, k, cap)
    ms_sign_q = t.stop()
    t.start()
    kd = pm.band(sd, tables, m, seed)
    sk, si = pm.index_build(kd)
    ms_index = t.stop()
    t.start()
    kq = pm.band(sq, tables, m, seed)
    ms_lookup = t.stop()
    cand_total = 0
    in_sample = np.zeros(Q.n, dtype=bool)
    in_sample[sample] = True
    ann_i = np.full((Q.n, max(KS)), -1, dtype=np.int32)
    ann_j = np.zeros((Q.n, max(KS)))
    for a in range(0, Q.n, batch):
        b = min(Q.n, a + batch)
        Qs = _slice(Q, a, b)
        t.start()
        off, ids = pm.query(sk, si, D.n, kq[a:b].contiguous())
        J = pm.refine(D, Qs, off, ids)
        ti, tj = pm.topk(off, ids, J, max(KS))
        ms_lookup += t.stop()
        cand_total += int(off[-1].item())
        if Q.n > batch:
            log(f"  m={m} tables={tables}: queries {a}-{b}, {int(off[-1].item())} candidates, {ms_lookup:.0f} ms")
        sel = np.flatnonzero(in_sample[a:b])
        if sel.size:
            ann_i[a + sel] = ti.cpu().numpy()[sel]
            ann_j[a + sel] = tj.cpu().numpy()[sel]
        del off, ids, J
    rec = {f"recall@{kk}": metrics.recall_at_k(ann_i[sample], ann_j[sample], bf_i, bf_j, kk) for kk in KS}
    return {"m": m, "tables": tables, "k": k, **rec, "sign_data_ms": ms_sign_d, "sign_queries_ms": ms_sign_q,
            "index_ms": ms_index, "lookup_refine_queries_ms": ms_lookup,
            "candidates_per_query": cand_total / Q.n, "pruning_pct": 100.0 * (1.0 - cand_total / (Q.n * D.n))}


def run_dataset(name, ms=None, tables=(1, 2), bf_queries=None, n=None, n_queries=None,
                cap=1 << 22, batch=None, seed=0):
    ms = PAPER_M[name] if ms is None else ms
    batch = BATCH[name] if batch is None else batch
    bf_queries = BF_QUERIES[name] if bf_queries is None else bf_queries
    n_queries = QUERIES[name] if n_queries is None else n_queries
    t0 = time.time()
    w = dg.table1_standin(name, n=n, n_queries=n_queries)
    q_full = dg.TABLE1[name][1]
    log(f"{name}: {w.data.n} polygons ({w.data.counts().mean():.2f} vertices on average), "
        f"{w.queries.n} queries, generated in {time.time() - t0:.1f}s")
    D0, Q0 = pm.to_device(w.data), pm.to_device(w.queries)
    # Sec. 3.1: centre dataset and queries; B = box of the centred dataset
    D, _ = pm.centre(D0)
    Q, _ = pm.centre(Q0)
    del D0, Q0
    box = pm.box_of(D)
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(Q.n, min(bf_queries, Q.n), replace=False))
    Qb = pm.DevicePolys(*_gather(Q, sample))
    bf_i, bf_j, bf_ms = brute_force(D, Qb, max(KS), log=log)
    scale_q = q_full / Q.n
    bf_total_s = bf_ms / 1e3 * q_full / sample.size
    log(f"{name}: brute force {bf_ms:.0f} ms for {sample.size} queries -> {bf_total_s:.1f} s for {q_full}")
    rows = []
    for tb in tables:
        for m in ms:
            r = run_config(D, Q, box, seed, m, tb, cap, sample, bf_i, bf_j, batch)
            minhash_s = (r["sign_data_ms"] + r["sign_queries_ms"] * scale_q) / 1e3
            lookup_s = (r["index_ms"] + r["lookup_refine_queries_ms"] * scale_q) / 1e3
            total_s = minhash_s + lookup_s
            r.update({"dataset": name, "minhash_s": minhash_s, "lookup_refine_s": lookup_s, "total_s": total_s,
                      "bf_s": bf_total_s, "speedup": bf_total_s / total_s})
            rows.append(r)
            log(f"{name} tables={tb} m={m}: recall@10/50/100 {r['recall@10']:.2f}/{r['recall@50']:.2f}/"
                f"{r['recall@100']:.2f}, minhash {r['minhash_s']:.3f} s, lookup+refine "
                f"{r['lookup_refine_s']:.3f} s, BF {bf_total_s:.1f} s, speedup {r['speedup']:.1f}, "
                f"pruning {r['pruning_pct']:.1f}%")
    meta = {"dataset": name, "n": D.n, "queries": Q.n, "table_queries": q_full, "bf_sample": int(sample.size),
            "mean_vertices": float(w.data.counts().mean()), "box": list(box), "cap": cap}
    return meta, rows


def _gather(P: pm.DevicePolys, ids: np.ndarray):
    """(xy, offsets) of the polygons ``ids`` of P, on the device."""
    off = P.offsets.cpu().numpy()
    cnt = off[ids + 1] - off[ids]
    new_off = np.zeros(ids.size + 1, dtype=np.int64)
    np.cumsum(cnt, out=new_off[1:])
    src = np.repeat(off[ids], cnt) + (np.arange(new_off[-1]) - np.repeat(new_off[:-1], cnt))
    idx = torch.from_numpy(src).to(P.xy.device)
    return P.xy[idx].contiguous(), torch.from_numpy(new_off).to(P.xy.device)


def table_markdown(results) -> str:
    lines = ["| dataset | tables | m | R@10 | R@50 | R@100 | MinHashing s | lookup+refine s | total s | BF s | "
             "speedup | pruning % |", "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for meta, rows in results:
        for r in rows:
            lines.append(f"| {meta['dataset']} | {r['tables']} | {r['m']} | {r['recall@10']:.2f} | "
                         f"{r['recall@50']:.2f} | {r['recall@100']:.2f} | {r['minhash_s']:.3f} | "
                         f"{r['lookup_refine_s']:.3f} | {r['total_s']:.3f} | {r['bf_s']:.2f} | "
                         f"{r['speedup']:.1f} | {r['pruning_pct']:.1f} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dataset", default="cemetery", choices=list(dg.TABLE1) + ["all"])
    ap.add_argument("--m", type=int, nargs="+", default=None)
    ap.add_argument("--tables", type=int, nargs="+", default=[1, 2])
    ap.add_argument("--bf-queries", type=int, default=None)
    ap.add_argument("--queries", type=int, default=None)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    pm.check_device()
    names = list(dg.TABLE1) if a.dataset == "all" else [a.dataset]
    results = [run_dataset(nm, ms=a.m, tables=a.tables, bf_queries=a.bf_queries, n=a.n, n_queries=a.queries,
                           batch=a.batch) for nm in names]
    md = table_markdown(results)
    print(md, flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump([{"meta": m_, "rows": r_} for m_, r_ in results], f, indent=1)


if __name__ == "__main__":
    main()
