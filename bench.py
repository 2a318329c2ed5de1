"""Benchmark of the PolyMinHash signing and search path on one MI355X.

One step = the whole path over one batch, inputs resident in HBM:
  sign the 100,000-polygon workload (k=128, cap 2^22, persistent launch),
  band it, build the bucket table, then answer 10,000 queries (sign, band,
  candidate lookup, exact-Jaccard refinement, top-10).
value = signatures produced per second of step time ((N + Q) * k / step).
The line also carries per-stage times (HIP events), the signing kernel's
roofline figures and the CPU oracle's rate on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "polygon-hash signatures/s; queries/s at recall@10≥0.95, learned vs plain"
PEAK_VALU = 256 * 4 * 16 * 2.4e9      # lane-cycles/s: 256 CUs x 4 SIMD16 x 2.4 GHz
# VALU issue cycles per lane, counted in the built gfx950 code of the signing
# kernel: one draw (SplitMix64 with two 64x64-bit products, lattice map, MBR
# check: 26 full-rate + 6 quarter-rate instructions) and one edge test of the
# point-in-polygon loop.
C_DRAW = 26 + 6 * 4
C_EDGE = 14


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=10_000)
    ap.add_argument("--bands", type=int, default=32)
    ap.add_argument("--rows", type=int, default=4)
    ap.add_argument("--recall-sample", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the signing path has no multi-GPU form in this "
              "build (see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2511_16576_amd import datagen as dg
    from paper_2511_16576_amd import polymh as pm

    torch.cuda.set_device(0)
    pm.check_device()
    t0 = time.time()
    w = dg.workload(2, n_queries=args.queries)
    log(f"workload 2 generated in {time.time() - t0:.1f}s: {w.data.n} polygons, "
        f"{w.data.xy.shape[0]} vertices, {w.queries.n} queries")
    D, Q = pm.to_device(w.data), pm.to_device(w.queries)
    k, cap, b, r = w.k, w.cap, args.bands, args.rows
    cfg = pm.default_sign_config()
    dev = D.offsets.device
    ws_d = torch.empty(pm.sign_workspace_size(D.n, cfg), dtype=torch.uint8, device=dev)
    ws_q = torch.empty(pm.sign_workspace_size(Q.n, cfg), dtype=torch.uint8, device=dev)
    sig = torch.empty((D.n, k), dtype=torch.int32, device=dev)
    qsig = torch.empty((Q.n, k), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    names = ["sign", "band+index", "qsign+qband", "query", "refine", "topk"]

    def step(times=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] if times is not None else None
        if ev: ev[0].record(stream)
        pm.sign(D, w.box, w.seed, k, cap, config=cfg, out=sig, ws=ws_d)
        if ev: ev[1].record(stream)
        keys = pm.band(sig, b, r, w.seed)
        sk, si = pm.index_build(keys)
        if ev: ev[2].record(stream)
        pm.sign(Q, w.box, w.seed, k, cap, config=cfg, out=qsig, ws=ws_q)
        qkeys = pm.band(qsig, b, r, w.seed)
        if ev: ev[3].record(stream)
        off, ids = pm.query(sk, si, D.n, qkeys)
        if ev: ev[4].record(stream)
        J = pm.refine(D, Q, off, ids)
        if ev: ev[5].record(stream)
        ti, tj = pm.topk(off, ids, J, 10)
        if ev: ev[6].record(stream)
        if times is not None:
            torch.cuda.synchronize()
            for i, nmk in enumerate(names):
                times.setdefault(nmk, []).append(ev[i].elapsed_time(ev[i + 1]))
        return off, ids, ti, tj

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms = 1e3 * elapsed / args.steps
    log(f"timed {args.steps} steps: {ms:.2f} ms/step")

    # per-stage breakdown from a separate instrumented pass
    times = {}
    for _ in range(2):
        out = step(times)
    stage_ms = {k_: float(np.median(v)) for k_, v in times.items()}
    off, ids, ti, tj = out
    n_cand = int(ids.numel())

    # realised draws (sum of signature values = Alg. 1's attempts) and the
    # expected point-in-polygon edge tests, for the signing roofline
    s_np = sig.cpu().numpy().view(np.uint32).astype(np.float64)
    draws = float(s_np.sum()) + float((s_np == 0).sum()) * cap
    mbr, area2, flags = pm.prepare(D)
    mbr = mbr.cpu().numpy().astype(np.float64)
    a_mbr = (mbr[:, 2] - mbr[:, 0] + 1) * (mbr[:, 3] - mbr[:, 1] + 1)
    a_p = np.maximum(np.abs(area2.cpu().numpy().astype(np.float64)) / 2, 0.5)
    nverts = np.diff(w.data.offsets).astype(np.float64)
    edges = float((k * nverts * np.minimum(a_mbr / a_p, s_np.mean(axis=1))).sum())
    sign_ops = draws * C_DRAW + edges * C_EDGE
    t_sign = stage_ms["sign"] / 1e3
    achieved = sign_ops / t_sign

    # recall@10 on a query sample against GPU brute force (all pairs refined)
    rs = min(args.recall_sample, Q.n)
    rec = None
    if rs > 0:
        import oracle  # noqa: F401  (recall helper only; the brute force runs on the GPU)
        qs = np.arange(rs)
        Qs = pm.to_device(w.queries.subset(qs))
        bf_off = torch.arange(rs + 1, device=dev, dtype=torch.int64) * D.n
        bf_ids = torch.arange(D.n, device=dev, dtype=torch.int32).repeat(rs)
        bfJ = pm.refine(D, Qs, bf_off, bf_ids)
        bi, bj = pm.topk(bf_off, bf_ids, bfJ, 10)
        rec = oracle.recall_at_k(ti[:rs].cpu().numpy(), tj[:rs].cpu().numpy(), bi.cpu().numpy(),
                                 bj.cpu().numpy(), 10)
        log(f"recall@10 over {rs} queries: {rec:.3f}")

    cpu = None
    if not args.no_cpu:
        import oracle
        th = oracle.max_threads()
        ids_s = np.arange(min(D.n, 100_000))
        t2 = time.perf_counter()
        oracle.sign(w.data.subset(ids_s), w.box, w.seed, k, cap, threads=th)
        tc = time.perf_counter() - t2
        cpu = {"value": ids_s.size * k / tc, "unit": "signatures/s", "cores": th, "kind": "oracle",
               "sample": f"oracle Alg. 1 signing of {ids_s.size} workload-2 polygons x {k} hashes "
                         f"({tc:.1f} s, OpenMP over polygons)"}
        log(f"cpu oracle: {cpu['value']:.3g} sig/s on {th} threads")

    total_sigs = (D.n + Q.n) * k
    line = {
        "metric": METRIC,
        "value": total_sigs / (ms / 1e3),
        "unit": "signatures/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "workload 2: 100,000 star polygons, lognormal 8-512 vertices, "
                               "R 2-15% of a 2^24 grid; k=128, cap 2^22; 10,000 queries (2% jitter)",
                   "n_data": D.n, "n_queries": Q.n, "k": k, "bands": b, "rows": r,
                   "sign_config": cfg.as_dict()},
        "sign_sig_per_s": D.n * k / t_sign,
        "queries_per_s": Q.n / (sum(stage_ms[s] for s in names[2:]) / 1e3),
        "candidates_per_query": n_cand / Q.n,
        "recall_at_10": rec,
        "stage_ms": stage_ms,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12,
                     "unit": "T lane-cycles/s", "frac": achieved / PEAK_VALU, "traffic": None,
                     "kernel": "k_sign", "draws_per_launch": draws, "edge_tests_per_launch": edges},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
