"""Launch-shape autotuner for the signing kernel.

Times every candidate configuration (persistent or plain launch, workgroup
size, hashes per work item, LDS edge capacity, samples per lane, blocks per
CU) on a seeded sample of the workload with HIP events, checks that each
produces the same signatures as the default shape, and caches the fastest
per workload fingerprint in a JSON file (POLYMH_TUNE_CACHE, default
~/.cache/polymh/sign_tune.json)."""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import torch

from . import polymh as pm

DEFAULT_SPACE = {
    "persistent": [1, 0],
    "block_threads": [64, 128, 256],
    "hash_block": [0, 32],
    "lds_edges": [256, 512, 1024],
    "samples_per_lane": [1, 2],
    "blocks_per_cu": [8, 16],
}


def _cache_path():
    return os.environ.get("POLYMH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "polymh", "sign_tune.json"))


def fingerprint(polys, box, k, cap) -> str:
    counts = np.diff(polys.offsets)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return (f"{arch}|n={polys.n}|v={int(counts.sum())}|vmax={int(counts.max()) if counts.size else 0}"
            f"|box={tuple(int(b) for b in box)}|k={k}|cap={cap}")


def _time(D, box, seed, k, cap, cfg, out, ws, reps):
    s = torch.cuda.current_stream()
    pm.sign(D, box, seed, k, cap, config=cfg, out=out, ws=ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        pm.sign(D, box, seed, k, cap, config=cfg, out=out, ws=ws)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_sign(polys, box, seed: int, k: int, cap: int, sample: int = 20000, reps: int = 3,
              space=None, use_cache: bool = True, log=None):
    """Best signing launch shape for this workload; returns (config, report)."""
    key = fingerprint(polys, box, k, cap)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return pm.sign_config(**cache[key]["config"]), cache[key]
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(polys.n, min(sample, polys.n), replace=False))
    sub = polys.subset(ids)
    D = pm.to_device(sub)
    space = space or DEFAULT_SPACE
    names = list(space)
    ref = pm.sign(D, box, seed, k, cap).clone()
    best, results = None, []
    ws = None
    for values in itertools.product(*(space[n] for n in names)):
        cfg_d = dict(zip(names, values))
        if not cfg_d["persistent"] and cfg_d["blocks_per_cu"] != space["blocks_per_cu"][0]:
            continue   # blocks_per_cu only shapes the persistent grid
        cfg = pm.sign_config(**cfg_d)
        need = pm.sign_workspace_size(D.n, cfg)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=D.offsets.device)
        out = torch.empty_like(ref)
        ms = _time(D, box, seed, k, cap, cfg, out, ws, reps)
        same = bool(torch.equal(out, ref))
        results.append({"config": cfg_d, "ms": ms, "bits_equal": same})
        if not same:
            raise RuntimeError(f"launch shape {cfg_d} changed the signatures")
        if best is None or ms < best["ms"]:
            best = {"config": cfg_d, "ms": ms}
        if log:
            log(f"tune {cfg_d}: {ms:.3f} ms")
    report = {"config": best["config"], "ms": best["ms"], "sample": int(ids.size),
              "default_ms": next(r["ms"] for r in results
                                 if r["config"] == {n: getattr(pm.default_sign_config(), n) for n in names}
                                 ) if any(r["config"] == {n: getattr(pm.default_sign_config(), n) for n in names}
                                         for r in results) else None,
              "tried": len(results)}
    if use_cache:
        cache[key] = report
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return pm.sign_config(**best["config"]), report
