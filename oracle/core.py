"""PolyMinHash CPU oracle (test infrastructure only): Python side.

Wraps the plain C oracle (``polymh_oracle.c``, built with gcc and OpenMP)
and adds what is clearest in Python: an exact rational version of the
intersection area, top-k, brute-force nearest neighbours and recall.

What each function follows in the paper, and what pins it (tests under
``tests/test_oracle_*.py``):

- ``mix64`` / ``splitmix64``: SplitMix64 (Steele, Lea, Flood 2014), the
  reading of Alg. 1's fixed-seed generators.  Pinned by the published
  SplitMix64 test vector for seed 0 and by an independent modular inverse.
- ``sample_point``: uniform sampling over the global MBR (Sec. 3.2,
  Alg. 1).  Pinned by the closed form for power-of-two widths and by
  big-integer floor division for other widths.
- ``inside``: Alg. 1's point-in-polygon test (half-open crossing rule).
  Pinned by exact cell counts of rectangles and rectilinear polygons, Pick's
  theorem bounds, and an independent winding-number test off the boundary.
- ``sign``: Alg. 1 / Def. 2.  Pinned by Thm. 2 (geometric law) and Thm. 1
  (collision rate = Jaccard) on rectangles with closed-form overlap, the
  first-hit index against a known cell set, the union law
  h(A u B) = min(h(A), h(B)), the 1-based count of Fig. 2, cap semantics,
  the prefix property and translation invariance.
- ``band`` / ``candidates``: the hashmap-of-codes filter of Sec. 3.2
  (banded).  Pinned by locality (a row change moves exactly its band's key)
  and by the candidate definition on hand-built keys.
- ``intersection_area`` / ``jaccard``: Sec. 1's Jaccard of areas.  Pinned by
  closed forms (rectangle overlap, identical, disjoint, nested, shoelace),
  by scipy's half-space intersection for convex pairs, and by the exact
  rational version.
- ``topk`` / ``brute_force_topk`` / ``recall_at_k``: Def. 1 and Sec. 5.2.
  Pinned by brute force on tiny sets.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polymh_oracle.c")
_LIB = os.path.join(_HERE, "libpolymh_oracle.so")
GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32, u64, f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        sig = {
            "orc_mix64": (u64, [u64]),
            "orc_splitmix64": (None, [u64, i64, P]),
            "orc_hash_keys": (None, [u64, i32, P]),
            "orc_sample_point": (None, [P, u64, u64, P]),
            "orc_inside": (ctypes.c_int, [P, i64, i32, i32]),
            "orc_inside_points": (None, [P, i64, P, i64, P]),
            "orc_sign": (i32, [P, P, i64, P, u64, i32, u32, i32, i32, P]),
            "orc_band": (None, [P, i64, i32, i32, i32, u64, P]),
            "orc_candidates": (i64, [P, i64, P, i64, i32, P, P, i64]),
            "orc_area2": (i64, [P, i64]),
            "orc_intersection_area": (f64, [P, i64, P, i64]),
            "orc_jaccard": (f64, [P, i64, P, i64]),
            "orc_jaccard_candidates": (None, [P, P, P, P, i64, P, P, i32, P]),
            "orc_jaccard_all": (None, [P, P, i64, P, P, i64, i32, P]),
            "orc_max_threads": (i32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(polys):
    """(xy int32 [V,2] contiguous, offsets int64 [N+1]) from a PolySet-like
    object (``.xy``/``.offsets``) or a (xy, offsets) pair."""
    if hasattr(polys, "xy"):
        xy, off = polys.xy, polys.offsets
    else:
        xy, off = polys
    return (np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2),
            np.ascontiguousarray(off, dtype=np.int64))


def _poly(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 2))


def _box(box) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(box, dtype=np.int32).reshape(4))


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ---------------------------------------------------------------- RNG -------

def mix64(z: int) -> int:
    return int(lib().orc_mix64(z & MASK64))


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().orc_splitmix64(seed & MASK64, count, _p(out))
    return out


def hash_keys(seed: int, k: int) -> np.ndarray:
    out = np.empty(k, dtype=np.uint64)
    lib().orc_hash_keys(seed & MASK64, k, _p(out))
    return out


def sample_point(box, key: int, j: int):
    b = _box(box)
    out = np.empty(2, dtype=np.int32)
    lib().orc_sample_point(_p(b), key & MASK64, j, _p(out))
    return int(out[0]), int(out[1])


def sample_points(box, key: int, count: int) -> np.ndarray:
    """The first ``count`` lattice points of one hash's stream, [count, 2]."""
    return np.array([sample_point(box, key, j) for j in range(count)], dtype=np.int64).reshape(-1, 2)


# ---------------------------------------------------------------- PnP -------

def inside(poly, px: int, py: int) -> bool:
    P = _poly(poly)
    return bool(lib().orc_inside(_p(P), P.shape[0], int(px), int(py)))


def inside_points(poly, pts) -> np.ndarray:
    P = _poly(poly)
    Q = np.ascontiguousarray(np.asarray(pts, dtype=np.int32).reshape(-1, 2))
    out = np.empty(Q.shape[0], dtype=np.uint8)
    lib().orc_inside_points(_p(P), P.shape[0], _p(Q), Q.shape[0], _p(out))
    return out.astype(bool)


# -------------------------------------------------------------- signing -----

def sign(polys, box, seed: int, k: int, cap: int, use_mbr: bool = True,
         threads: int = 0) -> np.ndarray:
    """Alg. 1 over every polygon: uint32 [N, k]."""
    xy, off = _csr(polys)
    n = off.shape[0] - 1
    out = np.zeros((n, k), dtype=np.uint32)
    if n == 0 or k == 0:
        return out
    b = _box(box)
    rc = lib().orc_sign(_p(xy), _p(off), n, _p(b), seed & MASK64, k, cap, int(use_mbr),
                        threads, _p(out))
    if rc != 0:
        raise MemoryError("oracle sign failed")
    return out


def band(sig: np.ndarray, bands: int, rows: int, band_seed: int = 0) -> np.ndarray:
    sig = np.ascontiguousarray(sig, dtype=np.uint32)
    n, k = sig.shape
    if bands * rows > k:
        raise ValueError("bands * rows exceeds the signature length")
    out = np.empty((n, bands), dtype=np.uint64)
    lib().orc_band(_p(sig), n, k, bands, rows, band_seed & MASK64, _p(out))
    return out


def candidates(dkeys: np.ndarray, qkeys: np.ndarray):
    """(cand_off int64 [nq+1], cand_ids int32 [C]) by brute-force comparison."""
    dkeys = np.ascontiguousarray(dkeys, dtype=np.uint64)
    qkeys = np.ascontiguousarray(qkeys, dtype=np.uint64)
    nd, b = dkeys.shape
    nq = qkeys.shape[0]
    off = np.zeros(nq + 1, dtype=np.int64)
    total = lib().orc_candidates(_p(dkeys), nd, _p(qkeys), nq, b, _p(off), None, 0)
    ids = np.empty(max(total, 1), dtype=np.int32)
    lib().orc_candidates(_p(dkeys), nd, _p(qkeys), nq, b, _p(off), _p(ids), total)
    return off, ids[:total]


# -------------------------------------------------------------- Jaccard -----

def area2(poly) -> int:
    P = _poly(poly)
    return int(lib().orc_area2(_p(P), P.shape[0]))


def intersection_area(P, Q) -> float:
    P, Q = _poly(P), _poly(Q)
    return float(lib().orc_intersection_area(_p(P), P.shape[0], _p(Q), Q.shape[0]))


def jaccard(P, Q) -> float:
    P, Q = _poly(P), _poly(Q)
    return float(lib().orc_jaccard(_p(P), P.shape[0], _p(Q), Q.shape[0]))


def jaccard_candidates(data, queries, cand_off, cand_ids, threads: int = 0) -> np.ndarray:
    dxy, doff = _csr(data)
    qxy, qoff = _csr(queries)
    cand_off = np.ascontiguousarray(cand_off, dtype=np.int64)
    cand_ids = np.ascontiguousarray(cand_ids, dtype=np.int32)
    out = np.zeros(cand_ids.shape[0], dtype=np.float64)
    if cand_ids.shape[0]:
        lib().orc_jaccard_candidates(_p(dxy), _p(doff), _p(qxy), _p(qoff), qoff.shape[0] - 1,
                                     _p(cand_off), _p(cand_ids), threads, _p(out))
    return out


def jaccard_all(data, queries, threads: int = 0) -> np.ndarray:
    dxy, doff = _csr(data)
    qxy, qoff = _csr(queries)
    nd, nq = doff.shape[0] - 1, qoff.shape[0] - 1
    out = np.zeros((nq, nd), dtype=np.float64)
    if nd and nq:
        lib().orc_jaccard_all(_p(dxy), _p(doff), nd, _p(qxy), _p(qoff), nq, threads, _p(out))
    return out


# Exact rational version of the same fan-decomposition clipping.

def _clip_half_exact(poly, a, b):
    out = []
    ex, ey = b[0] - a[0], b[1] - a[1]
    m = len(poly)
    for i in range(m):
        p, q = poly[i], poly[(i + 1) % m]
        sp = ex * (p[1] - a[1]) - ey * (p[0] - a[0])
        sq = ex * (q[1] - a[1]) - ey * (q[0] - a[0])
        if sp >= 0:
            out.append(p)
        if (sp > 0 and sq < 0) or (sp < 0 and sq > 0):
            t = sp / (sp - sq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def _area_exact(v):
    s = Fraction(0)
    m = len(v)
    for i in range(m):
        s += v[i][0] * v[(i + 1) % m][1] - v[(i + 1) % m][0] * v[i][1]
    return s / 2


def _fan_exact(P):
    tris = []
    a = (Fraction(int(P[0][0])), Fraction(int(P[0][1])))
    for i in range(1, len(P) - 1):
        b = (Fraction(int(P[i][0])), Fraction(int(P[i][1])))
        c = (Fraction(int(P[i + 1][0])), Fraction(int(P[i + 1][1])))
        o = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        if o > 0:
            tris.append(((a, b, c), 1))
        elif o < 0:
            tris.append(((a, c, b), -1))
    return tris


def intersection_area_exact(P, Q) -> Fraction:
    """area(P n Q) in exact rationals via the signed fan decomposition."""
    P, Q = _poly(P).tolist(), _poly(Q).tolist()
    if len(P) < 3 or len(Q) < 3:
        return Fraction(0)
    sP, sQ = np.sign(area2(P)), np.sign(area2(Q))
    if sP == 0 or sQ == 0:
        return Fraction(0)
    total = Fraction(0)
    for T, si in _fan_exact(P):
        for C, sj in _fan_exact(Q):
            poly = list(T)
            for e in range(3):
                if not poly:
                    break
                poly = _clip_half_exact(poly, C[e], C[(e + 1) % 3])
            if len(poly) >= 3:
                total += si * sj * _area_exact(poly)
    return int(sP * sQ) * total


def jaccard_exact(P, Q) -> Fraction:
    ai = intersection_area_exact(P, Q)
    u = Fraction(abs(area2(P)), 2) + Fraction(abs(area2(Q)), 2) - ai
    return ai / u if u > 0 else Fraction(0)


# --------------------------------------------------------- top-k, recall ----

def topk(cand_off, cand_ids, cand_j, k: int):
    """Per query, the k best candidates by (J desc, id asc); -1 / 0.0 pad."""
    nq = cand_off.shape[0] - 1
    ids = np.full((nq, k), -1, dtype=np.int32)
    js = np.zeros((nq, k), dtype=np.float64)
    for q in range(nq):
        a, b = int(cand_off[q]), int(cand_off[q + 1])
        ci, cj = cand_ids[a:b], cand_j[a:b]
        order = np.lexsort((ci, -cj))[:k]
        ids[q, :order.shape[0]] = ci[order]
        js[q, :order.shape[0]] = cj[order]
    return ids, js


def brute_force_topk(data, queries, k: int, threads: int = 0):
    """Def. 1 by brute force: exact J against every dataset polygon."""
    J = jaccard_all(data, queries, threads)
    nq, nd = J.shape
    off = np.arange(nq + 1, dtype=np.int64) * nd
    ids = np.tile(np.arange(nd, dtype=np.int32), nq)
    return topk(off, ids, J.reshape(-1), k)


def recall_at_k(ann_ids, ann_j, bf_ids, bf_j, k: int, tie_eps: float = 1e-12) -> float:
    """Sec. 5.2 recall@k: share of the brute-force top-k found by the ANN
    top-k, averaged over queries.  An ANN answer whose exact J ties the
    brute-force k-th value also counts (ties are otherwise arbitrary)."""
    nq = ann_ids.shape[0]
    if nq == 0:
        return 1.0
    tot = 0.0
    for q in range(nq):
        truth = set(int(i) for i in bf_ids[q, :k] if i >= 0)
        if not truth:
            tot += 1.0
            continue
        kth = bf_j[q, min(k, len(truth)) - 1]
        hit = 0
        for i, j in zip(ann_ids[q, :k], ann_j[q, :k]):
            if i < 0:
                continue
            if int(i) in truth or j >= kth - tie_eps:
                hit += 1
        tot += min(hit, len(truth)) / len(truth)
    return tot / nq
