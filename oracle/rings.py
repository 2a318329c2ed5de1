"""CPU oracle of polygons with holes and multipolygons -- TEST INFRASTRUCTURE
ONLY.

A polygon is a list of rings (filled rings counter-clockwise, holes
clockwise).  Following the paper's point-in-polygon step taken over every
ring of the shape (the even-odd rule), a lattice point is inside when the
half-open crossing count summed over all rings is odd, i.e. the XOR of the
per-ring tests of ``core.inside``.  Its area is the sum of the rings'
signed shoelace areas, and the area of the intersection of two such
shapes is the sum over ring pairs of (orientation sign) x (orientation
sign) x (area of the intersection of the two ring interiors), from
``core.intersection_area``, times the orientation signs of the two shapes'
total areas; for properly nested rings this is the area of
the intersection of the two even-odd regions (the product of their
winding numbers integrated over the plane).  Signatures walk Alg. 1's point
stream (``core.sample_points``) and stop at the first point inside.  The
centroid sums the rings' fan moments about the origin in exact integers and
rounds like ``centre.centroid_shift``.

Pinned (tests/test_oracle_rings.py) by closed forms: a square with a square
hole (area, membership of points in the hole and in the ring, centroid of an
off-centre hole as the area-weighted difference of two squares), the
intersection of a holed square with rectangles, J of a shape with itself,
of a two-component multipolygon with one component, the union law
h(A u B) = min(h(A), h(B)) for disjoint components, agreement with
``core.sign`` on single-ring shapes, and h(P with hole) >= h(outer ring)
with equality where the outer ring's first hit is outside the hole.
"""
from __future__ import annotations

import numpy as np

from . import core


def area2_rings(rings) -> int:
    """Twice the signed area: the sum of the rings' shoelace sums."""
    return sum(core.area2(r) for r in rings)


def inside_rings(rings, px: int, py: int) -> bool:
    odd = False
    for r in rings:
        odd ^= core.inside(r, px, py)
    return odd


def inside_points_rings(rings, pts) -> np.ndarray:
    pts = np.asarray(pts, dtype=np.int64).reshape(-1, 2)
    odd = np.zeros(pts.shape[0], dtype=bool)
    for r in rings:
        odd ^= core.inside_points(r, pts)
    return odd


def sign_rings(ringset, box, seed: int, k: int, cap: int) -> np.ndarray:
    """Alg. 1 / Def. 2 over every shape of a RingSet-like set: uint32 [N, k]
    (1-based first hit, 0 when none of the first ``cap`` points is inside)."""
    n = ringset.n
    keys = core.hash_keys(seed, k)
    out = np.zeros((n, k), dtype=np.uint32)
    for p in range(n):
        rings = ringset.rings(p)
        for i in range(k):
            count = min(256, cap)
            while True:
                pts = core.sample_points(box, int(keys[i]), count)
                hit = np.flatnonzero(inside_points_rings(rings, pts))
                if hit.size:
                    out[p, i] = int(hit[0]) + 1
                    break
                if count >= cap:
                    break
                count = min(4 * count, cap)
    return out


def intersection_area_rings(P, Q) -> float:
    """Area of the intersection; a shape given with every ring reversed (filled
    rings clockwise, holes counter-clockwise) is the same shape, so the sum is
    taken with the orientation of each shape's total area."""
    sP, sQ = np.sign(area2_rings(P)), np.sign(area2_rings(Q))
    if sP == 0 or sQ == 0:
        return 0.0
    total = 0.0
    for a in P:
        sa = np.sign(core.area2(a))
        if sa == 0:
            continue
        for b in Q:
            sb = np.sign(core.area2(b))
            if sb == 0:
                continue
            total += float(sa * sb) * core.intersection_area(a, b)
    return float(sP * sQ) * total


def jaccard_rings(P, Q) -> float:
    ai = intersection_area_rings(P, Q)
    u = 0.5 * abs(area2_rings(P)) + 0.5 * abs(area2_rings(Q)) - ai
    return ai / u if u > 0 else 0.0


def centroid_shift_rings(rings) -> tuple[int, int]:
    """Rounded area centroid of the shape (floor(c + 1/2) per coordinate);
    (0, 0) for fewer than 3 vertices in all or zero area."""
    a2 = nx = ny = 0
    nv = 0
    for r in rings:
        R = [(int(x), int(y)) for x, y in np.asarray(r).reshape(-1, 2)]
        nv += len(R)
        for i in range(len(R)):
            (x0, y0), (x1, y1) = R[i], R[(i + 1) % len(R)]
            c = x0 * y1 - x1 * y0
            a2 += c
            nx += (x0 + x1) * c
            ny += (y0 + y1) * c
    if nv < 3 or a2 == 0:
        return 0, 0
    return (2 * nx + 3 * a2) // (6 * a2), (2 * ny + 3 * a2) // (6 * a2)
