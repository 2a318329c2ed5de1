"""CPU oracle of centring (Sec. 3.1) -- TEST INFRASTRUCTURE ONLY.

Each polygon is translated so that its area centroid, rounded to the
lattice, lands on the origin.  The centroid of a simple polygon is the
area-weighted mean of its signed fan triangles,
    C = sum_i (v_i + v_{i+1}) cross(v_i, v_{i+1}) / (3 sum_i cross(v_i, v_{i+1})),
computed here in Python's exact integers; each coordinate is rounded by
floor(c + 1/2), a rounding that commutes with integer translations (so a
polygon and any integer translate of it centre to the same vertices).
Polygons with fewer than 3 vertices or zero area are not moved.

Pinned (tests) by closed forms independent of this formula: rectangle and
triangle centroids, an L-shape as the area-weighted mean of its two
rectangles, invariance under ring reversal and rotation, exact translation
equivariance, and identical signatures (J = 1) of a polygon and its
translate after centring.
"""
from __future__ import annotations

import numpy as np


def centroid_shift(poly) -> tuple[int, int]:
    """(sx, sy): the rounded area centroid, i.e. the translation removed."""
    P = [(int(x), int(y)) for x, y in np.asarray(poly).reshape(-1, 2)]
    n = len(P)
    if n < 3:
        return 0, 0
    a2 = nx = ny = 0
    for i in range(n):
        (x0, y0), (x1, y1) = P[i], P[(i + 1) % n]
        c = x0 * y1 - x1 * y0
        a2 += c
        nx += (x0 + x1) * c
        ny += (y0 + y1) * c
    if a2 == 0:
        return 0, 0
    # floor(nx / (3 a2) + 1/2) = floor((2 nx + 3 a2) / (6 a2)); // floors for either sign
    return (2 * nx + 3 * a2) // (6 * a2), (2 * ny + 3 * a2) // (6 * a2)


def centre(polys):
    """(xy int32 [V, 2] translated, shifts int64 [N, 2]) of a PolySet-like set."""
    xy = np.asarray(polys.xy, dtype=np.int64).reshape(-1, 2)
    off = np.asarray(polys.offsets, dtype=np.int64)
    out = xy.copy()
    shifts = np.zeros((off.shape[0] - 1, 2), dtype=np.int64)
    for p in range(off.shape[0] - 1):
        a, b = int(off[p]), int(off[p + 1])
        sx, sy = centroid_shift(xy[a:b])
        shifts[p] = (sx, sy)
        out[a:b, 0] -= sx
        out[a:b, 1] -= sy
    return out.astype(np.int32), shifts
