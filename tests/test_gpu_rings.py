"""Polygons with holes and multipolygons on the GPU path: shapes joined into
single rings (``polymh_join_rings``) sign bit-exactly like the ring-aware
oracle (even-odd membership over all rings), refine to its ring-pair
Jaccard within the refinement tolerance, and centre to its centroid."""
import numpy as np
import pytest

from oracle import rings as orr
from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu

REL, ABS = 1e-9, 1e-12


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh
    polymh.check_device()
    return polymh


def _shapes(n=40, seed=11):
    rng = np.random.default_rng(seed)
    return dg.ring_polygons(rng, n, 16, lambda r, m: r.integers(6, 40, m), 0.04, 0.12)


def _moved(rs, rng):
    """Every shape translated by up to a quarter of its extent."""
    polys = []
    for p in range(rs.n):
        rings = rs.rings(p)
        ext = int(np.ptp(rings[0][:, 0]))
        d = rng.integers(-ext // 4, ext // 4 + 1, 2)
        polys.append([r.astype(np.int64) + d for r in rings])
    return dg.from_rings(polys)


def _joined_host(rs):
    """The joined rings built here from their definition."""
    out, off = [], [0]
    for p in range(rs.n):
        rings = rs.rings(p)
        seq = [rings[0]]
        if len(rings) > 1:
            v0 = rings[0][:1]
            seq.append(v0)
            for i, r in enumerate(rings[1:]):
                seq.append(r)
                seq.append(r[:1])
                if i + 2 < len(rings):
                    seq.append(v0)
        ring = np.concatenate(seq)
        out.append(ring)
        off.append(off[-1] + ring.shape[0])
    return np.concatenate(out).astype(np.int32), np.asarray(off, dtype=np.int64)


def test_join_layout(pm):
    rs = _shapes()
    J = pm.join_rings(pm.rings_to_device(rs))
    xy, off = _joined_host(rs)
    assert np.array_equal(J.offsets.cpu().numpy(), off)
    assert np.array_equal(J.xy.cpu().numpy()[:off[-1]], xy)
    # a one-ring set is copied unchanged
    one = dg.from_rings([[rs.rings(0)[0]], [rs.rings(1)[0]]])
    J1 = pm.join_rings(pm.rings_to_device(one))
    assert np.array_equal(J1.xy.cpu().numpy(), one.xy)


@pytest.mark.parametrize("k,cap", [(16, 1 << 16), (5, 40)])
def test_sign_matches_ring_oracle(pm, orc, k, cap):
    rs = _shapes()
    box = (0, 0, (1 << 16) - 1, (1 << 16) - 1)
    want = orr.sign_rings(rs, box, 7, k, cap)
    D = pm.join_rings(pm.rings_to_device(rs))
    got = pm.sign(D, box, 7, k, cap).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]
    for bits, ratio in [(3, 0.0), (5, 300.0)]:
        gb = pm.sign_binned(D, box, 7, k, cap, horizon=min(cap, 4096), bin_bits=bits,
                            walk_ratio=ratio).cpu().numpy().view(np.uint32)
        assert np.array_equal(gb, want), (bits, ratio)


def test_refine_matches_ring_oracle(pm, orc):
    import torch
    rng = np.random.default_rng(5)
    data = _shapes(30, seed=12)
    queries = _moved(data, rng)
    D = pm.join_rings(pm.rings_to_device(data))
    Q = pm.join_rings(pm.rings_to_device(queries))
    # every query against every shape (its translate among them)
    off = torch.arange(Q.n + 1, dtype=torch.int64, device="cuda") * D.n
    ids = torch.arange(D.n, dtype=torch.int32, device="cuda").repeat(Q.n)
    got = pm.refine(D, Q, off, ids).cpu().numpy().reshape(Q.n, D.n)
    want = np.array([[orr.jaccard_rings(data.rings(p), queries.rings(q)) for p in range(D.n)]
                     for q in range(Q.n)])
    err = np.abs(got - want)
    assert np.all(err <= REL * np.abs(want) + ABS), (err.max(), np.unravel_index(np.argmax(err), err.shape))
    assert (np.diag(want) > 0.2).sum() >= 20       # translates overlap, holes included


def test_centre_matches_ring_oracle(pm):
    rs = _shapes(25, seed=13)
    C, shift = pm.centre(pm.join_rings(pm.rings_to_device(rs)))
    want = np.array([orr.centroid_shift_rings(rs.rings(p)) for p in range(rs.n)], dtype=np.int64)
    assert np.array_equal(shift.cpu().numpy().astype(np.int64), want)


def test_invalid_shapes_raise(pm):
    sq = dg.rectangle(0, 0, 5, 5)
    bad_ring = dg.from_rings([[sq, np.array([[1, 1], [2, 2]])]])
    with pytest.raises(ValueError):
        pm.join_rings(pm.rings_to_device(bad_ring))
    rs = dg.from_rings([[sq], [sq]])
    rs.poly_rings = np.array([0, 1, 1], dtype=np.int64)     # second shape without rings
    rs.ring_offsets = rs.ring_offsets[:2]
    rs.xy = rs.xy[:4]
    with pytest.raises(ValueError):
        pm.join_rings(pm.rings_to_device(rs))


def test_refine_large_rings_windowed(pm, orc):
    # joined shapes of about 500 to 3,000 vertices (components of 500-1,400
    # with holes and bridges): pairs beyond 512 edges take the tiled form in
    # windows (split over windows beyond 1,024 a side) and equal the ring
    # oracle and the general form (the call without workspace)
    import torch
    rng = np.random.default_rng(15)
    data = dg.ring_polygons(rng, 12, 16, lambda r, m: r.integers(500, 1400, m), 0.04, 0.12)
    queries = _moved(data, rng)
    D = pm.join_rings(pm.rings_to_device(data))
    Q = pm.join_rings(pm.rings_to_device(queries))
    nd = np.diff(D.offsets.cpu().numpy())
    assert nd.min() < 1024 < nd.max()
    off = torch.arange(Q.n + 1, dtype=torch.int64, device="cuda") * D.n
    ids = torch.arange(D.n, dtype=torch.int32, device="cuda").repeat(Q.n)
    got, st = pm.refine_stats(D, Q, off, ids)
    got = got.cpu().numpy().reshape(Q.n, D.n)
    inplace = pm.refine(D, Q, off, ids, split_heavy=False).cpu().numpy().reshape(Q.n, D.n)
    want = np.array([[orr.jaccard_rings(data.rings(p), queries.rings(q)) for p in range(D.n)]
                     for q in range(Q.n)])
    err = np.abs(got - want)
    assert np.all(err <= REL * np.abs(want) + ABS), (err.max(), np.unravel_index(np.argmax(err), err.shape))
    assert np.all(np.abs(inplace - want) <= REL * np.abs(want) + ABS)
    assert (np.diag(want) > 0.2).sum() >= 8 and st[2] == 0
