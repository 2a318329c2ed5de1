"""GPU parity of centring (Sec. 3.1) against the oracle (bit-exact), and its
purpose end to end: after centring, a polygon and its integer translates
sign identically (Thm. 1: collision rate 1) and refine to J = 1."""
import numpy as np
import pytest

from oracle import centre as oc
from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh
    polymh.check_device()
    return polymh


def _edge_set():
    rng = np.random.default_rng(4)
    big = dg.star_polygons(rng, [700], [[0, 0]], [3.0e6]).xy
    return dg.from_list([
        np.zeros((0, 2)), [[5, 5]], [[1, 1], [9, 9]],                  # fewer than 3 vertices
        [[0, 0], [4, 2], [8, 4]],                                      # zero area
        dg.rectangle(3, -7, 8, 2), dg.rectangle(-9, -9, -2, 5)[::-1],  # half-integer centroids
        [[-4, 1], [7, 3], [2, 11]],
        [(0, 0), (7, 0), (7, 2), (2, 2), (2, 9), (0, 9)],
        big, big + np.array([(1 << 30) - (1 << 23), -(1 << 30) + (1 << 23)]),
    ])


@pytest.mark.parametrize("which", ["workload1", "workload2_subset", "edges"])
def test_centre_matches_oracle(pm, which):
    if which == "workload1":
        ps = dg.workload(1).data
    elif which == "workload2_subset":
        ps = dg.workload(2, n=5000, n_queries=0).data
    else:
        ps = _edge_set()
    D = pm.to_device(ps)
    C, shift = pm.centre(D)
    want_xy, want_shift = oc.centre(ps)
    assert np.array_equal(C.xy.cpu().numpy(), want_xy)
    assert np.array_equal(shift.cpu().numpy().astype(np.int64), want_shift)


def test_translates_sign_identically_after_centring(pm, orc):
    import torch
    rng = np.random.default_rng(9)
    base = dg.workload(2, n=200, n_queries=0).data
    moves = rng.integers(-(1 << 22), 1 << 22, (base.n, 2))
    moved = dg.from_list([base.poly(p) + moves[p] for p in range(base.n)])
    both = dg.concat([base, moved])
    C, _ = pm.centre(pm.to_device(both))
    box = pm.box_of(C)
    sig = pm.sign(C, box, 0, 64, 1 << 22).cpu().numpy()
    assert np.array_equal(sig[:base.n], sig[base.n:])
    # J = 1 between each polygon and its translate, 0 < J < 1 before centring
    off = torch.arange(base.n + 1, dtype=torch.int64, device="cuda")
    ids = torch.arange(base.n, dtype=torch.int32, device="cuda")
    Cb = pm.DevicePolys(C.xy[:base.offsets[-1]].contiguous(), C.offsets[:base.n + 1].contiguous())
    Cm = pm.DevicePolys(C.xy[base.offsets[-1]:].contiguous(),
                        (C.offsets[base.n:] - C.offsets[base.n]).contiguous())
    J = pm.refine(Cb, Cm, off, ids).cpu().numpy()
    assert np.all(np.abs(J - 1.0) < 1e-12)
    # the same polygons uncentred differ
    D = pm.to_device(both)
    Du = pm.DevicePolys(D.xy[base.offsets[-1]:].contiguous(), (D.offsets[base.n:] - D.offsets[base.n]).contiguous())
    Db = pm.DevicePolys(D.xy[:base.offsets[-1]].contiguous(), D.offsets[:base.n + 1].contiguous())
    Ju = pm.refine(Db, Du, off, ids).cpu().numpy()
    assert np.all(Ju < 1.0)


def test_centre_range_flag(pm):
    tri = dg.from_list([[(-(1 << 31), 0), ((1 << 31) - 1, 0), ((1 << 31) - 1, 1)]])
    with pytest.raises(ValueError):
        pm.centre(pm.to_device(tri))
