"""GPU parity of signing and band keys against the CPU oracle: bit-exact."""
import numpy as np
import pytest

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


def _gpu_sign(pm, polys, box, seed, k, cap, **cfg):
    import torch
    D = pm.to_device(polys)
    config = pm.sign_config(**cfg) if cfg else None
    s = pm.sign(D, box, seed, k, cap, config=config)
    torch.cuda.synchronize()
    return s.cpu().numpy().view(np.uint32)


def _first_diff(a, b):
    d = np.argwhere(a != b)
    return None if d.size == 0 else (tuple(d[0]), a[tuple(d[0])], b[tuple(d[0])])


def test_sign_workload1_full(pm, orc):
    w = dg.workload(1)
    want = orc.sign(w.data, w.box, w.seed, w.k, w.cap)
    got = _gpu_sign(pm, w.data, w.box, w.seed, w.k, w.cap)
    assert _first_diff(got, want) is None, _first_diff(got, want)


CONFIGS = [
    dict(persistent=0),
    dict(persistent=1, block_threads=64, blocks_per_cu=16),
    dict(persistent=1, block_threads=512, hash_block=7),
    dict(persistent=0, block_threads=128, hash_block=1),
    dict(persistent=1, samples_per_lane=2),
    dict(persistent=1, lds_edges=64),            # most polygons stream their edges
    dict(persistent=0, samples_per_lane=2, lds_edges=64, hash_block=5),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=[str(c) for c in CONFIGS])
def test_sign_launch_shapes_agree(pm, orc, cfg):
    w = dg.workload(2, n=400, n_queries=0)
    k, cap = 40, w.cap
    want = orc.sign(w.data, w.box, w.seed, k, cap)
    got = _gpu_sign(pm, w.data, w.box, w.seed, k, cap, **cfg)
    assert _first_diff(got, want) is None, _first_diff(got, want)


def test_sign_workload2_subset(pm, orc):
    w = dg.workload(2, n=1500, n_queries=0)
    want = orc.sign(w.data, w.box, w.seed, w.k, w.cap)
    got = _gpu_sign(pm, w.data, w.box, w.seed, w.k, w.cap)
    assert _first_diff(got, want) is None, _first_diff(got, want)


def test_sign_workload2_full_size_sampled(pm, orc):
    # full 100,000-polygon set in the default (benchmarked) launch shape;
    # 300 sampled polygons recomputed by the oracle
    w = dg.workload(2)
    got = _gpu_sign(pm, w.data, w.box, w.seed, w.k, w.cap)
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(w.data.n, 300, replace=False))
    want = orc.sign(w.data.subset(ids), w.box, w.seed, w.k, w.cap)
    assert _first_diff(got[ids], want) is None, _first_diff(got[ids], want)
    assert (got > 0).all()


def test_sign_heavy_tail_sample(pm, orc):
    # workload 5's vertex-count and area distributions (Pareto counts up to
    # 8192 vertices, small polygons): a seeded subset with a reduced cap
    w = dg.workload(5, n=300, n_queries=0)
    k, cap = 16, 1 << 16
    want = orc.sign(w.data, w.box, w.seed, k, cap)
    got = _gpu_sign(pm, w.data, w.box, w.seed, k, cap)
    assert _first_diff(got, want) is None, _first_diff(got, want)


def test_sign_edge_cases(pm, orc):
    rng = np.random.default_rng(1)
    star = dg.star_polygons(rng, [40], [[500, 500]], [300.0]).xy
    big = dg.star_polygons(rng, [3000], [[600, 400]], [6000.0]).xy     # > lds_edges
    wide = dg.star_polygons(rng, [12], [[0, 0]], [float(1 << 26)]).xy  # 128-bit path
    polys = [
        np.zeros((0, 2)), [[1, 1]], [[1, 1], [5, 5]],
        [[0, 0], [40, 20], [80, 40], [20, 10]],          # collinear
        dg.rectangle(0, 0, 1, 1), dg.rectangle(3, 4, 900, 30),
        star, star[::-1], np.roll(star, 7, axis=0),
        dg.rectangle(-500, -500, 20, 20),                  # crosses B's corner
        dg.rectangle(2000, 2000, 2100, 2100),              # outside B
        big, wide,
    ]
    ps = dg.from_list(polys)
    for box in [(0, 0, 1023, 1023), (-7, 3, 993, 1099), (5, 5, 5, 5), (0, 0, 1, 2000),
                (-6000, -6000, 8191, 8191)]:
        for k, cap in [(1, 1), (9, 17), (33, 1 << 20)]:
            want = orc.sign(ps, box, 3, k, cap)
            got = _gpu_sign(pm, ps, box, 3, k, cap)
            assert _first_diff(got, want) is None, (box, k, cap, _first_diff(got, want))


def test_sign_extreme_box(pm, orc):
    # full-int32 box (2^32 wide), and a wide-but-not-power-of-two box
    ps = dg.from_list([dg.rectangle(-(1 << 30), -(1 << 30), 1 << 30, 1 << 30),
                       dg.rectangle(0, 0, 1 << 29, 1 << 28)])
    for box in [(-(1 << 31), -(1 << 31), (1 << 31) - 1, (1 << 31) - 1),
                (-(1 << 31), -5, (1 << 31) - 1, 3 * (1 << 29))]:
        want = orc.sign(ps, box, 11, 24, 1 << 12)
        got = _gpu_sign(pm, ps, box, 11, 24, 1 << 12)
        assert _first_diff(got, want) is None, (box, _first_diff(got, want))


def test_sign_empty_set(pm):
    ps = dg.from_list([])
    got = _gpu_sign(pm, ps, (0, 0, 15, 15), 0, 8, 100)
    assert got.shape == (0, 8)


def test_sign_invalid_arguments(pm):
    ps = pm.to_device(dg.from_list([dg.rectangle(0, 0, 2, 2)]))
    with pytest.raises(pm.PolymhError) as e:
        pm.sign(ps, (5, 0, 4, 10), 0, 8, 100)
    assert e.value.status == pm.ERANGE
    with pytest.raises(pm.PolymhError) as e:
        pm.sign(ps, (0, 0, 4, 10), 0, 0, 100)
    assert e.value.status == pm.EINVAL
    with pytest.raises(pm.PolymhError):
        pm.sign(ps, (0, 0, 4, 10), 0, 8, 100, config=pm.sign_config(block_threads=100))


def test_band_bitexact(pm, orc):
    import torch
    rng = np.random.default_rng(2)
    sig = rng.integers(0, 2**32, (777, 64), dtype=np.uint64).astype(np.uint32)
    sig[5] = sig[9]
    sig[100:110] = 0
    t = torch.from_numpy(sig.view(np.int32)).cuda()
    for b, r, seed in [(16, 4, 0), (1, 64, 5), (64, 1, 7), (7, 9, 2**64 - 1), (3, 1, 1)]:
        got = pm.band(t, b, r, seed).cpu().numpy().view(np.uint64)
        want = orc.band(sig, b, r, seed)
        assert np.array_equal(got, want), (b, r, seed)
