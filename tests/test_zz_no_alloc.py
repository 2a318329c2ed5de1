"""polymh_sign_static -- signing on the library's static scratch, with no
allocation -- against polymh_sign with a caller workspace: bit-exact on two
calls in a row, the second on fewer polygons (the scratch keeps the first
call's staging), in both launch forms, replayed from a captured graph, and
against the oracle; sizes beyond the scratch are rejected before any
launch."""
import numpy as np
import pytest

import oracle
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


@pytest.fixture(scope="module")
def sets(pm):
    w = dg.workload(2, n=6000, n_queries=0)
    big = pm.to_device(w.data)
    sub = w.data.subset(np.arange(0, 6000, 9))
    return w, big, sub, pm.to_device(sub)


@pytest.mark.parametrize("persistent", [1, 0])
def test_sign_static_equals_sign(pm, sets, persistent):
    import torch
    w, big, sub_h, small = sets
    cfg = pm.sign_config(persistent=persistent)
    for polys, k in ((big, 128), (small, 64)):     # second call on fewer polygons
        a = pm.sign_static(polys, w.box, 0, k, w.cap, config=cfg)
        b = pm.sign(polys, w.box, 0, k, w.cap, config=cfg)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (polys.n, k)
    want = oracle.sign(sub_h, w.box, 0, 64, w.cap)
    assert np.array_equal(a.cpu().numpy().view(np.uint32), want)


def test_sign_static_in_a_graph(pm, sets):
    """Captured and replayed (the callers it is for), with eager work of the
    program between replays."""
    import torch
    w, big, _, small = sets
    ref = pm.sign(small, w.box, 7, 32, w.cap)
    out = torch.empty_like(ref)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pm.sign_static(small, w.box, 7, 32, w.cap, out=out, stream=stream)
    stream.synchronize()
    assert torch.equal(out, ref)
    g = pm.capture(lambda: pm.sign_static(small, w.box, 7, 32, w.cap, out=out, stream=stream), stream)
    for _ in range(3):
        out.fill_(0)
        torch.cuda.synchronize()
        g.launch()
        stream.synchronize()
        assert torch.equal(out, ref)
        pm.sign_static(big, w.box, 1, 16, w.cap)      # another call between replays
        torch.cuda.synchronize()


def test_sign_static_rejects_too_many_polygons(pm):
    import torch
    n = pm.SIGN_STATIC_MAX_POLYS + 1
    polys = pm.DevicePolys(torch.zeros((3, 2), dtype=torch.int32, device="cuda"),
                           torch.zeros(n + 1, dtype=torch.int64, device="cuda"))
    sig = torch.empty((n, 4), dtype=torch.int32, device="cuda")   # sized as if it ran
    with pytest.raises(pm.PolymhError) as e:
        pm.sign_static(polys, (0, 0, 15, 15), 0, 4, 16, out=sig)
    assert e.value.status == pm.EINVAL and "at most" in str(e.value)
