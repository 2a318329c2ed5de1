"""Workload 5 at full size (4,000,000 polygons, Pareto vertex counts up to
8,192, small areas so first hits are long; k = 256, cap 2^26) in the
launch configuration the benchmark times: binned signing equals the walk on
every polygon, and the oracle recomputes the signatures and band keys
(32 x 8) of sampled polygons bit-exactly."""
import time

import numpy as np
import pytest

from paper_2511_16576_amd import datagen as dg

pytestmark = pytest.mark.gpu


def test_binned_signing_workload5_full_size(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_16576_amd import polymh as pm
    pm.check_device()
    t0 = time.time()
    w = dg.workload(5, n_queries=0)
    print(f"workload 5: {w.data.n} polygons, {w.data.xy.shape[0]} vertices, generated in "
          f"{time.time() - t0:.1f}s", flush=True)
    D = pm.to_device(w.data)
    h, b = pm.binned_params(D, w.box, w.k, w.cap)
    sig = pm.sign_binned(D, w.box, w.seed, w.k, w.cap, horizon=h, bin_bits=b)
    torch.cuda.synchronize()
    print(f"binned: horizon {h}, {1 << b} x {1 << b} cells", flush=True)
    walk = pm.sign(D, w.box, w.seed, w.k, w.cap)
    assert torch.equal(sig, walk)
    del walk
    keys = pm.band(sig, 32, 8, w.seed).cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(21)
    ids = np.sort(rng.choice(w.data.n, 48, replace=False))
    want = orc.sign(w.data.subset(ids), w.box, w.seed, w.k, w.cap)
    got = sig.cpu().numpy().view(np.uint32)[ids]
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]
    assert np.array_equal(keys[ids], orc.band(want, 32, 8, w.seed))
