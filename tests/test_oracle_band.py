"""Pins of the oracle's band keys and candidate sets (Sec. 3.2 hashmap filter,
banded as in the MMDS banding technique the paper cites)."""
import math

import numpy as np

from paper_2511_16576_amd import datagen as dg


def test_band_locality(orc):
    rng = np.random.default_rng(0)
    b, r = 6, 3
    sig = rng.integers(0, 2**32, (5, b * r + 2), dtype=np.uint64).astype(np.uint32)
    keys = orc.band(sig, b, r, band_seed=17)
    for p in range(sig.shape[0]):
        for u in range(b * r + 2):
            s2 = sig.copy()
            s2[p, u] ^= np.uint32(1 << (u % 32))
            k2 = orc.band(s2, b, r, band_seed=17)
            changed = np.flatnonzero((k2 != keys).any(axis=0))
            if u < b * r:
                # exactly the band holding row u changes, and only for polygon p
                assert changed.tolist() == [u // r]
                assert np.flatnonzero(k2[:, u // r] != keys[:, u // r]).tolist() == [p]
            else:
                assert changed.size == 0       # rows past b*r are unused


def test_band_index_and_seed_are_folded_in(orc):
    sig = np.tile(np.arange(1, 5, dtype=np.uint32), 4).reshape(1, 16)   # 4 identical bands
    keys = orc.band(sig, 4, 4, band_seed=0)
    assert len(set(keys[0].tolist())) == 4
    assert not np.array_equal(orc.band(sig, 4, 4, band_seed=1), keys)
    same = np.repeat(sig, 3, axis=0)
    k3 = orc.band(same, 4, 4, band_seed=0)
    assert (k3 == k3[0]).all()


def test_candidates_definition(orc):
    rng = np.random.default_rng(1)
    nd, nq, b = 60, 9, 5
    dkeys = rng.integers(0, 4, (nd, b), dtype=np.uint64)
    qkeys = rng.integers(0, 4, (nq, b), dtype=np.uint64)
    off, ids = orc.candidates(dkeys, qkeys)
    for q in range(nq):
        want = [p for p in range(nd) if any(dkeys[p, t] == qkeys[q, t] for t in range(b))]
        assert ids[off[q]:off[q + 1]].tolist() == want


def test_candidate_probability_s_curve(orc):
    # With J the rectangle pair's Jaccard, a pair shares a band with
    # probability 1 - (1 - J^r)^b (independent hashes, Thm. 1 per row).
    a, c = (0, 0, 40, 40), (8, 0, 48, 40)          # J = 1280 / 1920 = 2/3
    J = 1280 / 1920
    b, r, trials = 4, 3, 300
    polys = dg.from_list([dg.rectangle(*a), dg.rectangle(*c)])
    hits = 0
    for s in range(trials):
        sig = orc.sign(polys, (0, 0, 127, 127), seed=1000 + s, k=b * r, cap=1 << 30)
        keys = orc.band(sig, b, r, band_seed=s)
        hits += bool((keys[0] == keys[1]).any())
    p = 1 - (1 - J ** r) ** b
    assert abs(hits / trials - p) < 5 * math.sqrt(p * (1 - p) / trials)
