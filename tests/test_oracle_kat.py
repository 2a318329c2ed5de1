"""Known answers (tests/golden/kat_rng_band.txt) of the oracle's random
source, hash keys, samples, lattice map and band keys: the published
SplitMix64 outputs for seed 0 and values derived from the generator's
definition outside the oracle.  A shifted sample or band index, a swapped
half of the draw or a band seed folded in the wrong way changes them."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kat_rng_band.txt")


def _records():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            f = line.split()
            out[f[0]] = f[1:]
    return out


def test_splitmix64_and_keys():
    r = _records()
    seed, *want = r["splitmix64"]
    got = oracle.splitmix64(int(seed), len(want))
    assert [int(x) for x in got] == [int(w, 16) for w in want]
    seed, *want = r["keys"]
    got = oracle.hash_keys(int(seed), len(want))
    assert [int(x) for x in got] == [int(w, 16) for w in want]


def test_samples_and_lattice():
    r = _records()
    seed, i, *want = r["samples"]
    key = int(oracle.hash_keys(int(seed), int(i) + 1)[int(i)])
    got = oracle.splitmix64(key, len(want))
    assert [int(x) for x in got] == [int(w, 16) for w in want]
    seed, i, bits, *xy = r["lattice"]
    key = int(oracle.hash_keys(int(seed), int(i) + 1)[int(i)])
    W = (1 << int(bits)) - 1
    pts = [oracle.sample_point((0, 0, W, W), key, j) for j in range(len(xy) // 2)]
    assert pts == [(int(xy[2 * j]), int(xy[2 * j + 1])) for j in range(len(xy) // 2)]


def test_band_keys():
    r = _records()
    seed, b, rows, sig, *want = r["band"]
    row = np.array([int(v) for v in sig.split(",")], dtype=np.uint32)[None, :]
    got = oracle.band(row, int(b), int(rows), int(seed))[0]
    assert [int(x) for x in got] == [int(w, 16) for w in want]
