"""Pins of the scorer's CPU oracle (oracle/mlp.py): finite differences, the
erf form of GELU, Adam's first step and closed-form shape features."""
import math

import numpy as np
from scipy.special import erf

from oracle import mlp as om


def _params(rng, scale=0.1):
    return rng.normal(0, scale, om.N_PARAMS)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    p = _params(rng, 0.08)
    X = rng.normal(0, 1, (5, om.N_IN))
    lab = rng.random(5)
    g = om.backward(X, p, lab)
    idx = np.concatenate([rng.choice(om.N_PARAMS, 60, replace=False),
                          [om.OFF_B1, om.OFF_W2 + 7, om.OFF_B2 + 3, om.OFF_W3 + 11, om.OFF_B3]])
    h = 1e-6
    for i in idx:
        e = np.zeros(om.N_PARAMS)
        e[i] = h
        fd = (om.loss(X, p + e, lab) - om.loss(X, p - e, lab)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_mixed_precision_network_reduces_to_fp64_and_stays_within_bf16():
    """forward_mixed / backward_mixed with the rounding off are the FP64
    network and its chain-rule gradient (pinned by finite differences
    above); with it on, every gradient entry moves by at most a few BF16
    roundings of its terms, while a real change of the network (a
    perturbed weight) moves the gradient far more."""
    rng = np.random.default_rng(3)
    p = _params(rng, 0.06)
    X = om.bf16_round(rng.normal(0, 1, (24, om.N_IN)).astype(np.float32)).astype(np.float64)
    lab = rng.random(24)
    assert np.array_equal(om.forward_mixed(X, p, bf16=False)["y"], om.forward(X, p)["y"])
    assert np.array_equal(om.backward_mixed(X, p, lab, bf16=False), om.backward(X, p, lab))
    g, S = om.backward_mixed(X, p, lab, terms=True)
    g0 = om.backward(X, p, lab)
    assert np.all(np.abs(g - g0) <= 2 ** -6 * S + 1e-15)
    ya, yb = om.forward_mixed(X, p)["y"], om.forward(X, p)["y"]
    assert np.abs(ya - yb).max() < 2 ** -7 * 0.25 * np.abs(p[om.OFF_W3:om.OFF_B3]).sum()
    p2 = p.copy()
    p2[om.OFF_W2 + 5 * om.N_HID + 7] += 0.3        # one weight of W2 changed
    g2 = om.backward_mixed(X, p2, lab)
    assert (np.abs(g2 - g) > 2 ** -6 * S + 1e-15).sum() > 100


def test_adam_constant_gradient_every_step():
    """With the same gradient g at every step the bias-corrected moments are
    exactly g and g^2, so each step moves p by lr g / (|g| + eps): a
    correction frozen at its first-step value would not."""
    rng = np.random.default_rng(4)
    p = rng.normal(size=40)
    g = rng.normal(size=40)
    m, v = np.zeros(40), np.zeros(40)
    for step in range(1, 8):
        p1, m, v = om.adam_step(p, g, m, v, step, lr=1e-3, eps=1e-8)
        assert np.allclose(p - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15), step
        p = p1


def test_gelu_tanh_form_tracks_erf_form():
    z = np.linspace(-6, 6, 2001)
    exact = 0.5 * z * (1 + erf(z / math.sqrt(2)))
    assert np.abs(om.gelu(z) - exact).max() < 1e-3
    dz = 1e-6
    fd = (om.gelu(z + dz) - om.gelu(z - dz)) / (2 * dz)
    assert np.abs(fd - om.gelu_grad(z)).max() < 1e-6


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = om.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=1e-8)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.0, 1e-30, 65504.0], dtype=np.float32)
    r = om.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0          # tie rounds to even
    assert r[2] == np.float32(1.0078125)
    assert r[3] == -3.0
    assert (om.bf16_round(r) == r).all()


def test_poly_features_closed_forms():
    box = (0, 0, 1023, 1023)
    f = om.poly_features([[0, 0], [10, 0], [10, 5], [0, 5]], box)
    assert f[6] == 50
    assert math.isclose(f[0], math.log(50) / math.log(1024 * 1024))
    assert math.isclose(f[1], math.log(900 / (4 * math.pi * 50)) / 4)
    assert math.isclose(f[2], math.log(11 / 6) / 2)
    assert math.isclose(f[3], math.log(4) / 9)
    assert abs(f[4]) < 1e-12 and abs(f[5]) < 1e-12
    assert list(f[8:12]) == [0, 0, 11, 6]
    t = om.poly_features([[0, 0], [6, 0], [0, 3]], box)
    assert t[6] == 9
    assert math.isclose(t[4], (2 - 3) / 3) and math.isclose(t[5], (1 - 1.5) / 3)
    assert math.isclose(t[1], math.log((9 + math.sqrt(45)) ** 2 / (36 * math.pi)) / 4)


def test_pair_row_layout():
    rng = np.random.default_rng(2)
    s1 = rng.integers(1, 5, 256)
    s2 = s1.copy()
    s2[:64] += 1
    f1 = om.poly_features([[0, 0], [10, 0], [10, 10], [0, 10]], (0, 0, 99, 99))
    f2 = om.poly_features([[5, 0], [15, 0], [15, 10], [5, 10]], (0, 0, 99, 99))
    row = om.pair_features(s1, f1, s2, f2)
    assert row[:64].sum() == 0 and row[64:256].sum() == 192
    assert row[271] == 0.75
    assert row[269] == 1.0 and row[268] == 0.0
    assert math.isclose(row[270], (6 * 11) / (2 * 121 - 66))
    assert (row[272:] == 0).all()
