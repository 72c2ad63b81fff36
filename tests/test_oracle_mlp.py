"""Pins of the oracle's surrogate-network reference: finite differences and bf16 rounding."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-5])
    r = mlp.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[3] == 1.0 + 2 ** -6
    assert r[4] == -2.5
    assert abs(r[5] / 3.0e-5 - 1) < 2 ** -8


def test_dsilu_closed_form():
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.dsilu(z))) < 1e-9


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_par = 256 * 16 + 256 + 2 * (256 * 256 + 256) + 144 * 256 + 144
    w = rng.normal(0, 0.05, n_par)
    x = np.zeros((8, 16))
    x[:, :3] = rng.uniform(-1, 1, (8, 3))
    dy = rng.normal(size=(8, 144))
    y, cache = mlp.forward(w, x, bf=False)
    g = mlp.backward(w, cache, dy, bf=False)
    for idx in rng.choice(n_par, 40, replace=False):
        if 3 <= idx % 16 < 16 and idx < 256 * 16:
            continue   # padded input columns carry no gradient
        e = np.zeros(n_par)
        e[idx] = 1e-6
        fp = (mlp.forward(w + e, x, bf=False)[0] * dy).sum()
        fm = (mlp.forward(w - e, x, bf=False)[0] * dy).sum()
        assert abs((fp - fm) / 2e-6 - g[idx]) < 1e-6 * max(1.0, abs(g[idx]))
