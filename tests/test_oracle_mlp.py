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


def test_adam_first_step_is_signed_learning_rate():
    # from zero moments the bias-corrected first step is lr g / (|g| + eps): a step of lr against the gradient
    from oracle import mlp
    g = np.array([3.0, -1e-3, 0.0, 2e5])
    w1, m1, v1 = mlp.adam(np.ones(4), np.zeros(4), np.zeros(4), g, 1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(w1, 1.0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=0)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15) and np.allclose(v1, 0.001 * g * g, rtol=1e-15)


def test_adam_constant_gradient_keeps_unit_steps():
    # with a constant gradient the corrected moments are exactly g and g^2 at every step t
    from oracle import mlp
    g = np.array([0.5, -2.0])
    w, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 50):
        w_prev = w
        w, m, v = mlp.adam(w, m, v, g, 1e-2, 0.9, 0.999, 0.0, t)
        assert np.allclose(w_prev - w, 1e-2 * np.sign(g), rtol=1e-12)


def test_weighted_mse_matches_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(3)
    n = 5
    y = rng.normal(size=(n, mlp.OUT))
    t = rng.normal(size=(n, mlp.OUT))
    mean, std = rng.normal(size=mlp.OUT), rng.uniform(0.5, 2, mlp.OUT)
    t[2, 7] = np.nan                                   # this row is left out
    dy, rows = mlp.weighted_mse(y, t, mean, std)
    ok = np.arange(n) != 2

    def loss(yy):
        _, r = mlp.weighted_mse(yy, t, mean, std)
        return np.nansum(r) / (n * (2 * 64 + 3 * mlp.AUX_WEIGHT))
    for (i, c) in ((0, 0), (1, 64), (3, 128), (4, 130), (0, 131), (2, 5)):
        e = np.zeros_like(y)
        e[i, c] = 1e-6
        fd = (loss(y + e) - loss(y - e)) / 2e-6
        assert abs(fd - dy[i, c]) < 1e-9, (i, c, fd, dy[i, c])
    assert np.all(dy[:, mlp.NOUT:] == 0) and np.all(dy[2] == 0)
    assert np.isnan(rows[2]) and np.all(np.isfinite(rows[ok]))
    # the scalar outputs weigh AUX_WEIGHT times a table entry
    assert abs(dy[0, 128] / (y[0, 128] - (t[0, 128] - mean[128]) / std[128]) /
               (dy[0, 0] / (y[0, 0] - (t[0, 0] - mean[0]) / std[0])) - mlp.AUX_WEIGHT) < 1e-12
