"""FP64 reference of the profile-table surrogate network (TEST INFRASTRUCTURE ONLY).

Follows the algorithm documented with the library's network entry points:
FP32-style first layer, hidden activations and the weights of layers 2-4 and
the backpropagated errors rounded to bfloat16 (round to nearest even) exactly
where the documented algorithm rounds them, everything else in FP64.  The
network itself is an addition to the paper's method (no paper passage defines
it); its pins are the finite-difference check below and the closed-form
derivative of SiLU.
"""
from __future__ import annotations

import numpy as np

HID, IN, OUT, NIN, NOUT = 256, 16, 144, 3, 131


def bf16(a):
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    f = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((f + 0x7FFF + ((f >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    out = {}
    for name, shape in (("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
                        ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (OUT, HID)), ("b4", (OUT,))):
        n = int(np.prod(shape))
        out[name] = w[o:o + n].reshape(shape)
        o += n
    assert o == w.size
    return out


def forward(w, x, bf=True):
    P = unpack(w)
    r = bf16 if bf else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(x, np.float64)
    z1 = x[:, :NIN] @ P["W1"][:, :NIN].T + P["b1"]
    h1 = r(silu(z1))
    z2 = h1 @ r(P["W2"]).T + P["b2"]
    h2 = r(silu(z2))
    z3 = h2 @ r(P["W3"]).T + P["b3"]
    h3 = r(silu(z3))
    y = h3 @ r(P["W4"]).T + P["b4"]
    return y, dict(x=x, z1=z1, z2=z2, z3=z3, h1=h1, h2=h2, h3=h3)


def backward(w, cache, dy, bf=True):
    """Gradient of sum(dy * y) with respect to the flat parameter vector."""
    P = unpack(w)
    r = bf16 if bf else (lambda a: np.asarray(a, np.float64))
    g = {}
    dy = np.asarray(dy, np.float64)
    g4 = r(dy)
    g["W4"] = g4.T @ cache["h3"]
    g["b4"] = dy.sum(0)
    d3 = (g4 @ r(P["W4"])) * dsilu(cache["z3"])
    g["b3"] = d3.sum(0)
    g3 = r(d3)
    g["W3"] = g3.T @ cache["h2"]
    d2 = (g3 @ r(P["W3"])) * dsilu(cache["z2"])
    g["b2"] = d2.sum(0)
    g2 = r(d2)
    g["W2"] = g2.T @ cache["h1"]
    d1 = (g2 @ r(P["W2"])) * dsilu(cache["z1"])
    g["b1"] = d1.sum(0)
    W1 = np.zeros((HID, IN))
    W1[:, :NIN] = d1.T @ cache["x"][:, :NIN]
    g["W1"] = W1
    return np.concatenate([g[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])


def adam(w, m, v, g, lr, beta1, beta2, eps, t):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) in FP64 from the given state:
    m <- beta1 m + (1 - beta1) g;  v <- beta2 v + (1 - beta2) g^2;
    w <- w - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).  Returns (w, m, v)."""
    w, m, v, g = (np.asarray(a, np.float64) for a in (w, m, v, g))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


AUX_WEIGHT = 16.0


def weighted_mse(y, t, mean, std):
    """Training loss of the surrogate over the NOUT used outputs: residual r_c = y_c - (t_c - mean_c)/std_c,
    weight 1 for the 2x64 table entries and AUX_WEIGHT for each of the three scalars (ln x_f and the two
    amplitude ratios, which scale a whole footprint).  L = sum_i sum_c w_c r_c^2 / (n sum_c w_c).
    Returns (dL/dy [n, OUT], per-row sum_c w_c r_c^2 [n]); a row with a non-finite target contributes
    nothing (zero gradient), its row sum is not defined and is returned as NaN."""
    y, t = np.asarray(y, np.float64), np.asarray(t, np.float64)
    mean, std = np.asarray(mean, np.float64), np.asarray(std, np.float64)
    n = y.shape[0]
    wc = np.zeros(OUT)
    wc[:NOUT] = 1.0
    wc[NOUT - 3:NOUT] = AUX_WEIGHT
    r = np.zeros_like(y)
    r[:, :NOUT] = y[:, :NOUT] - (t[:, :NOUT] - mean[:NOUT]) / std[:NOUT]
    ok = np.all(np.isfinite(t[:, :NOUT]), axis=1)
    dy = np.where(ok[:, None], 2.0 * wc * r / (n * wc.sum()), 0.0)
    rows = np.where(ok, (wc * r * r).sum(1), np.nan)
    return dy, rows
