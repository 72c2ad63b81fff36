"""Flat-sky angular power spectrum of a square map (Sec. 5.3, power spectra) -- CPU oracle.

TEST INFRASTRUCTURE ONLY: the plain FP64 reference the HIP estimator is checked against.  Only
tests/, the smoke check and the benchmark's CPU-baseline leg use it; it shares no code with the
HIP library.

Definition (the paper measures flat-sky spectra with an FFT in 30 logarithmic bins over
10^2 < ell < 10^5 and gives no more detail; the readings are the standard flat-sky estimator):
  * the map f(x) has N x N pixels of side d (rad), L = N d, area A = L^2;
  * Fourier coefficients  F(ell) = d^2 sum_x f(x) exp(-i ell.x)  on the modes
    ell = 2 pi (kx, ky) / L, kx, ky in [-N/2, N/2) (every mode of the discrete transform);
  * per-mode power  C(ell) = |F(ell)|^2 / A  = d^2 |DFT|^2 / N^2;
  * bin b holds the modes with e_b <= |ell| < e_{b+1}; the edges are given in ell.  The decision
    is taken on the integer |k|^2 = kx^2 + ky^2 against t_b = (e_b N d / (2 pi))^2 in FP64, so the
    GPU, which takes it the same way, puts every mode in the same bin;
  * C_b = mean of C over the bin's modes, ell_b = mean |ell| over them, n_b = their number.
No mean subtraction, apodisation or window deconvolution (the lowest bin starts above the
fundamental 2 pi / L for the paper's 5 x 5 deg maps).
"""
from __future__ import annotations

import math

import numpy as np


def log_edges(nbins=30, lmin=1e2, lmax=1e5):
    """nbins + 1 logarithmically equal bin edges in ell."""
    return np.logspace(math.log10(lmin), math.log10(lmax), nbins + 1)


def thresholds(edges, npix, pix_rad):
    """t_b = (e_b N d / (2 pi))^2: the |k|^2 at each bin edge."""
    e = np.asarray(edges, dtype=np.float64)
    t = e * float(npix) * float(pix_rad) / (2.0 * math.pi)
    return t * t


def flat_power_spectrum(m, pix_rad, edges):
    """(ell_b, C_b, n_b) of the square map m (any float dtype, promoted to FP64)."""
    f = np.asarray(m, dtype=np.float64)
    n = f.shape[0]
    assert f.shape == (n, n)
    F = np.fft.fft2(f) * pix_rad ** 2                         # library FFT as the transform step
    area = (n * pix_rad) ** 2
    P = (F.real ** 2 + F.imag ** 2) / area
    k = np.fft.fftfreq(n) * n                                 # integers in [-N/2, N/2)
    k2 = (k[:, None] ** 2 + k[None, :] ** 2)
    ell = 2.0 * math.pi / (n * pix_rad) * np.sqrt(k2)
    t = thresholds(edges, n, pix_rad)
    nb = len(edges) - 1
    cl = np.zeros(nb)
    lb = np.zeros(nb)
    cnt = np.zeros(nb, dtype=np.int64)
    for b in range(nb):
        sel = (k2 >= t[b]) & (k2 < t[b + 1])
        cnt[b] = int(sel.sum())
        if cnt[b]:
            cl[b] = P[sel].sum() / cnt[b]
            lb[b] = ell[sel].sum() / cnt[b]
    return lb, cl, cnt
