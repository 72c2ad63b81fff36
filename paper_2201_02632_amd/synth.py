"""Seeded synthetic inputs shaped like the paper's workloads.

The paper pastes gas onto halo catalogues and particle light cones from its
N-body runs (Sec. 3.1); those data are not available, so these generators
stand in for them with the sizes and distributions of the benchmark
workloads.  This module holds NO arithmetic of the pasting method: it only
draws inputs (halo masses, concentrations, redshifts, positions, velocities,
particle positions).  It is the one module both the HIP path and the CPU
oracle consume.

All generators use ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math

import numpy as np

DEG = math.pi / 180.0


def _concentration(rng, M, z, scatter_dex=0.1):
    """c = 5 (M/1e14)^-0.1 (1+z)^-0.5 with lognormal scatter (the workload recipe;
    the paper's own c-M fit is not printed)."""
    c = 5.0 * (M / 1e14) ** -0.1 * (1.0 + z) ** -0.5
    return c * 10.0 ** rng.normal(0.0, scatter_dex, size=M.shape)


def _masses(rng, n, logM_lo, logM_hi, mass_function):
    if mass_function == "uniform":          # log10 M uniform
        return 10.0 ** rng.uniform(logM_lo, logM_hi, size=n)
    if mass_function == "powerlaw":          # dN/dlnM ~ M^-0.9, inverse CDF
        lo, hi = 10.0 ** logM_lo, 10.0 ** logM_hi
        u = rng.uniform(size=n)
        a = 0.9
        return (lo ** -a - u * (lo ** -a - hi ** -a)) ** (-1.0 / a)
    raise ValueError(mass_function)


def flat_catalogue(n, field_deg, logM=(13.0, 15.0), zr=(0.1, 1.0), mass_function="uniform",
                   v_sigma=300.0, seed=1):
    """Halo catalogue in a flat square field of side ``field_deg`` degrees.

    Returns float64 arrays: M [Msun/h], c, z, theta_x, theta_y [rad], v_los [km/s].
    """
    rng = np.random.default_rng(seed)
    M = _masses(rng, n, logM[0], logM[1], mass_function)
    z = rng.uniform(zr[0], zr[1], size=n)
    c = _concentration(rng, M, z)
    side = field_deg * DEG
    tx = rng.uniform(0.0, side, size=n)
    ty = rng.uniform(0.0, side, size=n)
    v = rng.normal(0.0, v_sigma, size=n)
    return dict(M=M, c=c, z=z, theta_x=tx, theta_y=ty, v_los=v)


def sky_catalogue(n, logM=(12.5, 15.5), zr=(0.01, 3.0), mass_function="powerlaw", v_sigma=300.0,
                  seed=5):
    """Halos isotropic on the sphere: theta (colatitude), phi [rad]."""
    rng = np.random.default_rng(seed)
    M = _masses(rng, n, logM[0], logM[1], mass_function)
    z = rng.uniform(zr[0], zr[1], size=n)
    c = _concentration(rng, M, z)
    cth = rng.uniform(-1.0, 1.0, size=n)
    th = np.arccos(cth)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n)
    v = rng.normal(0.0, v_sigma, size=n)
    return dict(M=M, c=c, z=z, theta=th, phi=ph, v_los=v)


# ------------------------------------------------------------------ presets --
def hp_flat_small(seed=1):
    """HP flat-sky, CPU-sized: 1x1 deg, 128^2 pixels, 2,000 halos, log10 M in [13,15]."""
    cat = flat_catalogue(2000, 1.0, logM=(13.0, 15.0), zr=(0.1, 1.0), mass_function="uniform", seed=seed)
    return cat, 128, 1.0 * DEG / 128


def hp_flat_large(n=500_000, seed=2):
    """HP flat-sky, GPU-sized: 5x5 deg, 4096^2 pixels, 5e5 halos, dN/dlnM ~ M^-0.9 on [12.5,15.5]."""
    cat = flat_catalogue(n, 5.0, logM=(12.5, 15.5), zr=(0.1, 1.0), mass_function="powerlaw", seed=seed)
    return cat, 4096, 5.0 * DEG / 4096


def surrogate_training(n, seed=4):
    """(M, c, z) samples over log10 M in [12.5,15.5], c in [2,15] (log-uniform), z in [0.05,3]."""
    rng = np.random.default_rng(seed)
    M = 10.0 ** rng.uniform(12.5, 15.5, size=n)
    c = np.exp(rng.uniform(math.log(2.0), math.log(15.0), size=n))
    z = rng.uniform(0.05, 3.0, size=n)
    return dict(M=M, c=c, z=z)


def subsample(cat, idx):
    return {k: np.asarray(v)[idx] for k, v in cat.items()}
