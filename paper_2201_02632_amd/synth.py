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


# ---------------------------------------------------------------- particles --
# Light-cone particles for particle-based pasting.  The generator places
# particles with its own rough distance-redshift relation (trapezoidal
# integration of a flat LCDM H(z)); the method itself recomputes every
# distance from the particle redshift, so these approximations only shape the
# synthetic input.
_C_KMS = 299792.458


def _chi_table(om=0.3, zmax=5.0, n=20001):
    z = np.linspace(0.0, zmax, n)
    f = 1.0 / np.sqrt(om * (1 + z) ** 3 + 1 - om)
    chi = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(z))]) * _C_KMS / 100.0
    return z, chi


def _nfw_inverse_cdf(u, c, iters=60):
    """x with m(x)/m(c) = u (bisection), m(x) = ln(1+x) - x/(1+x)."""
    m = lambda x: np.log1p(x) - x / (1 + x)  # noqa: E731
    target = u * m(c)
    lo = np.zeros_like(u)
    hi = np.array(c, dtype=np.float64) * np.ones_like(u)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        big = m(mid) > target
        hi = np.where(big, mid, hi)
        lo = np.where(big, lo, mid)
    return 0.5 * (lo + hi)


def _random_rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)


def pp_lightcone(n_halos, n_halo_particles, n_field, field_deg, zr=(0.05, 1.5), logM=(12.5, 15.5),
                 mass_function="powerlaw", field_cell=2.0, om=0.3, seed=3):
    """Halo catalogue plus particles for particle-based pasting.

    Halo particles: N_h proportional to M_vir (one particle mass M_p for all);
    ellipsoidal radius drawn from the NFW enclosed-mass profile inside an
    approximate virial radius, direction isotropic scaled by volume-preserving
    axis ratios b/a, c/a ~ U[0.5, 1], random orientation; velocity = halo bulk
    N(0, 300) + internal N(0, sigma) with sigma = sqrt(G M / (2 r_vir)).
    Field particles: lognormal density on a comoving grid of ``field_cell``
    Mpc/h (sigma_ln rho = 1, white), Poisson counts, uniform within cells,
    velocities N(0, 300).

    Returns (halos, particles, M_p); particles are float32 except halo_id (int32).
    """
    rng = np.random.default_rng(seed)
    side = field_deg * DEG
    M = _masses(rng, n_halos, logM[0], logM[1], mass_function)
    zh = rng.uniform(zr[0], zr[1], size=n_halos)
    c = _concentration(rng, M, zh)
    halos = dict(M=M, c=c, z=zh, theta_x=rng.uniform(0, side, n_halos), theta_y=rng.uniform(0, side, n_halos),
                 v_los=rng.normal(0.0, 300.0, n_halos))
    M_p = float(M.sum() / max(n_halo_particles, 1))
    Nh = np.floor(M / M_p + rng.uniform(size=n_halos)).astype(np.int64)
    hid = np.repeat(np.arange(n_halos, dtype=np.int32), Nh)
    zt, chit = _chi_table(om)
    # generator-side halo size: 200 rho_crit(z) overdensity (input shaping only)
    E2 = om * (1 + zh) ** 3 + 1 - om
    rho_c = 2.775e11 * E2
    rv = (3 * M / (4 * np.pi * 200 * rho_c)) ** (1.0 / 3.0)
    chih = np.interp(zh, zt, chit)
    DA = chih / (1 + zh)
    x = _nfw_inverse_cdf(rng.uniform(size=hid.size), c[hid])
    r_e = x * (rv / c)[hid]
    q = np.sort(rng.uniform(0.5, 1.0, size=(n_halos, 2)), axis=1)[:, ::-1]      # b/a >= c/a
    axes = np.stack([np.ones(n_halos), q[:, 0], q[:, 1]], 1) / np.cbrt(q[:, 0] * q[:, 1])[:, None]
    rot = _random_rotations(rng, n_halos)
    nvec = rng.normal(size=(hid.size, 3))
    nvec /= np.linalg.norm(nvec, axis=1, keepdims=True)
    off = np.einsum("nij,nj->ni", rot[hid], nvec * axes[hid]) * r_e[:, None]    # physical Mpc/h
    tx = halos["theta_x"][hid] + off[:, 0] / DA[hid]
    ty = halos["theta_y"][hid] + off[:, 1] / DA[hid]
    dchi = off[:, 2] * (1 + zh[hid])
    zp = np.interp(chih[hid] + dchi, chit, zt)
    sig = np.sqrt(4.30091e-9 * M / (2 * rv))
    v = halos["v_los"][hid] + rng.normal(size=hid.size) * sig[hid]
    parts = [dict(theta_x=tx, theta_y=ty, z=zp, v_los=v, halo_id=hid, r_i=r_e)]
    if n_field > 0:
        chi0, chi1 = np.interp(zr, zt, chit)
        nx = int(np.ceil(side * chi1 / field_cell))
        nz = int(np.ceil((chi1 - chi0) / field_cell))
        lam = None
        fx, fy, fz = [], [], []
        # expected counts proportional to exp(g - 1/2) on cells whose centre lies in the cone
        ix = np.arange(nx)
        for kz in range(nz):
            zc = chi0 + (kz + 0.5) * field_cell
            g = rng.normal(size=(nx, nx))
            xc = (ix + 0.5) * field_cell
            inside = (xc[:, None] < side * zc) & (xc[None, :] < side * zc)
            w = np.exp(g - 0.5) * inside
            fx.append(w)
        W = np.stack(fx, 0)
        lam = n_field / W.sum()
        cnt = rng.poisson(lam * W)
        kz, kx, ky = np.nonzero(cnt)
        nn = cnt[kz, kx, ky]
        X = (np.repeat(kx, nn) + rng.uniform(size=nn.sum())) * field_cell
        Y = (np.repeat(ky, nn) + rng.uniform(size=nn.sum())) * field_cell
        Z = chi0 + (np.repeat(kz, nn) + rng.uniform(size=nn.sum())) * field_cell
        keep = (X < side * Z) & (Y < side * Z) & (Z < chi1)
        X, Y, Z = X[keep], Y[keep], Z[keep]
        nf = X.size
        parts.append(dict(theta_x=X / Z, theta_y=Y / Z, z=np.interp(Z, chit, zt), v_los=rng.normal(0, 300.0, nf),
                          halo_id=np.full(nf, -1, dtype=np.int32), r_i=np.zeros(nf)))
    P = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    out = {k: (v.astype(np.int32) if k == "halo_id" else v.astype(np.float32)) for k, v in P.items()}
    return halos, out, M_p


def pp_small(seed=3):
    """CPU-sized particle workload: 0.4x0.4 deg, 96^2 pixels, 60 halos, ~6000 halo and ~3000 field particles."""
    halos, parts, M_p = pp_lightcone(60, 6000, 3000, 0.4, zr=(0.05, 0.4), logM=(12.5, 14.5), field_cell=2.0,
                                     seed=seed)
    return halos, parts, M_p, 96, 0.4 * DEG / 96


def pp_large(seed=3, n_particles=200_000_000):
    """GPU-sized: 5x5 deg, 4096^2 pixels, z in [0.05,1.5]; 60% of the particles in 2e5 halos, 40% field."""
    halos, parts, M_p = pp_lightcone(200_000, int(0.6 * n_particles), int(0.4 * n_particles), 5.0,
                                     zr=(0.05, 1.5), seed=seed)
    return halos, parts, M_p, 4096, 5.0 * DEG / 4096


# ------------------------------------------------- device-side particle draws --
# The same light-cone recipe as ``pp_lightcone``, drawn with torch on the
# device so that 2e8-particle workloads take seconds instead of minutes.  The
# halo catalogue still comes from numpy (it is small); the particle draws use a
# seeded ``torch.Generator`` on the target device, so they differ from the
# numpy draws of ``pp_lightcone`` but are reproducible on the same device.
def _interp_t(x, xp, fp):
    """Linear interpolation on an increasing table (torch)."""
    import torch
    i = torch.clamp(torch.searchsorted(xp, x), 1, xp.numel() - 1)
    x0, x1 = xp[i - 1], xp[i]
    w = (x - x0) / (x1 - x0)
    return fp[i - 1] + w * (fp[i] - fp[i - 1])


def _nfw_inverse_cdf_t(u, c, iters=60):
    import torch
    m = lambda x: torch.log1p(x) - x / (1 + x)  # noqa: E731
    target = u * m(c)
    lo = torch.zeros_like(u)
    hi = c.clone()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        big = m(mid) > target
        hi = torch.where(big, mid, hi)
        lo = torch.where(big, lo, mid)
    return 0.5 * (lo + hi)


def pp_lightcone_device(n_halos, n_halo_particles, n_field, field_deg, zr=(0.05, 1.5), logM=(12.5, 15.5),
                        mass_function="powerlaw", field_cell=2.0, om=0.3, seed=3, device="cuda", chunk=1 << 24):
    """``pp_lightcone`` with the particles drawn on ``device``.  Returns (halos as numpy float64,
    particles as device tensors: float32 theta_x, theta_y, z, v_los, r_i and int32 halo_id, M_p)."""
    import torch
    rng = np.random.default_rng(seed)
    side = field_deg * DEG
    M = _masses(rng, n_halos, logM[0], logM[1], mass_function)
    zh = rng.uniform(zr[0], zr[1], size=n_halos)
    c = _concentration(rng, M, zh)
    halos = dict(M=M, c=c, z=zh, theta_x=rng.uniform(0, side, n_halos), theta_y=rng.uniform(0, side, n_halos),
                 v_los=rng.normal(0.0, 300.0, n_halos))
    M_p = float(M.sum() / max(n_halo_particles, 1))
    Nh = np.floor(M / M_p + rng.uniform(size=n_halos)).astype(np.int64)
    zt, chit = _chi_table(om)
    E2 = om * (1 + zh) ** 3 + 1 - om
    rv = (3 * M / (4 * np.pi * 200 * 2.775e11 * E2)) ** (1.0 / 3.0)
    chih = np.interp(zh, zt, chit)
    DA = chih / (1 + zh)
    q = np.sort(rng.uniform(0.5, 1.0, size=(n_halos, 2)), axis=1)[:, ::-1]
    axes = np.stack([np.ones(n_halos), q[:, 0], q[:, 1]], 1) / np.cbrt(q[:, 0] * q[:, 1])[:, None]
    rot = _random_rotations(rng, n_halos)
    sig = np.sqrt(4.30091e-9 * M / (2 * rv))
    f64 = dict(dtype=torch.float64, device=device)
    T = {k: torch.as_tensor(np.ascontiguousarray(v), **f64) for k, v in
         dict(c=c, rs=rv / c, DA=DA, chih=chih, zh=zh, tx=halos["theta_x"], ty=halos["theta_y"], v=halos["v_los"],
              sig=sig, axes=axes, rot=rot).items()}
    zt_t, chit_t = torch.as_tensor(zt, **f64), torch.as_tensor(chit, **f64)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    hid_all = torch.repeat_interleave(torch.arange(n_halos, device=device, dtype=torch.int64),
                                      torch.as_tensor(Nh, device=device))
    nh_tot = hid_all.numel()
    out = {k: [] for k in ("theta_x", "theta_y", "z", "v_los", "halo_id", "r_i")}
    for s0 in range(0, nh_tot, chunk):
        hid = hid_all[s0:s0 + chunk]
        n = hid.numel()
        x = _nfw_inverse_cdf_t(torch.rand(n, generator=g, **f64), T["c"][hid])
        r_e = x * T["rs"][hid]
        nvec = torch.randn((n, 3), generator=g, **f64)
        nvec /= torch.linalg.norm(nvec, dim=1, keepdim=True)
        off = torch.bmm(T["rot"][hid], (nvec * T["axes"][hid]).unsqueeze(-1)).squeeze(-1) * r_e[:, None]
        out["theta_x"].append((T["tx"][hid] + off[:, 0] / T["DA"][hid]).float())
        out["theta_y"].append((T["ty"][hid] + off[:, 1] / T["DA"][hid]).float())
        dchi = off[:, 2] * (1 + T["zh"][hid])
        out["z"].append(_interp_t(T["chih"][hid] + dchi, chit_t, zt_t).float())
        out["v_los"].append((T["v"][hid] + torch.randn(n, generator=g, **f64) * T["sig"][hid]).float())
        out["halo_id"].append(hid.to(torch.int32))
        out["r_i"].append(r_e.float())
        del x, r_e, nvec, off, dchi
    if n_field > 0:
        chi0, chi1 = np.interp(zr, zt, chit)
        nx = int(np.ceil(side * chi1 / field_cell))
        nz = int(np.ceil((chi1 - chi0) / field_cell))
        zc = chi0 + (torch.arange(nz, **f64) + 0.5) * field_cell
        xc = (torch.arange(nx, **f64) + 0.5) * field_cell
        inside = (xc[None, :, None] < side * zc[:, None, None]) & (xc[None, None, :] < side * zc[:, None, None])
        W = torch.exp(torch.randn((nz, nx, nx), generator=g, **f64) - 0.5) * inside
        cnt = torch.poisson(W * (n_field / W.sum()), generator=g).to(torch.int64)
        del W, inside
        idx = torch.nonzero(cnt.reshape(-1)).squeeze(1)
        nn = cnt.reshape(-1)[idx]
        cell = torch.repeat_interleave(idx, nn)
        del cnt, idx, nn
        kz, rem = cell // (nx * nx), cell % (nx * nx)
        kx, ky = rem // nx, rem % nx
        nf = cell.numel()
        X = (kx.to(torch.float64) + torch.rand(nf, generator=g, **f64)) * field_cell
        Y = (ky.to(torch.float64) + torch.rand(nf, generator=g, **f64)) * field_cell
        Z = chi0 + (kz.to(torch.float64) + torch.rand(nf, generator=g, **f64)) * field_cell
        del cell, kz, rem, kx, ky
        keep = (X < side * Z) & (Y < side * Z) & (Z < chi1)
        X, Y, Z = X[keep], Y[keep], Z[keep]
        nf = X.numel()
        out["theta_x"].append((X / Z).float())
        out["theta_y"].append((Y / Z).float())
        out["z"].append(_interp_t(Z, chit_t, zt_t).float())
        out["v_los"].append((torch.randn(nf, generator=g, **f64) * 300.0).float())
        out["halo_id"].append(torch.full((nf,), -1, dtype=torch.int32, device=device))
        out["r_i"].append(torch.zeros(nf, dtype=torch.float32, device=device))
    parts = {k: torch.cat(v).contiguous() for k, v in out.items()}
    return halos, parts, M_p


def pp_large_device(seed=3, n_particles=200_000_000, device="cuda"):
    """``pp_large`` drawn on the device: 5x5 deg, 4096^2 pixels, 60% of the particles in 2e5 halos."""
    halos, parts, M_p = pp_lightcone_device(200_000, int(0.6 * n_particles), int(0.4 * n_particles), 5.0,
                                            zr=(0.05, 1.5), seed=seed, device=device)
    return halos, parts, M_p, 4096, 5.0 * DEG / 4096


# ------------------------------------------------- all-sky continuous light cone --
# Stand-in for the continuous light-cone output of App. A (all sky to z = 3.741, a 1 Gpc/h box of
# 512^3 particles replicated around the observer; particles recorded where they cross the past
# light cone).  Positions are uniform in comoving volume inside chi(z_max), a fraction of them in
# Gaussian clumps; the particle mass is that of the 512^3-in-(1 Gpc/h)^3 run.
ALLSKY_ZMAX = 3.741
ALLSKY_MP = 0.3 * 2.775e11 * 1000.0 ** 3 / 512 ** 3          # Omega_m rho_crit0 V / N  [Msun/h]
_PI_BELOW_F32 = float(np.nextafter(np.float32(np.pi), np.float32(0.0)))


def allsky_lightcone_device(n, zmax=ALLSKY_ZMAX, clustered=0.5, per_clump=1000, clump_sigma=1.0, v_sigma=300.0,
                            om=0.3, seed=7, device="cuda", chunk=1 << 25):
    """``n`` particles of an all-sky light cone to ``zmax``: float32 device tensors theta (colatitude,
    at most the float just below pi), phi in (-pi, pi], z and v_los [km/s].  A fraction ``clustered``
    sits in clumps of ``per_clump`` particles (isotropic Gaussian, comoving sigma ``clump_sigma``
    Mpc/h) whose centres are uniform in volume; the rest is uniform in volume.  Velocities are
    N(0, v_sigma) per particle plus an N(0, v_sigma) bulk shared by a clump.  Particle order is
    clump members first, then the uniform part, both in draw order."""
    import torch
    zt, chit = _chi_table(om, zmax=max(5.0, zmax + 1.0))
    f64 = dict(dtype=torch.float64, device=device)
    zt_t, chit_t = torch.as_tensor(zt, **f64), torch.as_tensor(chit, **f64)
    chi_max = float(np.interp(zmax, zt, chit))
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n_cl = int(round(clustered * n))
    n_clumps = max(1, -(-n_cl // per_clump)) if n_cl else 0

    def ball(m):
        r = chi_max * torch.rand(m, generator=g, **f64) ** (1.0 / 3.0)
        u = torch.randn((m, 3), generator=g, **f64)
        return u / torch.linalg.norm(u, dim=1, keepdim=True) * r[:, None]

    centres = ball(n_clumps) if n_clumps else None
    bulk = torch.randn(n_clumps, generator=g, **f64) * v_sigma if n_clumps else None
    out = {k: [] for k in ("theta", "phi", "z", "v_los")}
    for s0 in range(0, n, chunk):
        m = min(chunk, n - s0)
        v = torch.randn(m, generator=g, **f64) * v_sigma
        ncl = max(0, min(m, n_cl - s0))
        X = torch.empty((m, 3), **f64)
        if ncl:
            cid = torch.arange(s0, s0 + ncl, device=device) // per_clump
            X[:ncl] = centres[cid] + torch.randn((ncl, 3), generator=g, **f64) * clump_sigma
            v[:ncl] += bulk[cid]
        if m > ncl:
            X[ncl:] = ball(m - ncl)
        r = torch.linalg.norm(X, dim=1).clamp_min(1e-9)
        out["theta"].append(torch.acos((X[:, 2] / r).clamp(-1.0, 1.0)).float().clamp(0.0, _PI_BELOW_F32))
        out["phi"].append(torch.atan2(X[:, 1], X[:, 0]).float())
        out["z"].append(_interp_t(r, chit_t, zt_t).float())
        out["v_los"].append(v.float())
        del X, r, v
    return {k: torch.cat(v).contiguous() for k, v in out.items()}
