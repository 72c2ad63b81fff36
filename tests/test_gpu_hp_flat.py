"""GPU parity of the exact HP flat path (K1 solve, K2 tables, K3 paste) against the oracle."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hp_flat_small_oracle.npz")


@pytest.fixture(scope="module")
def bp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_02632_amd as bp
    return bp


def T(a, dt="f64"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64 if dt == "f64" else torch.float32,
                           device="cuda")


def rel_err(g, o, scale=None):
    """pixel-wise max relative error with a floor of 1e-6 of the map's peak |value|.

    For the signed kSZ map, ``scale`` is the per-pixel sum of |contributions|
    (the oracle map with |v|): where halos of opposite velocity cancel, the
    attainable accuracy is relative to that sum, not to the net value."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    ref = np.abs(o) if scale is None else np.asarray(scale, dtype=np.float64)
    floor = 1e-6 * ref.max() if ref.max() > 0 else 1e-300
    return float(np.max(np.abs(g - o) / (ref + floor)))


def oracle_flat_with_abs(orc, cat, npix, pix):
    p = orc.default_params()
    yo, bo, halos = orc.hp_flat(p, cat, npix, pix)
    _, babs = orc.hp_flat_solved(p, halos, dict(cat, v_los=np.abs(np.asarray(cat["v_los"], float))), npix, pix)
    return yo, bo, babs


def solve_gpu(bp, params, M, c, z):
    import torch
    sol, st = bp.icm_solve(params, T(M), T(c), T(z))
    torch.cuda.synchronize()
    return sol.cpu().numpy(), st.cpu().numpy()


def test_icm_solve_parity(bp, orc):
    rng = np.random.default_rng(101)
    n = 160
    M = 10 ** rng.uniform(12.5, 15.5, n)
    c = np.exp(rng.uniform(math.log(1.5), math.log(25.0), n))
    z = rng.uniform(0.01, 3.5, n)
    # domain corners and a thin-shell halo (x_f close to 1)
    M = np.r_[M, 10 ** 12.5, 10 ** 15.5, 10 ** 15.5, 10 ** 15.5, 3.16e15]
    c = np.r_[c, 15.0, 2.0, 15.0, 4.0, 15.0]
    z = np.r_[z, 3.0, 0.05, 0.05, 1.0, 0.05]
    print(f"icm parity: {len(M)} halos", flush=True)
    sol, st = solve_gpu(bp, bp.default_params(), M, c, z)
    halos = orc.solve_halos(orc.default_params(), M, c, z)
    tab = orc.halos_table(halos)
    assert np.array_equal(st, tab["status"].astype(np.int32))
    ok = st == 0
    S = bp.SOL
    pairs = [("RVIR", "r_vir", 1e-13), ("R500", "r500", 1e-11), ("M500", "M500", 1e-11), ("MSTAR", "M_star", 1e-11),
             ("XSTAR", "x_star", 1e-10), ("PS", "P_s", 1e-8), ("EGI", "E_gi", 1e-8), ("XF", "x_f", 1e-8),
             ("A", "a", 1e-8), ("RHO0", "rho0", 1e-8), ("P0", "P0", 1e-8), ("RF", "r_f", 1e-8),
             ("DA", "D_A", 1e-12), ("CHI", "chi", 1e-12), ("TAU", "tau", 1e-12), ("FNT", "f_nt", 1e-13),
             ("RT", "R_t", 1e-8)]
    for gk, ok_key, tol in pairs:
        g = sol[S[gk]][ok]
        o = tab[ok_key][ok]
        err = np.max(np.abs(g / o - 1))
        assert err < tol, (gk, err)
    assert np.all(np.abs(sol[S["RES_E"]][ok]) < 1e-9)


def test_icm_bad_inputs(bp):
    M = np.array([1e14, -1.0, 1e14, np.nan, 1e14])
    c = np.array([5.0, 5.0, 0.0, 5.0, 5.0])
    z = np.array([0.5, 0.5, 0.5, 0.5, -0.1])
    sol, st = solve_gpu(bp, bp.default_params(), M, c, z)
    assert list(st) == [0, bp.S_BAD_INPUT, bp.S_BAD_INPUT, bp.S_BAD_INPUT, bp.S_BAD_INPUT]
    _, st2 = solve_gpu(bp, bp.default_params(f_star=0.5), M[:1], c[:1], z[:1])
    assert st2[0] == bp.S_NO_STAR_ROOT
    with pytest.raises(bp.BPError):
        bp.icm_solve(bp.default_params(Gamma=1.0), T(M), T(c), T(z))


def test_meta_profile_constants(bp):
    # the profile-shape constants the table kernels read from meta are the FP32 values of their
    # definitions from the solve's FP64 fields (computed once per halo in the set-up kernel)
    import torch
    params = bp.default_params()
    rng = np.random.default_rng(7)
    n = 3000
    M = 10 ** rng.uniform(12.5, 15.5, n)
    c = rng.uniform(2.0, 15.0, n)
    z = rng.uniform(0.05, 3.0, n)
    sol, st = bp.icm_solve(params, T(M), T(c), T(z))
    _, meta = bp.profile_tables(params, sol, st)
    torch.cuda.synchronize()
    S, m, st = sol.cpu().numpy(), meta.cpu().numpy(), st.cpu().numpy()
    ok = (st & ~bp.S_MULTI_ROOT) == 0
    assert ok.sum() > 0.9 * n
    F = lambda name: S[bp.SOL[name]][ok]
    cc = F("C")
    mc = np.log1p(cc) - cc / (1.0 + cc)
    expect = {"PR_RV": F("RVIR"), "PR_INV_RS": 1.0 / F("RS"), "PR_RF": F("RF"), "PR_CM": cc / mc,
              "PR_PHI_OUT0": cc * cc / ((1.0 + cc) * mc), "PR_A": F("A"), "PR_INV_R500": 1.0 / F("R500"),
              "PR_ANT_F": params.alpha_nt * F("FNT")}
    for name, v in expect.items():
        g = m[bp.META[name]][ok].astype(np.float64)
        # one FP32 rounding of the same FP64 value, up to the last bit of the FP64 expression
        assert np.all(np.abs(g - v) <= 1.2e-7 * np.abs(v)), name
    assert np.all(m[bp.META["PR_RV"]:, ~ok] == 0.0)


def test_tables_against_los(bp, orc):
    import torch
    params = bp.default_params()
    M = np.array([3.16e15, 1e14, 3e12, 1e13, 10 ** 15.5])
    c = np.array([4.0, 5.0, 8.0, 6.0, 15.0])
    z = np.array([1.0, 0.5, 0.1, 2.0, 0.05])
    tM, tc, tz = T(M), T(c), T(z)
    sol, st = bp.icm_solve(params, tM, tc, tz)
    tab, meta = bp.profile_tables(params, sol, st)
    torch.cuda.synchronize()
    tab, meta, sol = tab.cpu().numpy(), meta.cpu().numpy(), sol.cpu().numpy()
    p = orc.default_params()
    units = orc.MPC / p.h
    for i in range(len(M)):
        h = orc.solve_halo(p, M[i], c[i], z[i])
        Pe0 = meta[bp.META["PE0"], i]
        ne0 = meta[bp.META["NE0"], i]
        rv, rf, Rt = h.r_vir, h.r_f, h.R_t
        ra = min(rv, rf)
        checks = []
        # zone A: the whole sight line, Y = S g_T with S = sqrt(u^2 + D), D = r_f^2 - r_vir^2 for a gas shell
        lo, hi = meta[bp.META["ETA_LO"], i], meta[bp.META["ETA_HI"], i]
        D = rf * rf - rv * rv if rf > rv else 0.0
        for k in range(0, bp.TAB_NA, 7):
            xi = math.expm1(lo + (hi - lo) * k / (bp.TAB_NA - 1))
            rp = ra / math.cosh(xi)
            u = math.sqrt(max(ra * ra - rp * rp, 0))
            S = math.sqrt(u * u + D)
            checks.append((rp, tab[i, k] * S, tab[i, bp.TAB_ZONE + k] * S))
        if Rt > rv:    # zone B nodes
            lo, hi = meta[bp.META["ZE_LO"], i], meta[bp.META["ZE_HI"], i]
            for k in range(bp.TAB_NB):
                ze = lo + (hi - lo) * k / (bp.TAB_NB - 1)
                rp = rf / math.cosh(ze)
                U = math.sqrt(max(rf * rf - rp * rp, 0))
                j = bp.TAB_NA + bp.TAB_NS + k
                checks.append((rp, tab[i, j] * U, tab[i, bp.TAB_ZONE + j] * U))
        assert checks
        for rp, gy, gn in checks:
            if rp > ra * (1 - 1e-9) and rf <= rv or rp > rf * (1 - 1e-9):
                continue          # the edge node: value and oracle are both ~0
            ty, tb = orc.los(p, h, rp)
            yo = ty / (orc.SIGMA_T / orc.ME_C2) / units / Pe0
            no = tb / orc.SIGMA_T / units / ne0
            # a zone-A node of a halo with a shell carries the shell part interpolated from the 32-node zone S
            # (the interpolation the deposit applied per pixel before the fold): 4e-6; else 2e-6
            tol = 4e-6 if (rf > rv and rp < ra) else 2e-6
            assert abs(gy / yo - 1) < tol, (i, rp / rv, gy, yo)
            assert abs(gn / no - 1) < tol, (i, rp / rv, gn, no)


def test_hp_flat_small_full_map(bp, orc):
    """CPU-sized HP workload: full 128^2 map against the oracle."""
    import torch
    from paper_2201_02632_amd.synth import hp_flat_small
    if not os.path.exists(GOLD):
        pytest.skip("golden oracle map missing: run tests/golden/make_oracle_maps.py")
    g = np.load(GOLD)
    cat, npix, pix = hp_flat_small(1)
    print(f"hp flat small: {len(cat['M'])} halos, {npix}^2", flush=True)
    y, b, sol, st = bp.hp_flat_map(bp.default_params(), cat, npix, pix)
    torch.cuda.synchronize()
    y, b = y.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(st.cpu().numpy(), g["halo_status"].astype(np.int32))
    ey, eb = rel_err(y, g["y"]), rel_err(b, g["b"], g["b_abs"])
    Yerr = abs(y.astype(np.float64).sum() / g["y"].sum() - 1)
    print(f"max rel err y {ey:.2e} b {eb:.2e} integrated-Y err {Yerr:.2e}")
    assert ey < 1e-5 and eb < 1e-5
    assert Yerr < 1e-6


def test_sign_reversal_and_determinism(bp):
    import torch
    from paper_2201_02632_amd.synth import hp_flat_small
    cat, npix, pix = hp_flat_small(1)
    params = bp.default_params()
    y1, b1, _, _ = bp.hp_flat_map(params, cat, npix, pix)
    y2, b2, _, _ = bp.hp_flat_map(params, cat, npix, pix)
    cat_neg = dict(cat, v_los=-cat["v_los"])
    y3, b3, _, _ = bp.hp_flat_map(params, cat_neg, npix, pix)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(b1, b2)
    assert torch.equal(y3, y1) and torch.equal(b3, -b1)


def test_accumulation_and_batches(bp):
    import torch
    from paper_2201_02632_amd.synth import hp_flat_small
    cat, npix, pix = hp_flat_small(1)
    params = bp.default_params()
    yf, bf, _, _ = bp.hp_flat_map(params, cat, npix, pix)
    t = {k: T(v) for k, v in cat.items()}
    sol, st = bp.icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = bp.profile_tables(params, sol, st)
    y = torch.zeros_like(yf)
    b = torch.zeros_like(bf)
    n = len(cat["M"])
    for a, e in ((0, n // 3), (n // 3, n)):
        sl = {k: T(v[a:e]) for k, v in cat.items()}
        s2, st2 = bp.icm_solve(params, sl["M"], sl["c"], sl["z"])
        tb2, mt2 = bp.profile_tables(params, s2, st2)
        bp.hp_paste_flat(params, npix, pix, sl["theta_x"], sl["theta_y"], sl["v_los"], s2, st2, tb2, mt2, y, b)
    torch.cuda.synchronize()
    yb = bp.hp_flat_map(params, dict(cat, v_los=np.abs(cat["v_los"])), npix, pix)[1]
    assert rel_err(y.cpu().numpy(), yf.cpu().numpy()) < 1e-6
    assert rel_err(b.cpu().numpy(), bf.cpu().numpy(), yb.cpu().numpy()) < 1e-6


def test_edges_ragged_and_empty(bp, orc):
    """Map not a multiple of the tile, halos straddling the edges and off the map, n = 0."""
    import torch
    rng = np.random.default_rng(7)
    npix = 100
    pix = 0.4 * math.pi / 180 / npix
    n = 40
    M = 10 ** rng.uniform(13.0, 14.8, n)
    zz = rng.uniform(0.1, 0.8, n)
    cc = 5 * (M / 1e14) ** -0.1 * (1 + zz) ** -0.5
    side = npix * pix
    tx = rng.uniform(-0.3, 1.3, n) * side
    ty = rng.uniform(-0.3, 1.3, n) * side
    tx[:3] = [-5 * side, 0.0, side]           # far off, on the left edge, on the right edge
    ty[:3] = [0.5 * side, 0.5 * side, side]
    v = rng.normal(0, 300, n)
    cat = dict(M=M, c=cc, z=zz, theta_x=tx, theta_y=ty, v_los=v)
    print(f"edges: {n} halos on a {npix}^2 map", flush=True)
    y, b, _, _ = bp.hp_flat_map(bp.default_params(), cat, npix, pix)
    torch.cuda.synchronize()
    yo, bo, babs = oracle_flat_with_abs(orc, cat, npix, pix)
    assert rel_err(y.cpu().numpy(), yo) < 1e-5
    assert rel_err(b.cpu().numpy(), bo, babs) < 1e-5
    # n = 0 leaves the maps untouched
    params = bp.default_params()
    e = T(np.zeros(0))
    sol, st = bp.icm_solve(params, e, e, e)
    tab, meta = bp.profile_tables(params, sol, st)
    y0 = torch.full((16, 16), 3.0, device="cuda")
    b0 = torch.full((16, 16), -1.0, device="cuda")
    bp.hp_paste_flat(params, 16, pix, e, e, e, sol, st, tab, meta, y0, b0)
    torch.cuda.synchronize()
    assert torch.all(y0 == 3.0) and torch.all(b0 == -1.0)


def test_single_large_halo_covering_map(bp, orc):
    """One massive nearby halo whose footprint exceeds the whole map (many tiles, all pixels)."""
    import torch
    npix = 64
    pix = 2e-4
    cat = dict(M=[2e15], c=[5.0], z=[0.05], theta_x=[32.3 * pix], theta_y=[31.6 * pix], v_los=[500.0])
    y, b, _, _ = bp.hp_flat_map(bp.default_params(), {k: np.array(v, float) for k, v in cat.items()}, npix, pix)
    torch.cuda.synchronize()
    yo, bo, _ = orc.hp_flat(orc.default_params(), cat, npix, pix)
    assert np.all(yo > 0)
    assert rel_err(y.cpu().numpy(), yo) < 1e-5
    assert rel_err(b.cpu().numpy(), bo) < 1e-5


def test_ang2pix_bit_exact(bp, orc):
    import torch
    rng = np.random.default_rng(3)
    for nside in (1, 2, 7, 64, 1000, 8192):
        n = 20000
        th = np.arccos(rng.uniform(-1, 1, n))
        ph = rng.uniform(0, 2 * math.pi, n)
        # boundary cases: poles, cap/belt transition, phi multiples of pi/2, pixel centres
        special_th = np.r_[0.0, math.pi, math.acos(2 / 3), math.acos(-2 / 3), math.pi / 2, 1e-12]
        special_ph = np.r_[0.0, math.pi / 2, math.pi, 3 * math.pi / 2, 2 * math.pi - 1e-15, 7.0]
        th = np.r_[th, np.repeat(special_th, len(special_ph))]
        ph = np.r_[ph, np.tile(special_ph, len(special_th))]
        if nside <= 64:
            cth, cph = orc.pix2ang_ring(nside, np.arange(12 * nside * nside))
            th, ph = np.r_[th, cth], np.r_[ph, cph]
        got = bp.healpix_ang2pix_ring(nside, T(th), T(ph)).cpu().numpy()
        exp = orc.ang2pix_ring(nside, th, ph)
        assert np.array_equal(got, exp), nside
    with pytest.raises(bp.BPError):
        bp.healpix_ang2pix_ring(0, T(th), T(ph))


def _ulp_steps(x, k):
    """x moved by k units in the last place (k may be negative)."""
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    for _ in range(abs(k)):
        out = np.nextafter(out, np.inf if k > 0 else -np.inf)
    return out


def test_ang2pix_boundary_directions_nside_8192(bp, orc):
    """Directions within +-4 ulp of every boundary family of the RING scheme at N_side 8192 (Gorski et al.
    2005): the cap/belt transition |z| = 2/3; the ascending and descending pixel edges of the belt
    (N(1/2 + t) -+ (3/4) N z an integer, t = phi / (pi/2)); the edges of the polar caps (t' N sqrt(3(1 - |z|))
    an integer, t' = t mod 1), in colatitude and in longitude.  The integer results depend on the FP64 cos
    and sin of the colatitude on both sides, so this is where the device's and the host's libm would part."""
    import torch
    N = 8192
    rng = np.random.default_rng(11)
    th_b, ph_b = [], []
    m = 300
    # cap / belt transition
    tt = rng.uniform(0, 4, m)
    th_b += [np.full(m // 2, math.acos(2 / 3)), np.full(m - m // 2, math.acos(-2 / 3))]
    ph_b += [tt * math.pi / 2]
    # belt edges in colatitude: z = (N (1/2 + t) - k) / (3N/4) and z = (k - N (1/2 + t)) / (3N/4)
    tt = rng.uniform(0, 4, m)
    zb = (N * (0.5 + tt) - rng.integers(0, 5 * N, m)) / (0.75 * N)
    ok = np.abs(zb) < 2 / 3
    th_b.append(np.arccos(zb[ok])); ph_b.append(tt[ok] * math.pi / 2)
    tt = rng.uniform(0, 4, m)
    zb = (rng.integers(0, 5 * N, m) - N * (0.5 + tt)) / (0.75 * N)
    ok = np.abs(zb) < 2 / 3
    th_b.append(np.arccos(zb[ok])); ph_b.append(tt[ok] * math.pi / 2)
    # cap edges in colatitude: N sqrt(3 (1 - |z|)) t' = k  ->  |z| = 1 - (k / (N t'))^2 / 3
    tf = rng.uniform(0.01, 0.99, m)
    kk = rng.integers(1, N, m)
    za = 1 - (kk / (N * tf)) ** 2 / 3
    ok = za > 2 / 3
    north = rng.random(m) < 0.5
    thc = np.where(north, np.arccos(za.clip(-1, 1)), math.pi - np.arccos(za.clip(-1, 1)))
    th_b.append(thc[ok]); ph_b.append((rng.integers(0, 4, m) + tf)[ok] * math.pi / 2)
    # belt edges in longitude: t = (k + (3/4) N z) / N - 1/2, and cap edges in longitude: t = k / ring
    zr = rng.uniform(-2 / 3, 2 / 3, m)
    tb = ((rng.integers(0, 5 * N, m) + 0.75 * N * zr) / N - 0.5) % 4
    th_lon = [np.arccos(zr)]
    ph_lon = [tb * math.pi / 2]
    ring = rng.integers(1, N, m)
    zc = 1 - (ring / N) ** 2 / 3 - 1e-9
    th_lon.append(np.arccos(zc)); ph_lon.append((rng.integers(0, 4 * ring) / ring) * math.pi / 2)
    th_b, ph_b = np.concatenate(th_b), np.concatenate(ph_b)
    th_l, ph_l = np.concatenate(th_lon), np.concatenate(ph_lon)
    th = np.concatenate([_ulp_steps(th_b, k) for k in range(-4, 5)] + [np.tile(th_l, 9)])
    ph = np.concatenate([np.tile(ph_b, 9)] + [_ulp_steps(ph_l, k) for k in range(-4, 5)])
    keep = (th >= 0) & (th <= math.pi) & np.isfinite(ph)
    th, ph = th[keep], ph[keep]
    got = bp.healpix_ang2pix_ring(N, T(th), T(ph)).cpu().numpy()
    exp = orc.ang2pix_ring(N, th, ph)
    bad = np.nonzero(got != exp)[0]
    print(f"{len(th)} boundary directions at N_side {N}: {len(bad)} differ")
    for k in bad[:10]:
        print(f"  theta {th[k]!r} phi {ph[k]!r}: gpu {got[k]} oracle {exp[k]}")
    assert len(bad) == 0


def test_workspace_protocol(bp):
    import ctypes as C
    import torch
    params = bp.default_params()
    from paper_2201_02632_amd.synth import hp_flat_small
    cat, npix, pix = hp_flat_small(1)
    t = {k: T(v) for k, v in cat.items()}
    sol, st = bp.icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = bp.profile_tables(params, sol, st)
    y = torch.zeros((npix, npix), device="cuda")
    b = torch.zeros_like(y)
    need = C.c_size_t(0)
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    code = bp._lib.bp_hp_paste_flat(C.byref(params), npix, pix, len(cat["M"]), bp._ptr(t["theta_x"]),
                                    bp._ptr(t["theta_y"]), bp._ptr(t["v_los"]), bp._ptr(sol), bp._ptr(st),
                                    bp._ptr(tab), bp._ptr(meta), bp._ptr(y), bp._ptr(b), None, None, bp._ptr(small),
                                    256, C.byref(need), bp._stream())
    assert code == bp.BP_E_WORKSPACE and need.value > 256
    torch.cuda.synchronize()
    assert torch.all(y == 0)


def test_batches_with_compensation_equal_one_call(bp):
    """Maps accumulate over halo batches (Sec. 3.3): with the Kahan compensation maps carried between calls,
    consecutive batches of a catalogue add their halos to every tile in the same catalogue order and from
    the same compensated state as one call over the whole catalogue, so the maps agree bit for bit."""
    import torch
    from paper_2201_02632_amd.synth import hp_flat_small
    params = bp.default_params()
    cat, npix, pix = hp_flat_small(1)
    t = {k: T(v) for k, v in cat.items()}
    sol, st = bp.icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = bp.profile_tables(params, sol, st)
    y1 = torch.zeros((npix, npix), device="cuda")
    b1 = torch.zeros_like(y1)
    bp.hp_paste_flat(params, npix, pix, t["theta_x"], t["theta_y"], t["v_los"], sol, st, tab, meta, y1, b1)
    n = len(cat["M"])
    cuts = [0, 317, 1000, 1001, 1650, n]
    yb, bb, yc, bc = (torch.zeros_like(y1) for _ in range(4))
    yn, bn = torch.zeros_like(y1), torch.zeros_like(y1)
    for a, e in zip(cuts[:-1], cuts[1:]):
        sub = {k: v[a:e].contiguous() for k, v in t.items()}
        s2, st2 = bp.icm_solve(params, sub["M"], sub["c"], sub["z"])
        tb2, mt2 = bp.profile_tables(params, s2, st2)
        bp.hp_paste_flat(params, npix, pix, sub["theta_x"], sub["theta_y"], sub["v_los"], s2, st2, tb2, mt2, yb, bb,
                         comp=(yc, bc))
        bp.hp_paste_flat(params, npix, pix, sub["theta_x"], sub["theta_y"], sub["v_los"], s2, st2, tb2, mt2, yn, bn)
    torch.cuda.synchronize()
    assert torch.equal(yb, y1) and torch.equal(bb, b1)
    print(f"batches without compensation differ from one call at {(yn != y1).sum().item()} of {npix * npix} pixels")


def _three_calls(bp, params, t, npix, pix, comp=None):
    import torch
    sol, st = bp.icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = bp.profile_tables(params, sol, st)
    y = torch.zeros((npix, npix), device="cuda")
    b = torch.zeros_like(y)
    bp.hp_paste_flat(params, npix, pix, t["theta_x"], t["theta_y"], t["v_los"], sol, st, tab, meta, y, b, comp=comp)
    return sol, st, tab, meta, y, b


@pytest.mark.parametrize("n,field,npix,seed", [(2000, 1.0, 203, 3), (7000, 2.0, 480, 4)])
def test_pipeline_equals_three_calls(bp, n, field, npix, seed):
    """The one-call pipeline (solve, tables, paste with the paste's plan on a second stream) returns the same
    solution, tables and maps, bit for bit, as the three calls in sequence: twice in a row on one workspace
    (the second call smaller), on a non-default stream, with and without the compensation maps."""
    import torch
    from paper_2201_02632_amd.synth import flat_catalogue
    params = bp.default_params()
    pix = field * math.pi / 180 / npix
    ws = bp.Workspace("cuda")
    side = torch.cuda.Stream()
    for m in (n, n // 3 + 1):
        cat = flat_catalogue(m, field, seed=seed + m)
        t = {k: T(v) for k, v in cat.items()}
        ref = _three_calls(bp, params, t, npix, pix)
        with torch.cuda.stream(side):
            side.wait_stream(torch.cuda.default_stream())
            y = torch.zeros((npix, npix), device="cuda")
            b = torch.zeros_like(y)
            got = bp.hp_flat_pipeline(params, npix, pix, t["M"], t["c"], t["z"], t["theta_x"], t["theta_y"],
                                      t["v_los"], y, b, ws=ws)
        torch.cuda.synchronize()
        for name, r, g in zip(("sol", "status", "tables", "meta", "y", "b"), ref, (*got, y, b)):
            assert torch.equal(r, g), (m, name)
        assert (ref[4] != 0).sum().item() > 0
        yc, bc = torch.zeros_like(y), torch.zeros_like(y)
        refc = _three_calls(bp, params, t, npix, pix, comp=(yc, bc))
        y2, b2 = torch.zeros_like(y), torch.zeros_like(y)
        yc2, bc2 = torch.zeros_like(y), torch.zeros_like(y)
        bp.hp_flat_pipeline(params, npix, pix, t["M"], t["c"], t["z"], t["theta_x"], t["theta_y"], t["v_los"], y2, b2,
                            ws=ws, comp=(yc2, bc2))
        torch.cuda.synchronize()
        assert torch.equal(refc[4], y2) and torch.equal(refc[5], b2)
        assert torch.equal(yc, yc2) and torch.equal(bc, bc2)


def test_pipeline_workspace_protocol(bp):
    """Too small a workspace: BP_E_WORKSPACE with the size, the solve and tables complete, the maps untouched;
    bp_hp_paste_flat on the returned outputs then gives the three-call maps."""
    import ctypes as C
    import torch
    from paper_2201_02632_amd.synth import hp_flat_small
    params = bp.default_params()
    cat, npix, pix = hp_flat_small(1)
    t = {k: T(v) for k, v in cat.items()}
    ref = _three_calls(bp, params, t, npix, pix)
    n = len(cat["M"])
    sol = torch.empty_like(ref[0])
    st = torch.empty_like(ref[1])
    tab = torch.empty_like(ref[2])
    meta = torch.empty_like(ref[3])
    y = torch.zeros((npix, npix), device="cuda")
    b = torch.zeros_like(y)
    need = C.c_size_t(0)
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    code = bp._lib.bp_hp_flat_pipeline(C.byref(params), npix, pix, n, bp._ptr(t["M"]), bp._ptr(t["c"]),
                                       bp._ptr(t["z"]), bp._ptr(t["theta_x"]), bp._ptr(t["theta_y"]),
                                       bp._ptr(t["v_los"]), bp._ptr(sol), bp._ptr(st), bp._ptr(tab), bp._ptr(meta),
                                       bp._ptr(y), bp._ptr(b), None, None, bp._ptr(small), 256, C.byref(need),
                                       bp._stream())
    assert code == bp.BP_E_WORKSPACE and need.value > 256
    torch.cuda.synchronize()
    assert torch.all(y == 0) and torch.all(b == 0)
    assert torch.equal(sol, ref[0]) and torch.equal(st, ref[1]) and torch.equal(tab, ref[2])
    assert torch.equal(meta, ref[3])
    bp.hp_paste_flat(params, npix, pix, t["theta_x"], t["theta_y"], t["v_los"], sol, st, tab, meta, y, b)
    torch.cuda.synchronize()
    assert torch.equal(y, ref[4]) and torch.equal(b, ref[5])
    # n = 0: nothing to do, nothing touched
    e = bp._lib.bp_hp_flat_pipeline(C.byref(params), npix, pix, 0, None, None, None, None, None, None, None, None,
                                    None, None, bp._ptr(y), bp._ptr(b), None, None, None, 0, C.byref(need),
                                    bp._stream())
    assert e == bp.BP_OK and need.value == 0


def test_pipeline_from_two_host_threads(bp):
    """Pipeline calls from two host threads, each on its own stream with its own workspace and maps: the
    library serialises them on the shared second stream, and every map equals the single-thread result."""
    import threading
    import torch
    from paper_2201_02632_amd.synth import flat_catalogue
    params = bp.default_params()
    npix = 256
    pix = 1.0 * math.pi / 180 / npix
    cats = [flat_catalogue(3000, 1.0, seed=21), flat_catalogue(1700, 1.0, seed=22)]
    tens = [{k: T(v) for k, v in c.items()} for c in cats]
    refs = [_three_calls(bp, params, t, npix, pix)[4:] for t in tens]
    torch.cuda.synchronize()
    out = [[None] * 4 for _ in tens]
    errors = []

    def work(k):
        try:
            st = torch.cuda.Stream()
            ws = bp.Workspace("cuda")
            t = tens[k]
            with torch.cuda.stream(st):
                for r in range(4):
                    y = torch.zeros((npix, npix), device="cuda")
                    b = torch.zeros_like(y)
                    bp.hp_flat_pipeline(params, npix, pix, t["M"], t["c"], t["z"], t["theta_x"], t["theta_y"],
                                        t["v_los"], y, b, ws=ws)
                    out[k][r] = (y, b)
            st.synchronize()
        except Exception as e:   # reported below, in the test's own thread
            errors.append(e)

    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=60)
    assert not any(x.is_alive() for x in th), "a pipeline thread did not finish"
    assert not errors, errors
    torch.cuda.synchronize()
    for k in range(2):
        for y, b in out[k]:
            assert torch.equal(y, refs[k][0]) and torch.equal(b, refs[k][1]), k
