"""GPU parity of the HP deposit onto HEALPix RING pixels against the oracle (brute force over all pixels)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_02632_amd as bp
    return bp


def rel_err(g, o, scale=None):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    ref = np.abs(o) if scale is None else np.asarray(scale, dtype=np.float64)
    floor = 1e-6 * ref.max() if ref.max() > 0 else 1e-300
    return float(np.max(np.abs(g - o) / (ref + floor)))


def sky_case(seed, n, nside):
    """Nearby halos (footprints of a few to tens of pixels), some at the poles and across phi = 0."""
    rng = np.random.default_rng(seed)
    M = 10 ** rng.uniform(13.0, 15.0, n)
    z = rng.uniform(0.02, 0.12, n)
    c = 5 * (M / 1e14) ** -0.1 * (1 + z) ** -0.5 * 10 ** rng.normal(0, 0.1, n)
    th = np.arccos(rng.uniform(-1, 1, n))
    ph = rng.uniform(0, 2 * math.pi, n)
    th[:4] = [0.004, math.pi - 0.003, math.acos(2 / 3) + 1e-3, math.pi / 2]
    ph[:4] = [1.0, 5.0, 2 * math.pi - 1e-3, 0.0]
    v = rng.normal(0, 300, n)
    return dict(M=M, c=c, z=z, theta=th, phi=ph, v_los=v)


@pytest.mark.parametrize("nside,n,seed", [(512, 24, 1), (1024, 16, 2)])
def test_hp_healpix_vs_oracle(bp, orc, nside, n, seed):
    import torch
    cat = sky_case(seed, n, nside)
    print(f"healpix nside={nside} n={n} seed={seed}", flush=True)
    y, b, _, st = bp.hp_healpix_map(bp.default_params(), cat, nside)
    torch.cuda.synchronize()
    p = orc.default_params()
    yo, bo, halos = orc.hp_healpix(p, cat, nside)
    _, babs, _ = orc.hp_healpix(p, dict(cat, v_los=np.abs(cat["v_los"])), nside)
    assert np.array_equal(st.cpu().numpy(), orc.halos_table(halos)["status"].astype(np.int32))
    assert (yo > 0).sum() > 200
    ey = rel_err(y.cpu().numpy(), yo)
    eb = rel_err(b.cpu().numpy(), bo, babs)
    Yerr = abs(y.cpu().double().sum().item() / yo.sum() - 1)
    print(f"max rel err y {ey:.2e} b {eb:.2e} integrated-Y {Yerr:.2e}")
    assert ey < 1e-5 and eb < 1e-5 and Yerr < 1e-6


@pytest.mark.parametrize("nside,n,zlo,zhi,seed", [(1, 60, 0.002, 0.004, 7), (3, 60, 0.002, 0.006, 8),
                                                   (13, 120, 0.003, 0.02, 9), (100, 60, 0.01, 0.05, 10)])
def test_hp_healpix_small_and_odd_nside(bp, orc, nside, n, zlo, zhi, seed):
    # few and short rings: a partial last band of rings, polar bands whose rings hold fewer pixels
    # than the band's longest one, and (odd N_side) a last tile half as wide as the others
    import torch
    cat = sky_case(seed, n, nside)
    cat["z"] = np.random.default_rng(seed + 100).uniform(zlo, zhi, n)
    print(f"healpix small nside={nside} n={n} seed={seed}", flush=True)
    y, b, _, _ = bp.hp_healpix_map(bp.default_params(), cat, nside)
    torch.cuda.synchronize()
    p = orc.default_params()
    yo, bo, _ = orc.hp_healpix(p, cat, nside)
    _, babs, _ = orc.hp_healpix(p, dict(cat, v_los=np.abs(cat["v_los"])), nside)
    assert (yo > 0).sum() >= 4
    yg = y.cpu().numpy()
    assert np.array_equal(yg > 0, yo > 0)
    ey = rel_err(yg, yo)
    eb = rel_err(b.cpu().numpy(), bo, babs)
    print(f"nside={nside}: pixels hit {(yo > 0).sum()}, max rel err y {ey:.2e} b {eb:.2e}")
    assert ey < 1e-5 and eb < 1e-5


def test_hp_healpix_sign_and_determinism(bp):
    import torch
    cat = sky_case(3, 20, 256)
    params = bp.default_params()
    y1, b1, _, _ = bp.hp_healpix_map(params, cat, 256)
    y2, b2, _, _ = bp.hp_healpix_map(params, cat, 256)
    y3, b3, _, _ = bp.hp_healpix_map(params, dict(cat, v_los=-cat["v_los"]), 256)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2) and torch.equal(b1, b2)
    assert torch.equal(y1, y3) and torch.equal(b3, -b1)


def test_hp_healpix_batches_with_compensation_equal_one_call(bp):
    """All-sky maps accumulate over halo batches: carrying the Kahan compensation maps between calls makes
    consecutive batches reproduce one call over the whole catalogue bit for bit."""
    import torch
    cat = sky_case(5, 300, 256)
    params = bp.default_params()
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    t = {k: T(v) for k, v in cat.items()}
    npx = 12 * 256 * 256
    sol, st = bp.icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = bp.profile_tables(params, sol, st)
    y1 = torch.zeros(npx, device="cuda")
    b1 = torch.zeros_like(y1)
    bp.hp_paste_healpix(params, 256, t["theta"], t["phi"], t["v_los"], sol, st, tab, meta, y1, b1)
    yb, bb, yc, bc = (torch.zeros_like(y1) for _ in range(4))
    for a, e in ((0, 77), (77, 78), (78, 250), (250, 300)):
        sub = {k: v[a:e].contiguous() for k, v in t.items()}
        s2, st2 = bp.icm_solve(params, sub["M"], sub["c"], sub["z"])
        tb2, mt2 = bp.profile_tables(params, s2, st2)
        bp.hp_paste_healpix(params, 256, sub["theta"], sub["phi"], sub["v_los"], s2, st2, tb2, mt2, yb, bb,
                            comp=(yc, bc))
    torch.cuda.synchronize()
    assert torch.equal(yb, y1) and torch.equal(bb, b1)


def test_hp_healpix_pipeline_equals_three_calls(bp):
    """bp_hp_healpix_pipeline returns the solution, tables and maps of the three calls bit for bit, also for
    batches that carry the compensation maps and on a second, smaller call on the same workspace."""
    import torch
    params = bp.default_params()
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    nside = 256
    npx = 12 * nside * nside
    ws = bp.Workspace("cuda")
    for n, seed in ((400, 8), (57, 9)):
        t = {k: T(v) for k, v in sky_case(seed, n, nside).items()}
        sol, st = bp.icm_solve(params, t["M"], t["c"], t["z"])
        tab, meta = bp.profile_tables(params, sol, st)
        y1, b1 = torch.zeros(npx, device="cuda"), torch.zeros(npx, device="cuda")
        bp.hp_paste_healpix(params, nside, t["theta"], t["phi"], t["v_los"], sol, st, tab, meta, y1, b1)
        y2, b2 = torch.zeros_like(y1), torch.zeros_like(y1)
        got = bp.hp_healpix_pipeline(params, nside, t["M"], t["c"], t["z"], t["theta"], t["phi"], t["v_los"], y2, b2,
                                     ws=ws)
        torch.cuda.synchronize()
        for name, r, g in zip(("sol", "status", "tables", "meta", "y", "b"), (sol, st, tab, meta, y1, b1),
                              (*got, y2, b2)):
            assert torch.equal(r, g), (n, name)
        assert (y1 != 0).sum().item() > 0
        # batches with compensation: pipeline calls against paste calls
        yb, bb, yc, bc = (torch.zeros_like(y1) for _ in range(4))
        yp, bq, ycp, bcp = (torch.zeros_like(y1) for _ in range(4))
        for a, e in ((0, n // 3), (n // 3, n)):
            sub = {k: v[a:e].contiguous() for k, v in t.items()}
            s2, st2 = bp.icm_solve(params, sub["M"], sub["c"], sub["z"])
            tb2, mt2 = bp.profile_tables(params, s2, st2)
            bp.hp_paste_healpix(params, nside, sub["theta"], sub["phi"], sub["v_los"], s2, st2, tb2, mt2, yb, bb,
                                comp=(yc, bc))
            bp.hp_healpix_pipeline(params, nside, sub["M"], sub["c"], sub["z"], sub["theta"], sub["phi"],
                                   sub["v_los"], yp, bq, ws=ws, comp=(ycp, bcp))
        torch.cuda.synchronize()
        assert torch.equal(yb, yp) and torch.equal(bb, bq) and torch.equal(yc, ycp) and torch.equal(bc, bcp)
