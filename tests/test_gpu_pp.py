"""GPU parity of the particle-based pasting path (K5-K8) against the oracle."""
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


def T(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda") if dtype is None else \
        torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.fixture(scope="module")
def small_case(orc):
    from paper_2201_02632_amd.synth import pp_small
    halos, parts, M_p, npix, pix = pp_small(3)
    p = orc.default_params()
    sol = orc.solve_halos(p, halos["M"], halos["c"], halos["z"])
    print(f"pp small: {len(parts['z'])} particles, {len(halos['M'])} halos", flush=True)
    y, b, h, H, ay, ab = orc.pp_flat(p, sol, parts, M_p, npix, pix)
    _, babs, _, _, _, _ = orc.pp_flat(p, sol, dict(parts, v_los=np.abs(parts["v_los"])), M_p, npix, pix)
    return dict(halos=halos, parts=parts, M_p=M_p, npix=npix, pix=pix, y=y, b=b, babs=babs, h=h, ay=ay)


@pytest.mark.parametrize("cell", [0.0, 0.5, 6.0])
def test_knn_matches_brute_force(bp, small_case, cell):
    import torch
    pr = small_case["parts"]
    h = bp.pp_smoothing_length(bp.default_params(), T(pr["theta_x"]), T(pr["theta_y"]), T(pr["z"]), 32, cell)
    torch.cuda.synchronize()
    h = h.cpu().numpy().astype(np.float64)
    err = np.max(np.abs(h / small_case["h"] - 1))
    print(f"kNN cell={cell}: max rel err {err:.2e}")
    assert np.all(np.isfinite(h)) and err < 2e-6


def test_knn_density_contrast(bp, orc):
    """Clustered blobs (1e4 x denser than the background) plus a sparse background."""
    import torch
    rng = np.random.default_rng(9)
    chi0 = 800.0
    pts = [rng.uniform([0, 0, chi0], [40, 40, chi0 + 40], size=(3000, 3))]
    for c in rng.uniform([5, 5, chi0 + 5], [35, 35, chi0 + 35], size=(5, 3)):
        pts.append(c + rng.normal(scale=0.05, size=(400, 3)))
    P = np.concatenate(pts)
    p = orc.default_params()
    # back to (theta_x, theta_y, z): invert chi(z) with the oracle's own distance
    zs = np.linspace(0.2, 0.35, 4001)
    chis = np.array([orc.chi(p, z) for z in zs])
    z = np.interp(P[:, 2], chis, zs).astype(np.float32)
    tx = (P[:, 0] / P[:, 2]).astype(np.float32)
    ty = (P[:, 1] / P[:, 2]).astype(np.float32)
    chi_exact = np.array([orc.chi(p, float(zz)) for zz in z])
    h_o = orc.knn_h(chi_exact * tx, chi_exact * ty, chi_exact, 32)
    h = bp.pp_smoothing_length(bp.default_params(), T(tx), T(ty), T(z), 32)
    torch.cuda.synchronize()
    h = h.cpu().numpy().astype(np.float64)
    assert h_o.max() / h_o.min() > 30
    assert np.max(np.abs(h / h_o - 1)) < 2e-6


@pytest.mark.parametrize("cell", [0.0, 6.0])
def test_neff_smoothing_matches_oracle(bp, orc, small_case, cell):
    """Smoothing length from the effective neighbour number 64 (Sec. 3.4) against the oracle's
    bisection over every particle, on 1,500 sampled particles of the small light cone."""
    import torch
    pr = small_case["parts"]
    p = orc.default_params()
    tx, ty, z = (np.asarray(pr[k], dtype=np.float32) for k in ("theta_x", "theta_y", "z"))
    chi = np.array([orc.chi(p, float(zz)) for zz in z])
    X, Y, Z = chi * tx.astype(np.float64), chi * ty.astype(np.float64), chi
    h = bp.pp_smoothing_length_eff(bp.default_params(), T(tx), T(ty), T(z), 64.0, cell)
    torch.cuda.synchronize()
    h = h.cpu().numpy().astype(np.float64)
    q = np.random.default_rng(31).choice(len(z), 1500, replace=False)
    ho = orc.neff_h_query(q, X, Y, Z, 64.0)
    err = np.max(np.abs(h[q] / ho - 1))
    print(f"N_eff smoothing cell={cell}: max rel err {err:.2e}; h/h_32NN median {np.median(h / small_case['h']):.3f}")
    assert np.all(np.isfinite(h)) and err < 2e-6


def test_neff_density_contrast_and_args(bp, orc):
    """The same on clustered blobs (1e4 x denser) over a sparse background, every point; and the
    argument range of the effective neighbour number."""
    import torch
    rng = np.random.default_rng(10)
    chi0 = 800.0
    pts = [rng.uniform([0, 0, chi0], [40, 40, chi0 + 40], size=(3000, 3))]
    for c in rng.uniform([5, 5, chi0 + 5], [35, 35, chi0 + 35], size=(5, 3)):
        pts.append(c + rng.normal(scale=0.05, size=(400, 3)))
    P = np.concatenate(pts)
    p = orc.default_params()
    zs = np.linspace(0.2, 0.35, 4001)
    chis = np.array([orc.chi(p, z) for z in zs])
    z = np.interp(P[:, 2], chis, zs).astype(np.float32)
    tx = (P[:, 0] / P[:, 2]).astype(np.float32)
    ty = (P[:, 1] / P[:, 2]).astype(np.float32)
    chi_exact = np.array([orc.chi(p, float(zz)) for zz in z])
    X, Y, Z = chi_exact * tx, chi_exact * ty, chi_exact
    h = bp.pp_smoothing_length_eff(bp.default_params(), T(tx), T(ty), T(z), 64.0)
    torch.cuda.synchronize()
    h = h.cpu().numpy().astype(np.float64)
    ho = orc.neff_h_query(np.arange(len(z)), X, Y, Z, 64.0)
    assert ho.max() / ho.min() > 30
    assert np.max(np.abs(h / ho - 1)) < 2e-6
    for bad in (10.0, 2000.0, float("nan")):
        with pytest.raises(RuntimeError):
            bp.pp_smoothing_length_eff(bp.default_params(), T(tx), T(ty), T(z), bad)


def test_pp_map_parity(bp, small_case):
    import torch
    c = small_case
    y, b, h, sol, st = bp.pp_flat_map(bp.default_params(), c["halos"], c["parts"], c["M_p"], c["npix"], c["pix"])
    torch.cuda.synchronize()
    y, b = y.cpu().numpy(), b.cpu().numpy()
    ey, eb = rel_err(y, c["y"]), rel_err(b, c["b"], c["babs"])
    Yerr = abs(y.astype(np.float64).sum() / c["y"].sum() - 1)
    print(f"PP map: max rel err y {ey:.2e} b {eb:.2e} integrated-Y {Yerr:.2e}")
    assert ey < 1e-5 and eb < 1e-5 and Yerr < 1e-6


def test_pp_sign_determinism_and_conservation(bp, small_case):
    import torch
    c = small_case
    params = bp.default_params()
    y1, b1, h1, _, _ = bp.pp_flat_map(params, c["halos"], c["parts"], c["M_p"], c["npix"], c["pix"])
    y2, b2, h2, _, _ = bp.pp_flat_map(params, c["halos"], c["parts"], c["M_p"], c["npix"], c["pix"])
    parts_neg = dict(c["parts"], v_los=-c["parts"]["v_los"])
    y3, b3, _, _, _ = bp.pp_flat_map(params, c["halos"], parts_neg, c["M_p"], c["npix"], c["pix"])
    torch.cuda.synchronize()
    assert torch.equal(h1, h2) and torch.equal(y1, y2) and torch.equal(b1, b2)
    assert torch.equal(y3, y1) and torch.equal(b3, -b1)
    # the weights sum to one: a map big enough to hold every footprint keeps the total amplitude
    npix = 3 * c["npix"]
    shift = c["npix"] * c["pix"]
    pr = dict(c["parts"])
    pr["theta_x"] = (pr["theta_x"].astype(np.float64) + shift).astype(np.float32)
    pr["theta_y"] = (pr["theta_y"].astype(np.float64) + shift).astype(np.float32)
    yb, _, _, _, _ = bp.pp_flat_map(params, c["halos"], pr, c["M_p"], npix, c["pix"])
    torch.cuda.synchronize()
    assert abs(yb.double().sum().item() / c["ay"].sum() - 1) < 1e-5


def test_pp_edge_inputs(bp):
    import torch
    params = bp.default_params()
    # too few particles for k and a redshift out of range are argument errors
    x = T(np.zeros(10, np.float32))
    with pytest.raises(bp.BPError):
        bp.pp_smoothing_length(params, x, x, x, 32)
    zz = T(np.full(100, 20.0, np.float32))
    xx = T(np.linspace(0, 1e-3, 100).astype(np.float32))
    with pytest.raises(bp.BPError):
        bp.pp_smoothing_length(params, xx, xx, zz, 32)


def test_pp_field_tsz_parity(bp, orc, small_case):
    # filament gas (field particles) with the pressure n_e k_B T at the field temperature 1e4 K
    import torch
    c = small_case
    p = orc.default_params()
    p.field_T = 1e4
    sol = orc.solve_halos(p, c["halos"]["M"], c["halos"]["c"], c["halos"]["z"])
    yo, bo, _, _, ay, _ = orc.pp_flat(p, sol, c["parts"], c["M_p"], c["npix"], c["pix"])
    field = c["parts"]["halo_id"] < 0
    assert np.all(ay[field] > 0)
    y, b, _, _, _ = bp.pp_flat_map(bp.default_params(field_T=1e4), c["halos"], c["parts"], c["M_p"], c["npix"],
                                   c["pix"])
    torch.cuda.synchronize()
    y, b = y.cpu().numpy(), b.cpu().numpy()
    ey, eb = rel_err(y, yo), rel_err(b, bo, c["babs"])
    dY = y.astype(np.float64).sum() - c["y"].sum()          # the field particles' share of integrated y
    print(f"PP field tSZ: max rel err y {ey:.2e} b {eb:.2e}; field share of Y {dY / y.sum():.3e}")
    assert ey < 1e-5 and eb < 1e-5
    assert abs(y.astype(np.float64).sum() / yo.sum() - 1) < 1e-6
    assert dY > 0
