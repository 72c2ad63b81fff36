"""GPU parity of the flat-sky power spectrum (K14, Sec. 5.3) against the oracle."""
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


def gpu_spectrum(bp, m, pix, edges):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(m, dtype=np.float32), device="cuda")
    ell, cl, nm = bp.flat_power_spectrum(t, pix, edges)
    torch.cuda.synchronize()
    return ell.cpu().numpy(), cl.cpu().numpy(), nm.cpu().numpy()


def compare(g, o):
    ell, cl, nm = g
    lo, co, no = o
    assert np.array_equal(nm, no)
    full = no > 0
    assert np.all(cl[~full] == 0) and np.all(ell[~full] == 0)
    dcl, dell = np.abs(cl - co)[full], np.abs(ell - lo)[full]
    assert np.all(dcl <= 1e-9 * np.abs(co[full])) and np.all(dell <= 1e-12 * lo[full])   # ell_b = 0 for k = 0 alone
    ecl = float(np.max(dcl / np.where(co[full] != 0, np.abs(co[full]), np.inf))) if full.any() else 0.0
    eell = float(np.max(dell / np.where(lo[full] > 0, lo[full], np.inf))) if full.any() else 0.0
    return ecl, eell


@pytest.mark.parametrize("n,seed", [(2, 1), (8, 2), (64, 3), (256, 4), (1024, 5)])
def test_spectrum_random_maps(bp, n, seed):
    from oracle import spectrum as S
    rng = np.random.default_rng(seed)
    m = rng.lognormal(0, 1, size=(n, n)).astype(np.float32) - 1.0
    pix = 5 * math.pi / 180 / 4096
    L = n * pix
    edges = S.log_edges(30, 2 * math.pi / L, math.pi * math.sqrt(2) / pix * 1.01)
    ecl, eell = compare(gpu_spectrum(bp, m, pix, edges), S.flat_power_spectrum(m, pix, edges))
    print(f"spectrum n={n}: max rel err C {ecl:.2e} ell {eell:.2e}")


def test_spectrum_of_paste_maps_and_paper_bins(bp, orc):
    import torch
    from oracle import spectrum as S
    from paper_2201_02632_amd.synth import hp_flat_small
    cat, npix, pix = hp_flat_small(1)
    y, b, _, _ = bp.hp_flat_map(bp.default_params(), cat, npix, pix)
    torch.cuda.synchronize()
    edges = S.log_edges(30, 1e2, 1e5)
    for m in (y.cpu().numpy(), b.cpu().numpy()):
        g = gpu_spectrum(bp, m, pix, edges)
        compare(g, S.flat_power_spectrum(m, pix, edges))
    # a bin list with empty bins and edges below the fundamental
    edges2 = np.array([0.0, 10.0, 20.0, 3e3, 3.0001e3, 1e4, 2e5])
    compare(gpu_spectrum(bp, y.cpu().numpy(), pix, edges2), S.flat_power_spectrum(y.cpu().numpy(), pix, edges2))


def test_spectrum_arguments(bp):
    import torch
    m = torch.zeros((48, 48), dtype=torch.float32, device="cuda")
    with pytest.raises(bp.BPError):
        bp.flat_power_spectrum(m, 1e-4, [1e2, 1e3])                 # not a power of two
    m = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    for bad in ([1e3, 1e2], [1e2, float("nan")], [-1.0, 1e2], list(np.logspace(2, 5, 70))):
        with pytest.raises(bp.BPError):
            bp.flat_power_spectrum(m, 1e-4, bad)
