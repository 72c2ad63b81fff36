"""The allocation-free flat paste against bp_hp_paste_flat: the same kernels on the library's fixed
per-GPU array instead of a caller workspace, so the maps must agree bit for bit, call after call (the
array keeps the previous call's contents, and the second call here is smaller than the first)."""
import ctypes as C

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


def _case(bp, n, seed, npix=256, field_deg=1.0):
    import torch

    from paper_2201_02632_amd.synth import flat_catalogue
    cat = flat_catalogue(n, field_deg, logM=(12.5, 15.0), seed=seed)
    t = {k: torch.as_tensor(v, dtype=torch.float64, device="cuda").contiguous() for k, v in cat.items()}
    params = bp.default_params()
    sol, st = bp.icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = bp.profile_tables(params, sol, st)
    return params, t, sol, st, tab, meta, npix, field_deg * np.pi / 180 / npix


def _noalloc(bp, params, t, sol, st, tab, meta, npix, pix, y, b, comp=None):
    need = C.c_size_t(0)
    yc, bc = (bp._ptr(comp[0]), bp._ptr(comp[1])) if comp else (None, None)
    code = bp._lib.bp_hp_paste_flat_noalloc(C.byref(params), npix, pix, t["M"].numel(), bp._ptr(t["theta_x"]),
                                            bp._ptr(t["theta_y"]), bp._ptr(t["v_los"]), bp._ptr(sol), bp._ptr(st),
                                            bp._ptr(tab), bp._ptr(meta), bp._ptr(y), bp._ptr(b), yc, bc,
                                            C.byref(need), bp._stream())
    return code, need.value


def test_noalloc_matches_workspace_paste(bp):
    import torch
    for n, seed, npix in ((3000, 71, 256), (700, 72, 96)):       # the second call is the smaller one
        print(f"no-alloc flat paste: n={n} seed={seed} npix={npix}", flush=True)
        params, t, sol, st, tab, meta, npix, pix = _case(bp, n, seed, npix)
        y1, b1, y2, b2 = (torch.zeros((npix, npix), dtype=torch.float32, device="cuda") for _ in range(4))
        bp.hp_paste_flat(params, npix, pix, t["theta_x"], t["theta_y"], t["v_los"], sol, st, tab, meta, y1, b1)
        code, need = _noalloc(bp, params, t, sol, st, tab, meta, npix, pix, y2, b2)
        torch.cuda.synchronize()
        assert code == bp.BP_OK, bp._lib.bp_strerror(code)
        assert 0 < need <= bp._lib.bp_hp_paste_flat_noalloc_max_bytes()
        assert torch.equal(y1, y2) and torch.equal(b1, b2)
        assert float(y1.abs().sum()) > 0


def test_noalloc_with_compensation_and_accumulation(bp):
    """Maps accumulate over calls (with the compensation maps carried) exactly as with the workspace paste."""
    import torch
    params, t, sol, st, tab, meta, npix, pix = _case(bp, 1500, 73, 128)
    ya, ba, yca, bca, yb, bb, ycb, bcb = (torch.zeros((npix, npix), dtype=torch.float32, device="cuda")
                                          for _ in range(8))
    for _ in range(2):
        bp.hp_paste_flat(params, npix, pix, t["theta_x"], t["theta_y"], t["v_los"], sol, st, tab, meta, ya, ba,
                         comp=(yca, bca))
        code, _ = _noalloc(bp, params, t, sol, st, tab, meta, npix, pix, yb, bb, comp=(ycb, bcb))
        assert code == bp.BP_OK
    torch.cuda.synchronize()
    assert torch.equal(ya, yb) and torch.equal(ba, bb) and torch.equal(yca, ycb) and torch.equal(bca, bcb)


def test_noalloc_refuses_more_than_its_array(bp):
    """A problem beyond the fixed array is refused before the maps are touched, with the size it needs."""
    import torch
    params, t, sol, st, tab, meta, _, _ = _case(bp, 200_000, 74, 4096, 5.0)
    npix = 4096
    pix = 5.0 * np.pi / 180 / npix
    y, b = torch.zeros((npix, npix), device="cuda"), torch.zeros((npix, npix), device="cuda")
    code, need = _noalloc(bp, params, t, sol, st, tab, meta, npix, pix, y, b)
    torch.cuda.synchronize()
    assert code == bp.BP_E_WORKSPACE
    assert need > bp._lib.bp_hp_paste_flat_noalloc_max_bytes()
    assert float(y.abs().max()) == 0.0 and float(b.abs().max()) == 0.0
    # and the array still serves a call that fits, right after
    params2, t2, sol2, st2, tab2, meta2, npix2, pix2 = _case(bp, 500, 75, 64)
    y1, b1, y2, b2 = (torch.zeros((npix2, npix2), dtype=torch.float32, device="cuda") for _ in range(4))
    bp.hp_paste_flat(params2, npix2, pix2, t2["theta_x"], t2["theta_y"], t2["v_los"], sol2, st2, tab2, meta2, y1, b1)
    code, _ = _noalloc(bp, params2, t2, sol2, st2, tab2, meta2, npix2, pix2, y2, b2)
    torch.cuda.synchronize()
    assert code == bp.BP_OK and torch.equal(y1, y2) and torch.equal(b1, b2)
