"""Host-side checks of bench.py (no GPU): the multi-GPU refusal, the recorded deposit traffic, and the
footprint-pixel count that sets the deposit's roofline units."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_recorded_deposit_traffic_matches_the_sources():
    """The HBM bytes bench.py reports for the deposit were measured on the committed deposit sources
    (a change to them must come with new counter runs)."""
    import bench
    assert bench.deposit_traffic() == bench.DEPOSIT_TRAFFIC["bytes"]


def test_footprint_pixel_count_against_brute_force():
    """The unit count of the deposit's roofline: (pixel, halo) pairs with the pixel centre strictly
    inside R_t = D_A-scaled footprint, clipped to the map; checked by enumerating every pixel."""
    torch = pytest.importorskip("torch")
    import bench
    import paper_2201_02632_amd as bp
    rng = np.random.default_rng(5)
    n, npix, pix = 40, 64, 1e-4
    S = bp.SOL
    sol = torch.zeros((bp.SOL_NFIELDS, n), dtype=torch.float64)
    DA = rng.uniform(100.0, 900.0, n)
    R_pix = rng.uniform(0.3, 20.0, n)                # footprint radius in pixels
    sol[S["DA"]] = torch.as_tensor(DA)
    sol[S["RT"]] = torch.as_tensor(R_pix * DA * pix)
    st = torch.zeros(n, dtype=torch.int32)
    st[3] = 1                                         # an unsolved halo contributes nothing
    cat = {"theta_x": torch.as_tensor(rng.uniform(-5, npix + 5, n) * pix),
           "theta_y": torch.as_tensor(rng.uniform(-5, npix + 5, n) * pix)}
    got = bench.footprint_pixel_count(cat, sol, st, bp, npix, pix)
    ii, jj = np.meshgrid(np.arange(npix) + 0.5, np.arange(npix) + 0.5, indexing="xy")
    want = 0
    for h in range(n):
        if h == 3:
            continue
        cx, cy = cat["theta_x"][h].item() / pix, cat["theta_y"][h].item() / pix
        want += int(np.sum(np.hypot(ii - cx, jj - cy) < R_pix[h]))
    assert got == want, (got, want)
