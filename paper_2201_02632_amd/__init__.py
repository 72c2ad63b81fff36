"""MI355X-native baryon pasting (Osato & Nagai 2022): Python binding of libbp.so.

Every step of the hot path runs in the HIP kernels of ``libbp.so``; this
module only marshals arguments (torch tensors on the GPU for device memory,
the current torch stream as the HIP stream).  There is no CPU fallback: if the
library is missing the import fails.

Entry points mirror include/bp.h:
    icm_solve, profile_tables, hp_paste_flat, healpix_ang2pix_ring, hp_paste_healpix,
    hp_flat_pipeline and hp_healpix_pipeline (the three calls of each path in one)
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libbp.so not built at {LIB_PATH}: run __graft_entry__.build() "
                      "(the HIP library is required; there is no fallback)")

_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------- mirrors --
BP_OK, BP_E_ARG, BP_E_HIP, BP_E_WORKSPACE, BP_E_OVERFLOW = 0, -1, -2, -3, -4
S_NO_BRACKET, S_MULTI_ROOT, S_NO_STAR_ROOT, S_NONFINITE, S_BAD_INPUT = 1, 2, 4, 8, 16

SOL_FIELDS = ["M", "C", "Z", "RVIR", "RS", "RHOS", "R500", "M500", "MSTAR", "XSTAR", "PS", "EGI",
              "A", "XF", "RF", "RHO0", "P0", "CHI", "DA", "TAU", "FNT", "RT", "RES_E"]
SOL = {name: k for k, name in enumerate(SOL_FIELDS)}
SOL_NFIELDS = len(SOL_FIELDS)

TAB_NA, TAB_NS, TAB_NB = 192, 32, 32
TAB_ZONE = TAB_NA + TAB_NS + TAB_NB
TAB_STRIDE = 2 * TAB_ZONE
META_FIELDS = ["ETA_LO", "ETA_HI", "OM_LO", "OM_HI", "ZE_LO", "ZE_HI", "PE0", "NE0", "PR_RV", "PR_INV_RS",
               "PR_RF", "PR_CM", "PR_PHI_OUT0", "PR_A", "PR_INV_R500", "PR_ANT_F"]
META = {name: k for k, name in enumerate(META_FIELDS)}
META_NFIELDS = len(META_FIELDS)


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "Omega_m", "Omega_b", "h", "Gamma", "eps_DM", "eps_star", "f_star", "S_star",
        "alpha_nt", "beta_nt", "n_nt", "X_H", "trunc_r500", "field_gas_frac", "field_T")] + [
        ("energy_sign", C.c_int32), ("reserved", C.c_int32)]


def default_params(**kw) -> Params:
    """Table 1 of the paper; cosmology Omega_m = 0.3, h = 0.7 with the paper's Omega_b = 0.046."""
    d = dict(Omega_m=0.3, Omega_b=0.046, h=0.7, Gamma=1.2, eps_DM=0.0, eps_star=3.97e-6,
             f_star=0.026, S_star=0.12, alpha_nt=0.18, beta_nt=0.5, n_nt=0.8, X_H=0.76,
             trunc_r500=3.0, field_gas_frac=0.046 / 0.3, field_T=0.0, energy_sign=0)
    d.update(kw)
    p = Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


_VP = C.c_void_p
_P = C.POINTER(Params)
_SIGS = {
    "bp_version": (C.c_int, []),
    "bp_strerror": (C.c_char_p, [C.c_int]),
    "bp_icm_solve": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bp_profile_tables": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, _VP, _VP]),
    "bp_hp_paste_flat": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                   _VP, _VP, _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_hp_flat_pipeline": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                      _VP, _VP, _VP, _VP, _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_hp_healpix_pipeline": (C.c_int, [_P, C.c_int64, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                         _VP, _VP, _VP, _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_hp_paste_flat_noalloc_max_bytes": (C.c_size_t, []),
    "bp_hp_paste_flat_noalloc": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                           _VP, _VP, _VP, _VP, C.POINTER(C.c_size_t), _VP]),
    "bp_healpix_ang2pix_ring": (C.c_int, [C.c_int64, C.c_int64, _VP, _VP, _VP, _VP]),
    "bp_hp_paste_healpix": (C.c_int, [_P, C.c_int64, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                      _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_pp_smoothing_length": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, C.c_int32, C.c_double, _VP, _VP,
                                         C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_pp_smoothing_length_eff": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, C.c_double, C.c_double, _VP, _VP,
                                             C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_pp_paste_flat": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                   C.c_double, C.c_int64, _VP, _VP, _VP, _VP, _VP, C.c_size_t,
                                   C.POINTER(C.c_size_t), _VP]),
    "bp_pp_paste_healpix_ngp": (C.c_int, [_P, C.c_int64, C.c_int64, _VP, _VP, _VP, _VP, C.c_double, _VP, _VP,
                                          C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_pp_healpix_ngp_selfcheck": (C.c_int, [C.c_int64, C.POINTER(C.c_double), _VP, C.c_size_t,
                                              C.POINTER(C.c_size_t), _VP]),
    "bp_flat_power_spectrum": (C.c_int, [C.c_int32, C.c_double, _VP, C.c_int32, C.POINTER(C.c_double), _VP, _VP,
                                         _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_mlp_nparams": (C.c_int64, []),
    "bp_mlp_act_bytes": (C.c_size_t, [C.c_int64]),
    "bp_mlp_backward_ws_bytes": (C.c_size_t, [C.c_int64]),
    "bp_mlp_forward": (C.c_int, [_VP, _VP, C.c_int64, _VP, _VP, _VP, _VP]),
    "bp_mlp_backward": (C.c_int, [_VP, _VP, C.c_int64, _VP, _VP, _VP, _VP, _VP, C.c_size_t, _VP]),
    "bp_mlp_adam": (C.c_int, [C.c_int64, _VP, _VP, _VP, _VP, _VP, C.c_float, C.c_float, C.c_float, C.c_float,
                              C.c_int64, _VP]),
    "bp_mlp_to_bf16": (C.c_int, [C.c_int64, _VP, _VP, _VP]),
    "bp_halo_structure": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bp_surrogate_features": (C.c_int, [C.c_int64, _VP, _VP, _VP, _VP, _VP]),
    "bp_surrogate_targets": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bp_surrogate_stats": (C.c_int, [C.c_int64, _VP, _VP, _VP, _VP]),
    "bp_gather_rows": (C.c_int, [C.c_int64, C.c_int32, _VP, _VP, _VP, _VP]),
    "bp_surrogate_mse": (C.c_int, [C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bp_surrogate_apply": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bp_surrogate_solve": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bp_surrogate_qtables_exact": (C.c_int, [_P, C.c_int64, _VP, _VP, _VP, _VP, _VP]),
    "bp_surrogate_state_bytes": (C.c_size_t, []),
    "bp_surrogate_state_offset": (C.c_size_t, [C.c_int32]),
    "bp_surrogate_init": (C.c_int, [_VP, C.c_uint64, _VP]),
    "bp_surrogate_blob_bytes": (C.c_size_t, []),
    "bp_surrogate_save": (C.c_int, [_VP, C.c_int64, _VP, C.c_size_t, _VP]),
    "bp_surrogate_load": (C.c_int, [_VP, _VP, C.c_size_t, C.POINTER(C.c_int64), _VP]),
    "bp_surrogate_fit": (C.c_int, [_P, _VP, C.c_int64, _VP, _VP, _VP, C.c_int64, C.c_int64, C.c_float, C.c_float,
                                   C.c_uint64, C.c_int64, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_surrogate_paste_flat": (C.c_int, [_P, _VP, C.c_int32, C.c_int32, C.c_double, C.c_int64, _VP, _VP, _VP, _VP,
                                          _VP, _VP, _VP, _VP, _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t),
                                          C.POINTER(C.c_int64), _VP]),
    "bp_surrogate_paste_healpix": (C.c_int, [_P, _VP, C.c_int32, C.c_int64, C.c_int64, _VP, _VP, _VP, _VP, _VP,
                                             _VP, _VP, _VP, _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t),
                                             C.POINTER(C.c_int64), _VP]),
    "bp_mlp_infer": (C.c_int, [_VP, _VP, C.c_int64, _VP, _VP, _VP]),
    "bp_hp_paste_flat_q": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                   _VP, _VP, _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_hp_paste_healpix_q": (C.c_int, [_P, C.c_int64, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                      _VP, _VP, _VP, C.c_size_t, C.POINTER(C.c_size_t), _VP]),
    "bp_surrogate_train_ws_bytes": (C.c_size_t, [C.c_int64]),
    "bp_surrogate_train": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, C.c_int64, _VP, _VP, C.c_int64, C.c_int64,
                                     C.c_float, C.c_float, C.c_uint64, C.c_int64, _VP, _VP, C.c_size_t, _VP]),
    "bp_profiling": (C.c_int, [C.c_int]),
    "bp_profile_read": (C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
}
PROF = {name: k for k, name in enumerate(["ICM", "TABLES", "FLAT_PLAN", "FLAT_DEPOSIT", "HPX_PLAN", "HPX_DEPOSIT",
                                          "PP_SORT", "PP_KNN", "PP_PLAN", "PP_DEPOSIT", "MLP_FWD", "MLP_BWD",
                                          "SURR_APPLY", "FLATQ_DEPOSIT", "HPXQ_DEPOSIT", "PP_NEFF", "NGP_PLAN",
                                          "NGP_DEPOSIT", "SPECTRUM", "SURR_SOLVE"])}
MLP_NIN, MLP_IN, MLP_HID, MLP_OUT, MLP_NOUT, MLP_NQ = 3, 16, 256, 144, 131, 64
SUR_ARRAYS = ["W", "WBF16", "M", "V", "G", "MEAN", "STD"]
SUR_TABLES = {"exact": 0, "network": 1}
S_OUT_OF_DOMAIN = 32
EXPORTED = list(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class BPError(RuntimeError):
    pass


def _check(code, what):
    if code != BP_OK:
        raise BPError(f"{what}: {_lib.bp_strerror(code).decode()} ({code})")


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def version() -> int:
    return _lib.bp_version()


# ------------------------------------------------------------- entry points --
def icm_solve(params: Params, M: torch.Tensor, c: torch.Tensor, z: torch.Tensor):
    """K1: returns (sol [SOL_NFIELDS, n] float64, status [n] int32) on the device."""
    n = M.numel()
    dev = M.device
    sol = torch.empty((SOL_NFIELDS, n), dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    if n:
        _check(_lib.bp_icm_solve(C.byref(params), n, _ptr(M), _ptr(c), _ptr(z), _ptr(sol), _ptr(status),
                                 _stream()), "bp_icm_solve")
    return sol, status


def surrogate_solve(params: Params, M: torch.Tensor, c: torch.Tensor, z: torch.Tensor, y: torch.Tensor,
                    mean: torch.Tensor, std: torch.Tensor):
    """K1 seeded by the surrogate network's output rows y [n, MLP_OUT] (standardised by mean, std):
    returns (sol [SOL_NFIELDS, n] float64, status [n] int32) on the device."""
    n = M.numel()
    dev = M.device
    sol = torch.empty((SOL_NFIELDS, n), dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    if n:
        assert y.dtype == torch.float32 and y.shape == (n, MLP_OUT), "network output rows [n, 144] float32 expected"
        _check(_lib.bp_surrogate_solve(C.byref(params), n, _ptr(M), _ptr(c), _ptr(z), _ptr(y), _ptr(mean), _ptr(std),
                                       _ptr(sol), _ptr(status), _stream()), "bp_surrogate_solve")
    return sol, status


def profile_tables(params: Params, sol: torch.Tensor, status: torch.Tensor):
    """K2: returns (tables [n, TAB_STRIDE] float32, meta [META_NFIELDS, n] float32)."""
    n = status.numel()
    dev = status.device
    tab = torch.empty((n, TAB_STRIDE), dtype=torch.float32, device=dev)
    meta = torch.empty((META_NFIELDS, n), dtype=torch.float32, device=dev)
    if n:
        _check(_lib.bp_profile_tables(C.byref(params), n, _ptr(sol), _ptr(status), _ptr(tab), _ptr(meta),
                                      _stream()), "bp_profile_tables")
    return tab, meta


class Workspace:
    """Grow-only device workspace reused across calls."""

    def __init__(self, device="cuda"):
        self.buf = None
        self.device = device

    def ensure(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes * 1.25) + 4096, dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws = {}


def _ws_for(device):
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def _with_workspace(fn, what, ws, args, tail=()):
    """Call fn(*args, ws, ws_bytes, &ws_needed, *tail, stream), growing the workspace while the library asks
    for more (a call that synchronises midway can ask again once it knows its data-dependent sizes)."""
    need = C.c_size_t(0)
    for _ in range(6):
        buf = ws.buf
        ptr = C.c_void_p(buf.data_ptr()) if buf is not None else C.c_void_p(0)
        nbytes = buf.numel() if buf is not None else 0
        code = fn(*args, ptr, nbytes, C.byref(need), *tail, _stream())
        if code == BP_E_WORKSPACE:
            ws.ensure(need.value)
            continue
        _check(code, what)
        return
    raise BPError(f"{what}: workspace negotiation did not converge")


def _comp_ptrs(comp, y_map):
    """Optional (y_comp, b_comp) Kahan compensation maps kept by the caller across calls."""
    if comp is None:
        return C.c_void_p(0), C.c_void_p(0)
    yc, bc = comp
    assert yc.shape == y_map.shape and bc.shape == y_map.shape and yc.dtype == torch.float32
    return _ptr(yc), _ptr(bc)


def hp_paste_flat(params: Params, npix: int, pix_rad: float, theta_x, theta_y, v_los, sol, status, tables, meta,
                  y_map, b_map, ws: Workspace | None = None, comp=None):
    """K3: accumulate the HP footprints of all halos into y_map, b_map ([npix, npix] float32); comp = (y_comp, b_comp)
    carries the Kahan compensation between calls."""
    ws = ws or _ws_for(y_map.device)
    _with_workspace(_lib.bp_hp_paste_flat, "bp_hp_paste_flat", ws,
                    (C.byref(params), int(npix), float(pix_rad), theta_x.numel(), _ptr(theta_x), _ptr(theta_y),
                     _ptr(v_los), _ptr(sol), _ptr(status), _ptr(tables), _ptr(meta), _ptr(y_map), _ptr(b_map),
                     *_comp_ptrs(comp, y_map)))


def hp_flat_pipeline(params: Params, npix: int, pix_rad: float, M, c, z, theta_x, theta_y, v_los, y_map, b_map,
                     ws: Workspace | None = None, comp=None):
    """K1, K2 and K3 in one call (bp_hp_flat_pipeline): the paste's plan overlaps the table quadratures.  Accumulates
    into y_map, b_map like hp_paste_flat and returns (sol, status, tables, meta) as icm_solve and profile_tables do."""
    n = M.numel()
    dev = y_map.device
    sol = torch.empty((SOL_NFIELDS, n), dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    tab = torch.empty((n, TAB_STRIDE), dtype=torch.float32, device=dev)
    meta = torch.empty((META_NFIELDS, n), dtype=torch.float32, device=dev)
    if n:
        ws = ws or _ws_for(dev)
        _with_workspace(_lib.bp_hp_flat_pipeline, "bp_hp_flat_pipeline", ws,
                        (C.byref(params), int(npix), float(pix_rad), n, _ptr(M), _ptr(c), _ptr(z), _ptr(theta_x),
                         _ptr(theta_y), _ptr(v_los), _ptr(sol), _ptr(status), _ptr(tab), _ptr(meta), _ptr(y_map),
                         _ptr(b_map), *_comp_ptrs(comp, y_map)))
    return sol, status, tab, meta


def hp_paste_flat_q(params: Params, npix: int, pix_rad: float, theta_x, theta_y, v_los, sol, status, qtables, meta,
                    y_map, b_map, ws: Workspace | None = None, comp=None):
    """K3 with surrogate q-tables (halos with a non-zero status are skipped)."""
    ws = ws or _ws_for(y_map.device)
    _with_workspace(_lib.bp_hp_paste_flat_q, "bp_hp_paste_flat_q", ws,
                    (C.byref(params), int(npix), float(pix_rad), theta_x.numel(), _ptr(theta_x), _ptr(theta_y),
                     _ptr(v_los), _ptr(sol), _ptr(status), _ptr(qtables), _ptr(meta), _ptr(y_map), _ptr(b_map),
                     *_comp_ptrs(comp, y_map)))


def hp_paste_healpix_q(params: Params, nside: int, theta, phi, v_los, sol, status, qtables, meta, y_map, b_map,
                       ws: Workspace | None = None, comp=None):
    """K4 with surrogate q-tables (halos with a non-zero status are skipped)."""
    ws = ws or _ws_for(y_map.device)
    _with_workspace(_lib.bp_hp_paste_healpix_q, "bp_hp_paste_healpix_q", ws,
                    (C.byref(params), int(nside), theta.numel(), _ptr(theta), _ptr(phi), _ptr(v_los), _ptr(sol),
                     _ptr(status), _ptr(qtables), _ptr(meta), _ptr(y_map), _ptr(b_map), *_comp_ptrs(comp, y_map)))


def hp_paste_healpix(params: Params, nside: int, theta, phi, v_los, sol, status, tables, meta, y_map, b_map,
                     ws: Workspace | None = None, comp=None):
    """K4: accumulate the HP footprints into HEALPix RING maps (12 nside^2 float32); comp = (y_comp, b_comp) carries
    the Kahan compensation between calls."""
    ws = ws or _ws_for(y_map.device)
    _with_workspace(_lib.bp_hp_paste_healpix, "bp_hp_paste_healpix", ws,
                    (C.byref(params), int(nside), theta.numel(), _ptr(theta), _ptr(phi), _ptr(v_los), _ptr(sol),
                     _ptr(status), _ptr(tables), _ptr(meta), _ptr(y_map), _ptr(b_map), *_comp_ptrs(comp, y_map)))


def hp_healpix_pipeline(params: Params, nside: int, M, c, z, theta, phi, v_los, y_map, b_map,
                        ws: Workspace | None = None, comp=None):
    """K1, K2 and K4 in one call (bp_hp_healpix_pipeline): the paste's plan overlaps the table quadratures.
    Accumulates into y_map, b_map like hp_paste_healpix and returns (sol, status, tables, meta)."""
    n = M.numel()
    dev = y_map.device
    sol = torch.empty((SOL_NFIELDS, n), dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    tab = torch.empty((n, TAB_STRIDE), dtype=torch.float32, device=dev)
    meta = torch.empty((META_NFIELDS, n), dtype=torch.float32, device=dev)
    if n:
        ws = ws or _ws_for(dev)
        _with_workspace(_lib.bp_hp_healpix_pipeline, "bp_hp_healpix_pipeline", ws,
                        (C.byref(params), int(nside), n, _ptr(M), _ptr(c), _ptr(z), _ptr(theta), _ptr(phi),
                         _ptr(v_los), _ptr(sol), _ptr(status), _ptr(tab), _ptr(meta), _ptr(y_map), _ptr(b_map),
                         *_comp_ptrs(comp, y_map)))
    return sol, status, tab, meta


def healpix_ang2pix_ring(nside: int, theta: torch.Tensor, phi: torch.Tensor) -> torch.Tensor:
    n = theta.numel()
    out = torch.empty(n, dtype=torch.int64, device=theta.device)
    if n:
        _check(_lib.bp_healpix_ang2pix_ring(int(nside), n, _ptr(theta), _ptr(phi), _ptr(out), _stream()),
               "bp_healpix_ang2pix_ring")
    return out


def pp_smoothing_length(params: Params, theta_x, theta_y, z, k: int = 32, cell: float = 0.0,
                        ws: Workspace | None = None) -> torch.Tensor:
    """K5+K6: distance to the k-th nearest other particle [comoving Mpc/h] (float32 inputs)."""
    n = theta_x.numel()
    h = torch.empty(n, dtype=torch.float32, device=theta_x.device)
    ws = ws or _ws_for(theta_x.device)
    if n:
        _with_workspace(_lib.bp_pp_smoothing_length, "bp_pp_smoothing_length", ws,
                        (C.byref(params), n, _ptr(theta_x), _ptr(theta_y), _ptr(z), int(k), float(cell), _ptr(h)))
    return h


def pp_smoothing_length_eff(params: Params, theta_x, theta_y, z, n_ngb: float = 64.0, cell: float = 0.0,
                            ws: Workspace | None = None) -> torch.Tensor:
    """K5+K6+K6b: smoothing length with effective neighbour number n_ngb [comoving Mpc/h]."""
    n = theta_x.numel()
    h = torch.empty(n, dtype=torch.float32, device=theta_x.device)
    ws = ws or _ws_for(theta_x.device)
    if n:
        _with_workspace(_lib.bp_pp_smoothing_length_eff, "bp_pp_smoothing_length_eff", ws,
                        (C.byref(params), n, _ptr(theta_x), _ptr(theta_y), _ptr(z), float(n_ngb), float(cell),
                         _ptr(h)))
    return h


def pp_paste_flat(params: Params, npix: int, pix_rad: float, parts: dict, h, M_p: float, sol, status, y_map, b_map,
                  ws: Workspace | None = None):
    """K7+K8: accumulate the SPH footprints of all particles into y_map, b_map."""
    n = parts["theta_x"].numel()
    ws = ws or _ws_for(y_map.device)
    nh = status.numel() if status is not None else 0
    sp = _ptr(sol) if nh else C.c_void_p(0)
    stp = _ptr(status) if nh else C.c_void_p(0)
    _with_workspace(_lib.bp_pp_paste_flat, "bp_pp_paste_flat", ws,
                    (C.byref(params), int(npix), float(pix_rad), n, _ptr(parts["theta_x"]), _ptr(parts["theta_y"]),
                     _ptr(parts["z"]), _ptr(parts["v_los"]), _ptr(parts["halo_id"]), _ptr(parts["r_i"]), _ptr(h),
                     float(M_p), nh, sp, stp, _ptr(y_map), _ptr(b_map)))


def pp_paste_healpix_ngp(params: Params, nside: int, theta, phi, z, v_los, M_p: float, b_map,
                         ws: Workspace | None = None):
    """K13: accumulate the nearest-pixel kSZ of field particles into b_map (12 nside^2 float32, RING)."""
    n = theta.numel()
    for t in (theta, phi, z, v_los, b_map):
        assert t.dtype == torch.float32, "float32 tensors expected"
    assert phi.numel() == n and z.numel() == n and v_los.numel() == n
    assert b_map.numel() == 12 * nside * nside or not 1 <= nside <= 2048, "b_map must hold 12 nside^2 pixels"
    ws = ws or _ws_for(b_map.device)
    _with_workspace(_lib.bp_pp_paste_healpix_ngp, "bp_pp_paste_healpix_ngp", ws,
                    (C.byref(params), int(nside), n, _ptr(theta), _ptr(phi), _ptr(z), _ptr(v_los), float(M_p),
                     _ptr(b_map)))


def pp_healpix_ngp_selfcheck(nside: int = 1024, ws: Workspace | None = None):
    """Measured (z error, cap-factor error / N) of the nearest-pixel paste's FP32 screen and the
    bounds it assumes, over every float colatitude."""
    out = (C.c_double * 4)()
    ws = ws or _ws_for(torch.device("cuda", torch.cuda.current_device()))
    _with_workspace(_lib.bp_pp_healpix_ngp_selfcheck, "bp_pp_healpix_ngp_selfcheck", ws, (int(nside), out))
    return {"z_err": out[0], "tmp_err_per_n": out[1], "z_bound": out[2], "tmp_bound_per_n": out[3]}


def flat_power_spectrum(m, pix_rad: float, edges, ws: Workspace | None = None):
    """K14: (ell_b, C_b, n_b) of a square float32 device map in the bins given by edges (ell)."""
    assert m.dtype == torch.float32 and m.dim() == 2 and m.shape[0] == m.shape[1]
    e = [float(x) for x in edges]
    nb = len(e) - 1
    ell = torch.empty(nb, dtype=torch.float64, device=m.device)
    cl = torch.empty_like(ell)
    nm = torch.empty(nb, dtype=torch.int64, device=m.device)
    ws = ws or _ws_for(m.device)
    _with_workspace(_lib.bp_flat_power_spectrum, "bp_flat_power_spectrum", ws,
                    (int(m.shape[0]), float(pix_rad), _ptr(m), nb, (C.c_double * len(e))(*e), _ptr(ell), _ptr(cl),
                     _ptr(nm)))
    return ell, cl, nm


def pp_flat_map(params: Params, halos: dict, parts: dict, M_p: float, npix: int, pix_rad: float, k: int = 32,
                cell: float = 0.0, device="cuda"):
    """Convenience: full PP path (halo solve, smoothing lengths, amplitudes, deposit) from numpy inputs."""
    th = {kk: torch.as_tensor(v, dtype=torch.float64, device=device).contiguous() for kk, v in halos.items()}
    tp = {kk: torch.as_tensor(v, device=device).contiguous() for kk, v in parts.items()}
    sol, status = icm_solve(params, th["M"], th["c"], th["z"])
    h = pp_smoothing_length(params, tp["theta_x"], tp["theta_y"], tp["z"], k, cell)
    y = torch.zeros((npix, npix), dtype=torch.float32, device=device)
    b = torch.zeros_like(y)
    pp_paste_flat(params, npix, pix_rad, tp, h, M_p, sol, status, y, b)
    return y, b, h, sol, status


def profiling(enable: bool):
    _lib.bp_profiling(1 if enable else 0)


def profile_read(name: str):
    tot, cnt = C.c_double(0), C.c_int64(0)
    _check(_lib.bp_profile_read(PROF[name], C.byref(tot), C.byref(cnt)), "bp_profile_read")
    return tot.value, cnt.value


def hp_flat_map(params: Params, cat: dict, npix: int, pix_rad: float, device="cuda"):
    """Convenience: full exact HP flat path (solve, tables, paste) for a catalogue of numpy arrays."""
    t = {k: torch.as_tensor(v, dtype=torch.float64, device=device).contiguous() for k, v in cat.items()}
    sol, status = icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = profile_tables(params, sol, status)
    y = torch.zeros((npix, npix), dtype=torch.float32, device=device)
    b = torch.zeros_like(y)
    hp_paste_flat(params, npix, pix_rad, t["theta_x"], t["theta_y"], t["v_los"], sol, status, tab, meta, y, b)
    return y, b, sol, status


def hp_healpix_map(params: Params, cat: dict, nside: int, device="cuda"):
    """Convenience: exact HP path onto HEALPix RING pixels for a catalogue (theta, phi) of numpy arrays."""
    t = {k: torch.as_tensor(v, dtype=torch.float64, device=device).contiguous() for k, v in cat.items()}
    sol, status = icm_solve(params, t["M"], t["c"], t["z"])
    tab, meta = profile_tables(params, sol, status)
    y = torch.zeros(12 * nside * nside, dtype=torch.float32, device=device)
    b = torch.zeros_like(y)
    hp_paste_healpix(params, nside, t["theta"], t["phi"], t["v_los"], sol, status, tab, meta, y, b)
    return y, b, sol, status
