"""FP64 CPU oracle of the baryon-pasting method (Osato & Nagai 2022).

TEST INFRASTRUCTURE ONLY.  Plain single-threaded C (``bp_oracle.c``) behind a
ctypes shim.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product path
(``paper_2201_02632_amd``) never imports it and shares no code with it.

Function-by-function citations of the paper sections live in ``bp_oracle.c``.
Parity status: every piece is pinned by the CPU tests except the solved ICM
amplitude as a whole (the paper prints no worked halo solution): "parity
unpinned" for the composite (rho0, P0, r_f) beyond its pieces and residuals.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bp_oracle.c")
LIB = os.path.join(HERE, "libbp_oracle.so")

# status bits (mirror of the C definitions)
OK, NO_BRACKET, MULTI_ROOT, NO_STAR_ROOT, NONFINITE, BAD_INPUT = 0, 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FP contraction: the HEALPix integer
    steps must be reproducible)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", LIB + ".tmp", SRC, "-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "Omega_m", "Omega_b", "h", "Gamma", "eps_DM", "eps_star", "f_star", "S_star",
        "alpha_nt", "beta_nt", "n_nt", "X_H", "trunc_r500", "field_gas_frac", "field_T")] + [
        ("energy_sign", C.c_int), ("pad_", C.c_int)]


HALO_FIELDS = (
    "M", "c", "z", "E", "rho_crit", "Delta_vir", "r_vir", "r_s", "rho_s",
    "x500", "r500", "M500", "F_star", "M_star", "x_star", "sigma2_vir", "P_s",
    "E_gi", "E_DM", "a", "x_f", "r_f", "rho0", "P0", "res_M", "res_P", "res_E",
    "chi", "D_A", "tau", "f_nt", "r_nt", "R_t")


class Halo(C.Structure):
    _fields_ = [(n, C.c_double) for n in HALO_FIELDS] + [
        ("status", C.c_int), ("n_sign_changes", C.c_int)]

    def as_dict(self):
        d = {n: getattr(self, n) for n in HALO_FIELDS}
        d["status"] = self.status
        d["n_sign_changes"] = self.n_sign_changes
        return d


def default_params(**kw) -> Params:
    """Table 1 of the paper plus the cosmology used by the synthetic workloads
    (Omega_m = 0.3, h = 0.7; Omega_b = 0.046 from the paper's WMAP9 set)."""
    d = dict(Omega_m=0.3, Omega_b=0.046, h=0.7, Gamma=1.2, eps_DM=0.0, eps_star=3.97e-6,
             f_star=0.026, S_star=0.12, alpha_nt=0.18, beta_nt=0.5, n_nt=0.8, X_H=0.76,
             trunc_r500=3.0, field_gas_frac=0.046 / 0.3, field_T=0.0, energy_sign=0)
    d.update(kw)
    p = Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.POINTER(Params)
        H = C.POINTER(Halo)
        sig = {
            "orc_chi": (C.c_double, [P, C.c_double]),
            "orc_DA": (C.c_double, [P, C.c_double]),
            "orc_tau": (C.c_double, [P, C.c_double]),
            "orc_m": (C.c_double, [C.c_double]),
            "orc_jeans_I_quad": (C.c_double, [C.c_double]),
            "orc_jeans_I_closed": (C.c_double, [C.c_double]),
            "orc_li2_neg": (C.c_double, [C.c_double]),
            "orc_f_nt": (C.c_double, [P, C.c_double]),
            "orc_halo_solve": (C.c_int, [P, C.c_double, C.c_double, C.c_double, H]),
            "orc_energy_quad": (C.c_double, [P, H, C.c_double]),
            "orc_energy_closed": (C.c_double, [P, H, C.c_double]),
            "orc_sigma2": (C.c_double, [P, H, C.c_double]),
            "orc_energy_residual_at": (C.c_double, [P, H, C.c_double]),
            "orc_profile": (None, [P, H, C.c_double, _D, _D]),
            "orc_los": (None, [P, H, C.c_double, _D, _D]),
            "orc_los_model": (C.c_double, [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]),
            "orc_hp_flat": (C.c_int, [P, C.c_int64, _D, _D, _D, _D, _D, _D, C.c_int, C.c_double,
                                      _D, _D, H]),
            "orc_hp_flat_solved": (None, [P, C.c_int64, H, _D, _D, _D, C.c_int, C.c_double, _D, _D]),
            "orc_hp_flat_pixels": (None, [P, C.c_int64, H, _D, _D, _D, C.c_double, C.c_int64,
                                          _I32, _I32, _D, _D]),
            "orc_ang2pix_ring": (C.c_int64, [C.c_int64, C.c_double, C.c_double]),
            "orc_pix2ang_ring": (None, [C.c_int64, C.c_int64, _D, _D]),
            "orc_hp_healpix": (C.c_int, [P, C.c_int64, _D, _D, _D, _D, _D, _D, C.c_int64, _D, _D, H]),
            "orc_hp_healpix_pixels": (None, [P, C.c_int64, H, _D, _D, _D, C.c_int64, C.c_int64,
                                             _I64, _D, _D]),
            "orc_W_sph": (C.c_double, [C.c_double]),
            "orc_w_sph": (C.c_double, [C.c_double]),
            "orc_knn_h": (None, [C.c_int64, _D, _D, _D, C.c_int, _D]),
            "orc_knn_h_query": (None, [C.c_int64, _I64, C.c_int64, _D, _D, _D, C.c_int, _D]),
            "orc_neff_h_query": (None, [C.c_int64, _I64, C.c_int64, _D, _D, _D, C.c_double, _D]),
            "orc_neff_at": (C.c_double, [C.c_int64, _D, _D, _D, C.c_int64, C.c_double]),
            "orc_pp_amplitudes": (None, [P, C.c_int64, _D, _D, _I32, _D, C.c_double, C.c_double,
                                         H, _D, _D]),
            "orc_pp_deposit": (None, [C.c_int64, _D, _D, _D, _D, _D, C.c_int, C.c_double, _D, _D]),
            "orc_pp_healpix_ngp": (None, [P, C.c_int64, _D, _D, _D, _D, C.c_double, C.c_int64, _I64, _D]),
            "orc_pp_healpix_ngp_map": (None, [P, C.c_int64, _D, _D, _D, _D, C.c_double, C.c_int64, _D, _D]),
            "orc_sizeof_halo": (C.c_int, []),
            "orc_sizeof_params": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        assert L.orc_sizeof_halo() == C.sizeof(Halo), "orc_halo layout mismatch"
        assert L.orc_sizeof_params() == C.sizeof(Params), "orc_params layout mismatch"
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- wrappers --
def chi(p, z):
    return lib().orc_chi(C.byref(p), float(z))


def D_A(p, z):
    return lib().orc_DA(C.byref(p), float(z))


def tau(p, z):
    return lib().orc_tau(C.byref(p), float(z))


def m_nfw(x):
    return lib().orc_m(float(x))


def jeans_I(x, closed=False):
    L = lib()
    return L.orc_jeans_I_closed(float(x)) if closed else L.orc_jeans_I_quad(float(x))


def li2_neg(x):
    return lib().orc_li2_neg(float(x))


def f_nt(p, z):
    return lib().orc_f_nt(C.byref(p), float(z))


def solve_halo(p, M, c, z) -> Halo:
    h = Halo()
    lib().orc_halo_solve(C.byref(p), float(M), float(c), float(z), C.byref(h))
    return h


def solve_halos(p, M, c, z):
    M, c, z = _f64(M), _f64(c), _f64(z)
    out = (Halo * len(M))()
    L = lib()
    for k in range(len(M)):
        L.orc_halo_solve(C.byref(p), M[k], c[k], z[k], C.byref(out[k]))
    return out


def halos_table(halos, fields=HALO_FIELDS + ("status",)):
    return {f: np.array([getattr(h, f) for h in halos]) for f in fields}


def energy(p, h: Halo, x_lo, closed=False):
    L = lib()
    f = L.orc_energy_closed if closed else L.orc_energy_quad
    return f(C.byref(p), C.byref(h), float(x_lo))


def sigma2(p, h: Halo, x):
    return lib().orc_sigma2(C.byref(p), C.byref(h), float(x))


def energy_residual_at(p, h: Halo, x_f):
    return lib().orc_energy_residual_at(C.byref(p), C.byref(h), float(x_f))


def profile(p, h: Halo, r):
    Pe, ne = C.c_double(), C.c_double()
    lib().orc_profile(C.byref(p), C.byref(h), float(r), C.byref(Pe), C.byref(ne))
    return Pe.value, ne.value


def los(p, h: Halo, rperp):
    ty, tb = C.c_double(), C.c_double()
    lib().orc_los(C.byref(p), C.byref(h), float(rperp), C.byref(ty), C.byref(tb))
    return ty.value, tb.value


def los_model(kind, par1, par2, rmax, rperp):
    """2 int f dl along the sight line at impact parameter rperp through a model profile ending at rmax
    (kind 0: uniform sphere; 1: beta model, par1 = beta, par2 = core radius; 2: 1 inside par1, par2
    outside), by the same integration as the halo projection."""
    return lib().orc_los_model(int(kind), float(par1), float(par2), float(rmax), float(rperp))


def hp_flat(p, cat, npix, pix_rad):
    """Full HP flat map [npix, npix] (row-major [j][i]) and the solved halos."""
    n = len(cat["M"])
    y = np.zeros(npix * npix)
    b = np.zeros(npix * npix)
    halos = (Halo * n)()
    arrs = [_f64(cat[k]) for k in ("M", "c", "z", "theta_x", "theta_y", "v_los")]
    lib().orc_hp_flat(C.byref(p), n, *[_dp(a) for a in arrs], int(npix), float(pix_rad),
                      _dp(y), _dp(b), halos)
    return y.reshape(npix, npix), b.reshape(npix, npix), halos


def hp_flat_solved(p, halos, cat, npix, pix_rad):
    n = len(halos)
    y = np.zeros(npix * npix)
    b = np.zeros(npix * npix)
    arrs = [_f64(cat[k]) for k in ("theta_x", "theta_y", "v_los")]
    lib().orc_hp_flat_solved(C.byref(p), n, halos, *[_dp(a) for a in arrs], int(npix),
                             float(pix_rad), _dp(y), _dp(b))
    return y.reshape(npix, npix), b.reshape(npix, npix)


def hp_flat_pixels(p, halos, cat, pix_rad, pi, pj):
    n = len(halos)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    oy = np.zeros(len(pi))
    ob = np.zeros(len(pi))
    arrs = [_f64(cat[k]) for k in ("theta_x", "theta_y", "v_los")]
    lib().orc_hp_flat_pixels(C.byref(p), n, halos, *[_dp(a) for a in arrs], float(pix_rad),
                             len(pi), pi.ctypes.data_as(_I32), pj.ctypes.data_as(_I32),
                             _dp(oy), _dp(ob))
    return oy, ob


def ang2pix_ring(nside, theta, phi):
    L = lib()
    th, ph = _f64(theta), _f64(phi)
    return np.array([L.orc_ang2pix_ring(int(nside), th[k], ph[k]) for k in range(len(th))],
                    dtype=np.int64)


def pix2ang_ring(nside, pix):
    L = lib()
    pix = np.asarray(pix, dtype=np.int64)
    th = np.empty(len(pix))
    ph = np.empty(len(pix))
    t, f = C.c_double(), C.c_double()
    for k in range(len(pix)):
        L.orc_pix2ang_ring(int(nside), int(pix[k]), C.byref(t), C.byref(f))
        th[k], ph[k] = t.value, f.value
    return th, ph


def hp_healpix(p, cat, nside):
    n = len(cat["M"])
    npx = 12 * nside * nside
    y = np.zeros(npx)
    b = np.zeros(npx)
    halos = (Halo * n)()
    arrs = [_f64(cat[k]) for k in ("M", "c", "z", "theta", "phi", "v_los")]
    lib().orc_hp_healpix(C.byref(p), n, *[_dp(a) for a in arrs], int(nside), _dp(y), _dp(b), halos)
    return y, b, halos


def hp_healpix_pixels(p, halos, cat, nside, pix):
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    oy = np.zeros(len(pix))
    ob = np.zeros(len(pix))
    arrs = [_f64(cat[k]) for k in ("theta", "phi", "v_los")]
    lib().orc_hp_healpix_pixels(C.byref(p), len(halos), halos, *[_dp(a) for a in arrs], int(nside),
                                len(pix), pix.ctypes.data_as(_I64), _dp(oy), _dp(ob))
    return oy, ob


def W_sph(x):
    return lib().orc_W_sph(float(x))


def w_sph(x):
    return lib().orc_w_sph(float(x))


def knn_h(X, Y, Z, k=32):
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    h = np.empty(len(X))
    lib().orc_knn_h(len(X), _dp(X), _dp(Y), _dp(Z), int(k), _dp(h))
    return h


def knn_h_query(qidx, X, Y, Z, k=32):
    """k-th nearest other point of X[qidx] among all points (brute force per query)."""
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    q = np.ascontiguousarray(qidx, dtype=np.int64)
    h = np.empty(len(q))
    lib().orc_knn_h_query(len(q), q.ctypes.data_as(_I64), len(X), _dp(X), _dp(Y), _dp(Z), int(k), _dp(h))
    return h


def neff_h_query(qidx, X, Y, Z, n_ngb=64.0):
    """Smoothing length of X[qidx] with effective neighbour number n_ngb (Sec. 3.4): the root of
    (32/3) sum_j W(r_ij / h) = n_ngb over all points, the point itself included."""
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    q = np.ascontiguousarray(qidx, dtype=np.int64)
    h = np.empty(len(q))
    lib().orc_neff_h_query(len(q), q.ctypes.data_as(_I64), len(X), _dp(X), _dp(Y), _dp(Z), float(n_ngb), _dp(h))
    return h


def neff_at(X, Y, Z, i, h):
    """N_eff(h) = (32/3) sum_j W(|x_j - x_i| / h) of point i."""
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    return lib().orc_neff_at(len(X), _dp(X), _dp(Y), _dp(Z), int(i), float(h))


def pp_amplitudes(p, halos, z, v, halo_id, r_i, M_p, pix_rad):
    z, v, r_i = _f64(z), _f64(v), _f64(r_i)
    hid = np.ascontiguousarray(halo_id, dtype=np.int32)
    ay = np.empty(len(z))
    ab = np.empty(len(z))
    hal = halos if halos is not None and len(halos) else (Halo * 1)()
    lib().orc_pp_amplitudes(C.byref(p), len(z), _dp(z), _dp(v), hid.ctypes.data_as(_I32), _dp(r_i),
                            float(M_p), float(pix_rad), hal, _dp(ay), _dp(ab))
    return ay, ab


def pp_deposit(thx, thy, H, amp_y, amp_b, npix, pix_rad):
    arrs = [_f64(a) for a in (thx, thy, H, amp_y, amp_b)]
    y = np.zeros(npix * npix)
    b = np.zeros(npix * npix)
    lib().orc_pp_deposit(len(arrs[0]), *[_dp(a) for a in arrs], int(npix), float(pix_rad), _dp(y), _dp(b))
    return y.reshape(npix, npix), b.reshape(npix, npix)


def pp_healpix_ngp(p, theta, phi, z, v, M_p, nside):
    """Per-particle (RING pixel, kSZ amplitude) of the all-sky nearest-pixel paste (App. A)."""
    arrs = [_f64(a) for a in (theta, phi, z, v)]
    n = len(arrs[0])
    pix = np.empty(n, dtype=np.int64)
    amp = np.empty(n)
    lib().orc_pp_healpix_ngp(C.byref(p), n, *[_dp(a) for a in arrs], float(M_p), int(nside),
                             pix.ctypes.data_as(_I64), _dp(amp))
    return pix, amp


def pp_healpix_ngp_map(p, theta, phi, z, v, M_p, nside):
    """All-sky kSZ map by nearest-pixel assignment (App. A) and the per-pixel sum of |b_i|."""
    arrs = [_f64(a) for a in (theta, phi, z, v)]
    b = np.zeros(12 * nside * nside)
    babs = np.zeros(12 * nside * nside)
    lib().orc_pp_healpix_ngp_map(C.byref(p), len(arrs[0]), *[_dp(a) for a in arrs], float(M_p), int(nside),
                                 _dp(b), _dp(babs))
    return b, babs


# constants used by the tests' closed forms (the oracle's own copies, CODATA 2018 / IAU)
SIGMA_T = 6.6524587321e-25
ME_C2 = 8.1871057769e-7
C_CGS = 2.99792458e10
M_P = 1.67262192369e-24
G_CGS = 6.67430e-8
MSUN = 1.988409870698051e33
MPC = 3.0856775814913673e24


def pp_flat(p, halos, parts, M_p, npix, pix_rad, k=32):
    """Full PP map (Sec. 3.4): smoothing lengths by brute-force k-NN in comoving
    Cartesian coordinates, per-particle amplitudes, separable SPH deposit.
    ``parts`` arrays may be float32 (they are promoted exactly to float64).
    Returns y, b maps [npix, npix], comoving h, angular H."""
    z = _f64(parts["z"])
    tx, ty = _f64(parts["theta_x"]), _f64(parts["theta_y"])
    chis = np.array([chi(p, zz) for zz in z])
    X, Y, Z = chis * tx, chis * ty, chis
    h = knn_h(X, Y, Z, k)
    H = h / chis
    ay, ab = pp_amplitudes(p, halos, z, parts["v_los"], parts["halo_id"], parts["r_i"], M_p, pix_rad)
    y, b = pp_deposit(tx, ty, H, ay, ab, npix, pix_rad)
    return y, b, h, H, ay, ab


def _solve_chunk(args):
    """Worker of solve_halos_parallel: plain tuples cross the process boundary."""
    pd, M, c, z = args
    p = default_params(**pd)
    out = []
    for k in range(len(M)):
        h = solve_halo(p, M[k], c[k], z[k])
        out.append(tuple(getattr(h, f) for f in HALO_FIELDS) + (h.status, h.n_sign_changes))
    return out


def solve_halos_parallel(p, M, c, z, workers=None):
    """solve_halos over a pool of fresh single-threaded processes (spawned, so a caller that has
    initialised a GPU is never forked).  Returns the same ctypes array of Halo as solve_halos."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    M, c, z = _f64(M), _f64(c), _f64(z)
    n = len(M)
    workers = workers or min(16, os.cpu_count() or 1)
    if n < 64 or workers <= 1:
        return solve_halos(p, M, c, z)
    pd = {f: getattr(p, f) for f, _ in Params._fields_ if f != "pad_"}
    chunks = [(pd, M[a:a + 256], c[a:a + 256], z[a:a + 256]) for a in range(0, n, 256)]
    out = (Halo * n)()
    k = 0
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for res in ex.map(_solve_chunk, chunks):
            for vals in res:
                h = out[k]
                for f, v in zip(HALO_FIELDS, vals[:len(HALO_FIELDS)]):
                    setattr(h, f, v)
                h.status, h.n_sign_changes = vals[-2], vals[-1]
                k += 1
    return out
