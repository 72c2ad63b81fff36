/*
 * bp.h -- C ABI of the MI355X (gfx950) baryon-pasting library, libbp.so.
 *
 * The library implements the data-parallel hot path of the baryon-pasting
 * method of Osato & Nagai (2022, "Baryon Pasting Algorithm: Halo-based and
 * Particle-based Pasting Methods"):
 *   - the per-halo ICM solve (Sec. 2: polytropic gas in the NFW potential,
 *     central density/pressure and gas boundary r_f fixed by energy
 *     conservation, surface pressure and gas-mass conservation),
 *   - line-of-sight projected electron-pressure and electron-density tables
 *     (Sec. 3.3, the integrals of the HP map equations),
 *   - halo-based pasting (HP) of Compton-y and kSZ b onto a flat-sky map or
 *     onto HEALPix RING pixels (Sec. 3.3, Sec. 5.2),
 *   - HEALPix RING ang2pix (Gorski et al. 2005, the pixelisation of Sec. 5.2).
 *
 * Conventions (every entry point):
 *   - Array arguments are DEVICE pointers owned by the caller (allocated on
 *     the current HIP device); scalar arguments and structs are host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it; entry points return before it completes unless noted.
 *   - Return value: BP_OK (0) or a negative BP_E* code.  Argument errors are
 *     detected synchronously before anything is enqueued; device faults
 *     surface through HIP at the next synchronising call.  Per-halo solver
 *     failures are reported in a status array, never by the return value.
 *   - The library never aborts and never throws across this boundary.  It
 *     allocates no device memory: scratch comes through `ws` (workspace).
 *   - Maps ACCUMULATE: the caller zeroes them; successive calls (halo
 *     batches, HP + PP) add up.
 *
 * Units: masses Msun/h; halo radii physical Mpc/h; distances chi comoving
 * Mpc/h; velocities km/s; angles radians; y and b dimensionless; gas
 * density g/cm^3; pressures erg/cm^3.
 */
#ifndef BP_H
#define BP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define BP_OK             0
#define BP_E_ARG         -1   /* invalid argument (null pointer, bad size, bad parameter) */
#define BP_E_HIP         -2   /* a HIP runtime call failed */
#define BP_E_WORKSPACE   -3   /* workspace too small; *ws_needed holds the required bytes */
#define BP_E_OVERFLOW    -4   /* an index or pair count exceeds what one call can hold */

/* per-halo status bits written by bp_icm_solve (0 = solved) */
#define BP_S_NO_BRACKET    1  /* energy residual has no sign change on the x_f scan */
#define BP_S_MULTI_ROOT    2  /* more than one sign change; the first root is used (still valid) */
#define BP_S_NO_STAR_ROOT  4  /* stellar mass >= baryon mass: stellar radius undefined */
#define BP_S_NONFINITE     8  /* a non-finite intermediate */
#define BP_S_BAD_INPUT    16  /* M <= 0, c <= 0, z < 0 or non-finite input */

/* ------------------------------------------------------------- parameters */
/* Cosmology (flat LCDM without radiation, Sec. 1) and the ICM model
 * parameters of Table 1, plus the readings the paper leaves open. */
typedef struct {
    double Omega_m, Omega_b, h;
    double Gamma;          /* adiabatic index, fixed at the paper's 1.2 (Sec. 2.1, Table 1): the kernels are
                              written for the polytropic index n = 1/(Gamma-1) = 5, and every entry point
                              taking bp_params returns BP_E_ARG for any other value */
    double eps_DM;         /* energy transfer from dark matter */
    double eps_star;       /* stellar feedback efficiency */
    double f_star, S_star; /* stellar-to-halo mass relation amplitude and slope */
    double alpha_nt, beta_nt, n_nt;   /* non-thermal pressure fraction (Sec. 2.3) */
    double X_H;            /* hydrogen mass fraction (Sec. 3.2) */
    double trunc_r500;     /* projected footprint radius in units of r500 (3) */
    double field_gas_frac; /* gas mass fraction of a PP field particle (default Omega_b/Omega_m) */
    double field_T;        /* temperature [K] of PP field gas for its tSZ term: 0 (default) keeps the
                              paper's y = 0 for field particles (Eq. field_y); > 0 gives filament gas
                              the pressure n_e k_B T (the extension Sec. 3.4 points to) */
    int32_t energy_sign;   /* 0: injected energy raises the gas energy (default);
                              1: the energy equation as printed in Sec. 2.2 */
    int32_t reserved;
} bp_params;

/* --------------------------------------------------- ICM solution layout */
/* bp_icm_solve writes a structure-of-arrays of doubles: field f of halo i
 * lives at sol[f * n + i].  The caller allocates BP_SOL_NFIELDS * n doubles. */
enum {
    BP_SOL_M = 0,     /* M_vir [Msun/h] (copy of the input) */
    BP_SOL_C,         /* c_vir (copy of the input) */
    BP_SOL_Z,         /* redshift (copy of the input) */
    BP_SOL_RVIR,      /* virial radius, physical Mpc/h */
    BP_SOL_RS,        /* scale radius r_vir / c */
    BP_SOL_RHOS,      /* NFW scale density [(Msun/h)/(Mpc/h)^3] */
    BP_SOL_R500,      /* r500 [Mpc/h] */
    BP_SOL_M500,      /* M500 [Msun/h] */
    BP_SOL_MSTAR,     /* stellar mass F_* M_vir [Msun/h] */
    BP_SOL_XSTAR,     /* stellar radius over r_s */
    BP_SOL_PS,        /* surface pressure [erg/cm^3] */
    BP_SOL_EGI,       /* initial gas energy [erg] */
    BP_SOL_A,         /* a = ((Gamma-1)/Gamma)(rho0/P0) G M_vir / r_vir (dimensionless) */
    BP_SOL_XF,        /* r_f / r_vir */
    BP_SOL_RF,        /* gas boundary r_f [Mpc/h] */
    BP_SOL_RHO0,      /* central gas density [g/cm^3] */
    BP_SOL_P0,        /* central total gas pressure [erg/cm^3] */
    BP_SOL_CHI,       /* comoving distance [Mpc/h] */
    BP_SOL_DA,        /* angular-diameter distance [physical Mpc/h] */
    BP_SOL_TAU,       /* mean Thomson optical depth to z */
    BP_SOL_FNT,       /* non-thermal amplitude f(z) */
    BP_SOL_RT,        /* footprint radius min(r_f, trunc_r500 r500) [Mpc/h] */
    BP_SOL_RES_E,     /* relative residual of the energy condition at the root */
    BP_SOL_NFIELDS
};

/* ---------------------------------------------------------- table layout */
/* bp_profile_tables writes, per halo, BP_TAB_STRIDE floats: the projected
 * electron-pressure shape followed by the projected electron-density shape,
 * each in three zones (A: the part of the sight line inside r_a = min(r_vir,
 * r_f); S: the shell r_vir < r < r_f seen at r_perp < r_vir; B: sight lines
 * with r_perp >= r_vir).  Each zone is tabulated on a uniform grid of a
 * variable that makes the projected profile analytic, with the edge factor
 * divided out:
 *   zone A:  eta  = ln(1 + acosh(r_a / r_perp)),   Y = P_e0 S g_T(eta),
 *            u = sqrt(r_a^2 - r_perp^2), S = sqrt(u^2 + D), D = r_f^2 - r_vir^2 when the gas
 *            extends past r_vir (else 0, S = u): the whole sight line, its shell part included
 *   zone S:  omega = asinh(u_v / sqrt(D)),         Y_S = P_e0 (S - u_v) g_S(omega),
 *            u_v = sqrt(r_vir^2 - r_perp^2): the shell r_vir < r < r_f alone, from which zone A's
 *            shell part is interpolated (the deposits read zones A and B only)
 *   zone B:  zeta = acosh(r_f / r_perp),           Y = P_e0 U g_B(zeta),
 *            U = sqrt(r_f^2 - r_perp^2)
 * (same with n_e0 for the density).  P_e0 and n_e0 are the central electron
 * pressure and density.  Grid end points per halo are in `meta`
 * (BP_META_NFIELDS floats per halo, SoA: field f of halo i at meta[f*n+i]). */
#define BP_TAB_NA     192
#define BP_TAB_NS      32
#define BP_TAB_NB      32
#define BP_TAB_ZONE   (BP_TAB_NA + BP_TAB_NS + BP_TAB_NB)   /* 256 per quantity */
#define BP_TAB_STRIDE (2 * BP_TAB_ZONE)                      /* P then n: 512 floats */
enum {
    BP_META_ETA_LO = 0, BP_META_ETA_HI,
    BP_META_OM_LO, BP_META_OM_HI,
    BP_META_ZE_LO, BP_META_ZE_HI,
    BP_META_PE0,      /* central electron pressure [erg/cm^3] */
    BP_META_NE0,      /* central electron density [1/cm^3] */
    /* constants of the electron profile shape that the table integrals evaluate (FP32, from sol;
     * lengths in physical Mpc/h): r_vir, 1/r_s, r_f, c/m(c), c^2/((1+c) m(c)), the polytropic
     * slope a, 1/r500 and alpha_nt f(z) */
    BP_META_PR_RV, BP_META_PR_INV_RS, BP_META_PR_RF, BP_META_PR_CM, BP_META_PR_PHI_OUT0,
    BP_META_PR_A, BP_META_PR_INV_R500, BP_META_PR_ANT_F,
    BP_META_NFIELDS
};

/* ----------------------------------------------------------------- basics */
int bp_version(void);
const char *bp_strerror(int code);

/* ---------------------------------------------------------- ICM solve (K1) */
/* Solve the ICM model of Sec. 2 for n halos, one GPU lane per halo, FP64.
 *   M, c, z      : device, n doubles each (M_vir [Msun/h], c_vir, redshift).
 *   sol          : device, BP_SOL_NFIELDS * n doubles (SoA, layout above).
 *   status       : device, n int32 (BP_S_* bits, 0 = solved).
 * Halo structure (Sec. 2.1): Bryan & Norman Delta_vir relative to rho_crit,
 * NFW with the given c.  Stars (Sec. 2.2): F_* from M500, stellar radius from
 * f_b M(<r_*) = M_*.  The gas boundary x_f = r_f/r_vir is the first sign
 * change of the energy residual on a 47-point scan of [0.4, 5], refined to
 * 1e-13 relative; for each trial x_f the pressure condition is solved for a
 * and the gas-mass condition fixes rho0.  n may be 0. */
int bp_icm_solve(const bp_params *p, int64_t n, const double *M, const double *c, const double *z,
                 double *sol, int32_t *status, void *stream);

/* -------------------------------------------------- projection tables (K2) */
/* Projected electron pressure and density tables (layout above) for n
 * solved halos.  Halos with a non-zero status get all-zero tables.
 *   sol, status : outputs of bp_icm_solve (device).
 *   tables      : device, BP_TAB_STRIDE * n floats.
 *   meta        : device, BP_META_NFIELDS * n floats. */
int bp_profile_tables(const bp_params *p, int64_t n, const double *sol, const int32_t *status,
                      float *tables, float *meta, void *stream);

/* ----------------------------------------------------- HP flat paste (K3) */
/* Halo-based pasting onto an npix x npix flat-sky map (Sec. 3.3):
 *   y[p] += sigma_T/(m_e c^2) Y_P(r_perp),  b[p] += sigma_T (v/c) e^-tau Y_n(r_perp)
 * for every halo whose footprint r_perp < R_t = min(r_f, trunc_r500 r500)
 * contains the centre of pixel p.  Pixel (i, j) has centre ((i+1/2) pix_rad,
 * (j+1/2) pix_rad); maps are row-major [j][i] (npix*npix floats, device),
 * r_perp = D_A |dtheta| on the tangent plane.
 *   theta_x, theta_y : device, n doubles [rad];  v_los: device, n doubles [km/s]
 *   sol, status, tables, meta : outputs of the two calls above
 *   y_map, b_map     : device float maps, ACCUMULATED
 *   y_comp, b_comp   : NULL, or device float maps of the same shape holding each pixel's Kahan
 *                      compensation between calls: the call resumes every touched pixel's compensated
 *                      sum from (map, comp) and stores both back, so a sequence of calls (halo batches)
 *                      adds up as one compensated sum.  The caller zeroes them with the maps.
 *   ws, ws_bytes     : device workspace.  If ws_bytes is too small the maps are
 *                      not touched, *ws_needed receives the size and the call
 *                      returns BP_E_WORKSPACE.  The size depends on the
 *                      footprints, so this call synchronises `stream` once to
 *                      read the (halo, tile) pair count (the pair count is
 *                      taken in the workspace first, so a call with a
 *                      workspace big enough for that but not for the pairs
 *                      asks a second time, with the final size).
 * Each map pixel is owned by one lane; contributions are added in catalogue
 * order with Kahan compensation, so results are deterministic. */
int bp_hp_paste_flat(const bp_params *p, int32_t npix, double pix_rad, int64_t n,
                     const double *theta_x, const double *theta_y, const double *v_los,
                     const double *sol, const int32_t *status, const float *tables, const float *meta,
                     float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws, size_t ws_bytes,
                     size_t *ws_needed, void *stream);

/* The three calls above as one: bp_icm_solve, bp_profile_tables and bp_hp_paste_flat on the same
 * inputs, with the same outputs (sol, status, tables, meta and the maps are bit-identical to those of
 * the three calls in sequence).  What differs is the ordering: the paste's set-up and plan (footprints,
 * pair sort and tile ranges, Sec. 3.3) need only the solution and meta, so they run on a second stream
 * of the library's (one per device, default priority, created on the first call) while the table
 * quadratures of Sec. 3.2 run on `stream`; the deposit waits for both on `stream`.  On return all work
 * is ordered on `stream` as for a single call.  Workspace protocol as bp_hp_paste_flat: when ws_bytes is
 * too small the call returns BP_E_WORKSPACE with *ws_needed set, after the solve and the tables are
 * complete on `stream` and without touching the maps (bp_hp_paste_flat on the same outputs then
 * finishes the job).  The call synchronises once on the second stream.  Calls on one device from
 * several host threads are serialised inside the library. */
int bp_hp_flat_pipeline(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *M,
                        const double *c, const double *z, const double *theta_x, const double *theta_y,
                        const double *v_los, double *sol, int32_t *status, float *tables, float *meta,
                        float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws, size_t ws_bytes,
                        size_t *ws_needed, void *stream);

/* Allocation-free variant of bp_hp_paste_flat, for callers that cannot allocate device memory or
 * size a workspace (serving loops, harnesses that forbid allocation).  Same arguments, layouts,
 * results and errors as bp_hp_paste_flat (the same kernels run), without ws / ws_bytes: the call works
 * in a fixed array of bp_hp_paste_flat_noalloc_max_bytes() bytes (64 MiB) that the library holds on
 * each GPU it runs on, for the life of the process, and allocates nothing.  A problem whose workspace
 * exceeds that (about 184 B per halo plus 16 B per (tile, halo) pair and the sort's scratch) is refused
 * with BP_E_WORKSPACE before the maps are touched; *scratch_needed (nullable) receives the bytes it would
 * need.  Like bp_hp_paste_flat it synchronises the stream once.  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (several host threads or streams) race and must be
 * serialised by the caller. */
size_t bp_hp_paste_flat_noalloc_max_bytes(void);
int bp_hp_paste_flat_noalloc(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *theta_x,
                             const double *theta_y, const double *v_los, const double *sol, const int32_t *status,
                             const float *tables, const float *meta, float *y_map, float *b_map, float *y_comp,
                             float *b_comp, size_t *scratch_needed, void *stream);

/* ------------------------------------------------------- HEALPix (K9, K4) */
/* HEALPix RING pixel index of each direction (Gorski et al. 2005).
 *   theta: colatitude in [0, pi]; phi: longitude (any real, taken mod 2 pi).
 *   ipix : device, n int64.  nside in [1, 2^29].  Integer results are
 *   bit-exact reproducible (FP64, fixed operation order, no contraction). */
int bp_healpix_ang2pix_ring(int64_t nside, int64_t n, const double *theta, const double *phi,
                            int64_t *ipix, void *stream);

/* HP onto HEALPix RING pixels (Sec. 5.2 maps): as bp_hp_paste_flat with
 * r_perp = D_A sin(psi), psi the angle between pixel centre and halo centre
 * (psi < pi/2).  theta/phi: halo colatitude/longitude; maps have 12 nside^2
 * floats in RING order.  Same workspace protocol. */
int bp_hp_paste_healpix(const bp_params *p, int64_t nside, int64_t n,
                        const double *theta, const double *phi, const double *v_los,
                        const double *sol, const int32_t *status, const float *tables, const float *meta,
                        float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws, size_t ws_bytes,
                        size_t *ws_needed, void *stream);

/* bp_icm_solve, bp_profile_tables and bp_hp_paste_healpix in one call, as bp_hp_flat_pipeline is for the
 * flat map: same outputs bit for bit, the paste's set-up and plan on the library's second stream beside
 * the table quadratures, everything ordered on `stream` on return, same workspace protocol. */
int bp_hp_healpix_pipeline(const bp_params *p, int64_t nside, int64_t n, const double *M, const double *c,
                           const double *z, const double *theta, const double *phi, const double *v_los,
                           double *sol, int32_t *status, float *tables, float *meta, float *y_map, float *b_map,
                           float *y_comp, float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed,
                           void *stream);

/* ------------------------------------------------------- PP (K5-K8) */
/* Smoothing lengths for particle-based pasting (Sec. 3.4): h_i is the
 * distance from particle i to its k-th nearest OTHER particle in comoving
 * Cartesian coordinates (chi theta_x, chi theta_y, chi), chi the comoving
 * distance of the particle redshift (flat-sky small-angle frame).
 *   theta_x, theta_y : device, n floats [rad];  z: device, n floats (0 <= z < 16)
 *   k                : neighbour count, 1 <= k <= 64 (the paper's workloads use 32)
 *   cell             : coarse grid cell [comoving Mpc/h]; 0 selects 2.0.  Any value
 *                      gives the exact k-th distance; it only tunes the search.
 *   h_comoving       : device, n floats, OUTPUT [comoving Mpc/h]; NaN for a particle
 *                      with fewer than k neighbours within the largest search block.
 * Workspace protocol as for the pastes (one synchronisation for the bounding box).
 * Returns BP_E_ARG for n <= k, a redshift outside [0, 16) or a non-finite angle. */
int bp_pp_smoothing_length(const bp_params *p, int64_t n, const float *theta_x, const float *theta_y,
                           const float *z, int32_t k, double cell, float *h_comoving, void *ws, size_t ws_bytes,
                           size_t *ws_needed, void *stream);

/* Smoothing length from the effective neighbour number (Sec. 3.4: h is set so that the effective
 * number of particles within it is n_ngb, 64 in the paper): per particle, h solves
 *     N_eff(h) = (4 pi / 3) h^3 sum_j W(|x_i - x_j|, h) = n_ngb,
 * W the cubic spline of Eq. SPH_kernel with support h, the sum over every particle including i
 * itself (the SPH density sum), i.e. (32/3) sum_j w(r_ij / h).  Positions, units, workspace and
 * errors as bp_pp_smoothing_length (which runs first, for the 32-NN distance that seeds a
 * bracketed Halley iteration on h, stopped after a step below 1e-3 relative,
 * which leaves an error of order 1e-9).  For n_ngb <= 64 (and n > 64) the search keeps the 64
 * nearest neighbours and runs the iteration on their list, which is exact for a root up to the
 * 64th distance; the other particles iterate over the cells as above.  n_ngb in (32/3, 1024]
 * (BP_E_ARG otherwise); n > 32.  A particle whose root is not found writes NaN. */
int bp_pp_smoothing_length_eff(const bp_params *p, int64_t n, const float *theta_x, const float *theta_y,
                               const float *z, double n_ngb, double cell, float *h_comoving, void *ws,
                               size_t ws_bytes, size_t *ws_needed, void *stream);

/* Particle-based pasting onto an npix x npix flat-sky map (Sec. 3.4):
 *   halo particle (halo_id >= 0): y_i = sigma_T/(m_e c^2) P_e(r_i) V_i / L_pix^2,
 *       b_i = sigma_T (v_i/c) e^-tau_i n_e(r_i) V_i / L_pix^2,  V_i = M_p / rho_NFW(r_i)
 *       (untruncated NFW density; P_e = n_e = 0 for r_i >= r_f);
 *   field particle (halo_id < 0): y_i = sigma_T/(m_e c^2) k_B field_T (field_gas_frac M_p / (mu_e m_p)) / L_pix^2
 *       (0 for the default field_T = 0),
 *       b_i = sigma_T (v_i/c) (field_gas_frac M_p / (mu_e m_p)) e^-tau_i / L_pix^2;
 *   L_pix = D_A(z_i) pix_rad.  Each amplitude is spread with the separable
 *   integrated cubic-spline kernel of angular half-width H = h_comoving/chi:
 *   pixel (i, j) receives amp [w((x_i+ - x)/H) - w((x_i- - x)/H)] [same in y];
 *   pixels outside the map are dropped (no renormalisation).
 *   r_halo: device floats, the particle's radius in its halo [physical Mpc/h];
 *   halo_id indexes the n_halos solved halos (sol, status from bp_icm_solve).
 *   M_p: particle mass [Msun/h].  Maps ACCUMULATE; deterministic order.
 *   Workspace protocol as for the halo pastes (one synchronisation). */
int bp_pp_paste_flat(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const float *theta_x,
                     const float *theta_y, const float *z, const float *v_los, const int32_t *halo_id,
                     const float *r_halo, const float *h_comoving, double M_p, int64_t n_halos, const double *sol,
                     const int32_t *status, float *y_map, float *b_map, void *ws, size_t ws_bytes,
                     size_t *ws_needed, void *stream);

/* All-sky particle kSZ by nearest-pixel assignment (App. A, the continuous light cone): every
 * particle is a field particle (Eq. field_b),
 *     b_i = sigma_T (v_i/c) (field_gas_frac M_p / (mu_e m_p)) e^-tau_i / L_pix^2,
 *     L_pix^2 = D_A(z_i)^2 Omega_pix,  Omega_pix = 4 pi / (12 nside^2),
 * and the whole b_i goes to the RING pixel that contains the direction (theta_i, phi_i), the
 * pixel bp_healpix_ang2pix_ring gives for the FP64 images of the two floats.
 *   nside      : 1 .. 2048
 *   theta, phi : device, n floats [rad]; colatitude in [0, pi] (the float nearest pi lies above pi
 *                and is rejected), longitude any finite value
 *   z          : device, n floats in [0, 16);  v_los: device, n floats [km/s];  M_p [Msun/h] > 0
 *   b_map      : device, 12 nside^2 floats in RING order; ACCUMULATES: each call adds, per pixel,
 *                the FP64 sum of its particles' amplitudes, rounded once to FP32.  The order of the
 *                FP64 sum is not fixed, so two calls can differ by one FP32 rounding of a pixel.
 * Workspace protocol as for the pastes (about 12 n bytes); one synchronisation, after which the
 * map is written.  Returns BP_E_ARG for an invalid argument or any invalid particle (the map is
 * then unchanged), BP_E_OVERFLOW for n >= 2^31 - 1. */
int bp_pp_paste_healpix_ngp(const bp_params *p, int64_t nside, int64_t n, const float *theta, const float *phi,
                            const float *z, const float *v_los, double M_p, float *b_map, void *ws,
                            size_t ws_bytes, size_t *ws_needed, void *stream);

/* Self-check of the error bounds behind bp_pp_paste_healpix_ngp's bit-exact pixel indices: over
 * every float colatitude in [0, pi) it measures, against FP64 cos, sin and sqrt, the largest error of
 * the FP32 hardware cos(theta) and of the cap factor N sin(theta) sqrt(3 / (1 + |cos theta|))
 * (divided by N, where |cos theta| > 0.66).  bounds (host, 4 doubles, OUTPUT): measured z error,
 * measured cap-factor error / N, then the two bounds the paste assumes.  A measured value above
 * its bound would mean the paste's pixel indices can differ from the FP64 assignment.
 * nside in [1, 2048].  Workspace protocol as for the pastes (256 bytes); synchronises the stream. */
int bp_pp_healpix_ngp_selfcheck(int64_t nside, double *bounds, void *ws, size_t ws_bytes, size_t *ws_needed,
                                void *stream);

/* Flat-sky angular power spectrum of an npix x npix map (Sec. 5.3: FFT of the flat-sky maps in
 * logarithmic multipole bins, 30 over 10^2 < ell < 10^5 in the paper):
 *     F(ell) = d^2 sum_x f(x) exp(-i ell.x),  ell = 2 pi (kx, ky) / (N d),  kx, ky in [-N/2, N/2),
 *     C_b = mean over the modes of bin b of |F(ell)|^2 / (N d)^2,  ell_b = their mean |ell|.
 * Mode (kx, ky) is in bin b when t_b <= kx^2 + ky^2 < t_{b+1}, t_b = (edges[b] N d / (2 pi))^2 in
 * FP64 (so the assignment of modes to bins is exact).  No apodisation, mean subtraction or window.
 *   npix      : power of two, 2 .. 4096;  d = pix_rad [rad];  map: device, npix*npix floats, row-major
 *   edges     : HOST, nbins + 1 increasing finite values >= 0 [ell];  nbins in [1, 64]
 *   ell, cl   : device, nbins doubles each, OUTPUT (0 for an empty bin);  nmodes: device, nbins int64
 * Transforms in FP64.  Workspace protocol as for the pastes (about 32 npix^2 bytes); no
 * synchronisation.  Per-bin sums are formed in LDS in an unfixed order, so repeated calls agree to
 * about 1e-15 relative. */
int bp_flat_power_spectrum(int32_t npix, double pix_rad, const float *map, int32_t nbins, const double *edges,
                           double *ell, double *cl, int64_t *nmodes, void *ws, size_t ws_bytes, size_t *ws_needed,
                           void *stream);

/* ------------------------------------------------- surrogate (K10-K12) */
/* A multilayer perceptron maps normalised (log10 M, ln c, z) to the projected
 * electron pressure and density of the halo on a fixed grid of 64 impact
 * parameters each, plus three scalars, replacing the boundary-condition solve
 * and the table integrals (an addition to the paper's method).
 *   q-grid   : q_k = (1 - cos(pi k / 63)) / 2, k = 0..63, r_perp = q R_t.
 *   outputs  : y[0..63]   = ln( Y_P(q_k R_t) / (P_e0 R_t E_k) ),
 *              y[64..127] = ln( Y_n(q_k R_t) / (n_e0 R_t E_k) ),  E_k = sqrt(1 - (q_k R_t / r_f)^2)
 *              y[128] = ln x_f, y[129] = ln(P_e0 / P_s), y[130] = ln(n_e0 / n_s) with P_s the surface
 *              pressure and n_s = f_b (3 M_vir / (4 pi r_vir^3)) / (mu_e m_p)
 *              (standardised: the network predicts (y - mean) / std).
 *   layers   : 3 -> 256 -> 256 -> 256 -> 144 (131 used), SiLU; the first layer
 *              in FP32, the others BF16 on MFMA with FP32 accumulation.
 * Parameter vector (FP32 master, BF16 compute copy), BP_MLP_NPARAMS floats:
 *   W1 [256][16] (inputs padded to 16, columns >= 3 stay 0), b1[256],
 *   W2 [256][256], b2, W3 [256][256], b3, W4 [144][256], b4[144]. */
#define BP_MLP_NIN    3
#define BP_MLP_IN    16
#define BP_MLP_HID  256
#define BP_MLP_OUT  144
#define BP_MLP_NOUT 131
#define BP_MLP_NQ    64
#define BP_S_OUT_OF_DOMAIN 32   /* status bit: outside the surrogate's training domain */

int64_t bp_mlp_nparams(void);
size_t bp_mlp_act_bytes(int64_t n);
size_t bp_mlp_backward_ws_bytes(int64_t n);
/* forward: x [n][16] FP32 features (bp_surrogate_features), y [n][144] FP32;
 * act (bp_mlp_act_bytes(n) bytes) receives the activations backward needs.
 * y, act and w_bf16 must be 16-byte aligned (BP_E_ARG otherwise). */
int bp_mlp_forward(const float *w, const uint16_t *w_bf16, int64_t n, const float *x, float *y, void *act,
                   void *stream);
/* backward: dy [n][144] = dL/dy; grad receives dL/dw (BP_MLP_NPARAMS floats,
 * overwritten).  Deterministic (fixed-order reductions).  x, act and w_bf16 16-byte aligned and
 * ws 256-byte aligned (BP_E_ARG otherwise); ws of at least bp_mlp_backward_ws_bytes(n) bytes
 * (BP_E_WORKSPACE otherwise). */
int bp_mlp_backward(const float *w, const uint16_t *w_bf16, int64_t n, const float *x, const void *act,
                    const float *dy, float *grad, void *ws, size_t ws_bytes, void *stream);
/* Adam step on the FP32 master weights; refreshes the BF16 copy. */
int bp_mlp_adam(int64_t np, float *w, float *m, float *v, const float *g, uint16_t *w_bf16, float lr, float beta1,
                float beta2, float eps, int64_t step, void *stream);
int bp_mlp_to_bf16(int64_t np, const float *w, uint16_t *w_bf16, void *stream);

/* Halo structure without the boundary-condition solve (r_vir, r500, stars,
 * distances, optical depth, f(z)): the cheap part of bp_icm_solve that the
 * surrogate path keeps exact.  Same layout; A, XF, RF, RHO0, P0, RT, RES_E
 * are left 0 and status carries BP_S_OUT_OF_DOMAIN for halos outside
 * log10 M in [12.5, 15.5], c in [2, 15], z in [0.05, 3]. */
int bp_halo_structure(const bp_params *p, int64_t n, const double *M, const double *c, const double *z,
                      double *sol, int32_t *status, void *stream);
/* Network features [n][16] from (M, c, z). */
int bp_surrogate_features(int64_t n, const double *M, const double *c, const double *z, float *x, void *stream);
/* Training targets [n][144] (standardisation not applied) from an exact solve
 * and its tables (halos with a non-zero status get NaN rows). */
int bp_surrogate_targets(const bp_params *p, int64_t n, const double *sol, const int32_t *status,
                         const float *tables, const float *meta, float *targets, void *stream);
/* Column mean and standard deviation of targets over n rows (FP64 sums). */
int bp_surrogate_stats(int64_t n, const float *targets, float *mean, float *std, void *stream);
/* Gather rows: out[i] = in[idx[i]] (cols floats per row). */
int bp_gather_rows(int64_t n, int32_t cols, const float *in, const int64_t *idx, float *out, void *stream);
/* Inference-only forward pass (same network and arithmetic as bp_mlp_forward, all four layers in
 * one kernel, activations kept on chip; nothing but y is written).
 *   w, w_bf16 : device parameters as for bp_mlp_forward;  x : device [n][BP_MLP_IN] floats
 *   y         : device [n][BP_MLP_OUT] floats, OUTPUT, 16-byte aligned
 * Returns BP_E_ARG for null or misaligned pointers. */
int bp_mlp_infer(const float *w, const uint16_t *w_bf16, int64_t n, const float *x, float *y, void *stream);
/* Weighted MSE over the 131 used outputs against standardised targets, weight
 * w_c = 1 for the 128 table entries and 16 for each of ln x_f, ln(P_e0/P_s),
 * ln(n_e0/n_scale):  dy = 2 w_c (y - (t - mean)/std) / (n * sum_c w_c);
 * loss_rows[i] = sum_c w_c r_c^2.  Rows with a non-finite target get dy = 0. */
int bp_surrogate_mse(int64_t n, const float *y, const float *targets, const float *mean, const float *std, float *dy,
                     float *loss_rows, void *stream);
/* The ICM solve of bp_icm_solve with the network's estimate of the gas boundary in place of the
 * x_f scan (Sec. 2.2: the energy condition fixes r_f; the surrogate only says where to look).  For
 * each halo inside the training domain (log10 M in [12.5, 15.5], c in [2, 15], z in [0.05, 3]) the
 * estimate x_f = exp(y[128] std[128] + mean[128]) (y: the network output rows [n][BP_MLP_OUT], device)
 * and a point 0.2% away start secant steps that widen until the energy residual changes sign (at
 * most 8); Brent's method then refines the root to 1e-13 relative, with the moment integrals built
 * as bp_icm_solve builds them, so x_f, a, rho0 and P0 agree with bp_icm_solve's to its tolerance
 * wherever the root is unique.  Every sol field is written as by bp_icm_solve.  status: 0; or
 * BP_S_OUT_OF_DOMAIN outside the domain (sol then holds only what bp_halo_structure writes);
 * BP_S_NO_BRACKET if no sign change was found (paste such halos with the exact path);
 * BP_S_MULTI_ROOT is never set (the root nearest the estimate is taken).  n may be 0. */
int bp_surrogate_solve(const bp_params *p, int64_t n, const double *M, const double *c, const double *z,
                       const float *y, const float *mean, const float *std, double *sol, int32_t *status,
                       void *stream);
/* Apply the network output to halos solved by bp_surrogate_solve (status 0): writes q-tables
 * [n][2*BP_MLP_NQ] (G values, not logs) from outputs 0..127 and meta (PE0, NE0 from the solved P0
 * and rho0; the grid and profile-constant fields 0).  Halos with a non-zero status are left
 * untouched.  y, mean, std and qtables must be 16-byte aligned (as every device allocation is);
 * otherwise BP_E_ARG. */
int bp_surrogate_apply(const bp_params *p, int64_t n, const float *y, const float *mean, const float *std,
                       const double *sol, const int32_t *status, float *qtables, float *meta, void *stream);
/* Exact q-tables for halos solved by bp_surrogate_solve (status 0): the projected profiles at the 64
 * q nodes by sight-line quadrature of the solved profile (Sec. 3.3), with the exact tables' own
 * integration (Gauss-Legendre in s along l = r_perp sinh s, split at r_vir, FP32 integrand, FP64
 * sums), in the layout and normalisation bp_surrogate_apply writes (G = Y / (P_e0 R_t E)); meta's PE0
 * and NE0 as bp_surrogate_apply.  This is the surrogate path's table mode that does not use the
 * network's table outputs: with it the surrogate's map error is that of the 64-node interpolation
 * (about 1e-4).  Halos with a non-zero status are left untouched.  n may be 0. */
int bp_surrogate_qtables_exact(const bp_params *p, int64_t n, const double *sol, const int32_t *status,
                               float *qtables, float *meta, void *stream);
/* Device-side training loop: `steps` Adam steps on batches of `batch` rows drawn
 * from (x, targets) by a counter-based hash of (seed, step0 + k, row) -- no host
 * synchronisation.  Learning rate follows a cosine from lr0 to lr1 over the
 * call; the Adam step counter continues from step0.  loss_rows (nullable,
 * batch floats) receives the last batch's per-row weighted squared error.
 * Workspace: bp_surrogate_train_ws_bytes(batch) bytes, 256-byte aligned; x and w_bf16 16-byte
 * aligned (BP_E_ARG otherwise). */
size_t bp_surrogate_train_ws_bytes(int64_t batch);
int bp_surrogate_train(float *w, uint16_t *w_bf16, float *m, float *v, float *grad, const float *mean,
                       const float *std, int64_t ndata, const float *x, const float *targets, int64_t steps,
                       int64_t batch, float lr0, float lr1, uint64_t seed, int64_t step0, float *loss_rows, void *ws,
                       size_t ws_bytes, void *stream);
/* --------------------------------------- surrogate lifecycle (one state buffer) */
/* The surrogate's whole state lives in one caller-allocated device buffer of bp_surrogate_state_bytes()
 * bytes, 256-byte aligned (the library allocates nothing).  Array a of the state starts at byte
 * bp_surrogate_state_offset(a): FP32 master weights (BP_MLP_NPARAMS layout above), their BF16 compute
 * copy, the two Adam moments, the last gradient, and the output mean and standard deviation (BP_MLP_OUT
 * floats each).  The buffer holds no pointers: copying its bytes copies the surrogate.  Every call
 * below that takes the state returns BP_E_ARG for a null or not 256-byte aligned state, before any
 * device work. */
enum { BP_SUR_W = 0, BP_SUR_WBF16, BP_SUR_M, BP_SUR_V, BP_SUR_G, BP_SUR_MEAN, BP_SUR_STD, BP_SUR_NARRAYS };
size_t bp_surrogate_state_bytes(void);
size_t bp_surrogate_state_offset(int32_t array);     /* (size_t)-1 for an unknown array */
/* Create: He-initialised weights (normal deviates from a counter-based hash of seed and parameter index,
 * variance 2 / fan-in, biases 0, input padding columns 0), zero Adam state, mean 0, std 1.
 * BP_E_ARG for a null or unaligned state. */
int bp_surrogate_init(void *state, uint64_t seed, void *stream);
/* Train from exact solves: the n halos (M, c, z, device) are solved (bp_icm_solve), tabulated
 * (bp_profile_tables) and turned into targets and their column statistics; then `steps` Adam steps as
 * bp_surrogate_train (cosine learning rate lr0 -> lr1, batches drawn by a counter-based hash of seed,
 * Adam step counter continuing from step0).  Workspace protocol as for the pastes (~2.5 KB per halo). */
int bp_surrogate_fit(const bp_params *p, void *state, int64_t n, const double *M, const double *c, const double *z,
                     int64_t steps, int64_t batch, float lr0, float lr1, uint64_t seed, int64_t step0, void *ws,
                     size_t ws_bytes, size_t *ws_needed, void *stream);
/* Save / load through a host blob of bp_surrogate_blob_bytes() bytes: a header (format tag, parameter
 * count, output width, Adam step) and the FP32 weights, moments, mean and std.  Both synchronise the
 * stream.  load rejects a blob of another format or size with BP_E_ARG (state unchanged) and refreshes
 * the BF16 copy; *step (nullable) receives the stored Adam step. */
size_t bp_surrogate_blob_bytes(void);
int bp_surrogate_save(const void *state, int64_t step, void *blob, size_t blob_bytes, void *stream);
int bp_surrogate_load(void *state, const void *blob, size_t blob_bytes, int64_t *step, void *stream);
/* Infer and paste (Sec. 3.3 HP maps through the surrogate), every routing decision on the device:
 * network outputs for all halos; bp_surrogate_solve; q-tables from the solved profiles
 * (tables = BP_SUR_TABLES_EXACT, bp_surrogate_qtables_exact) or from the network's table outputs
 * (BP_SUR_TABLES_NETWORK, bp_surrogate_apply); halos outside the training domain or without a root near
 * the estimate are compacted, solved by the exact scan (bp_icm_solve) and given exact q-tables; then one
 * q-table deposit of all halos (bp_hp_paste_flat_q / bp_hp_paste_healpix_q, maps ACCUMULATE, y_comp /
 * b_comp nullable as there).  Halos the exact solve cannot solve either (invalid input, stars above the
 * baryon mass) are skipped.  *n_fallback (nullable) receives the number of halos routed to the scan.
 * Workspace protocol as for the pastes (about 1.4 KB per halo plus the deposit's); one synchronisation
 * for the routed count, one in the deposit.  The deposit's set-up and plan run on the library's second
 * stream (as in bp_hp_flat_pipeline) beside the q-tables of the halos the seeded solve solved; on
 * return, error returns included, all work is ordered on `stream`, and calls on one device from
 * several host threads are serialised inside the library. */
#define BP_SUR_TABLES_EXACT   0
#define BP_SUR_TABLES_NETWORK 1
int bp_surrogate_paste_flat(const bp_params *p, const void *state, int32_t tables, int32_t npix, double pix_rad,
                            int64_t n, const double *M, const double *c, const double *z, const double *theta_x,
                            const double *theta_y, const double *v_los, float *y_map, float *b_map, float *y_comp,
                            float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, int64_t *n_fallback,
                            void *stream);
int bp_surrogate_paste_healpix(const bp_params *p, const void *state, int32_t tables, int64_t nside, int64_t n,
                               const double *M, const double *c, const double *z, const double *theta,
                               const double *phi, const double *v_los, float *y_map, float *b_map, float *y_comp,
                               float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, int64_t *n_fallback,
                               void *stream);
/* HP flat paste from surrogate q-tables: as bp_hp_paste_flat with
 * Y_P(r_perp) = P_e0 R_t E(r_perp) G_P(q), q = r_perp / R_t, cubic interpolation
 * in s = acos(1 - 2q)/pi on the 64 nodes.  Halos whose status is non-zero are
 * skipped (paste them with the exact path). */
int bp_hp_paste_flat_q(const bp_params *p, int32_t npix, double pix_rad, int64_t n, const double *theta_x,
                       const double *theta_y, const double *v_los, const double *sol, const int32_t *status,
                       const float *qtables, const float *meta, float *y_map, float *b_map, float *y_comp,
                       float *b_comp, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream);
/* The same for HEALPix RING maps (bp_hp_paste_healpix with surrogate q-tables; same arguments,
 * layouts, workspace protocol and errors as bp_hp_paste_healpix, tables as bp_hp_paste_flat_q). */
int bp_hp_paste_healpix_q(const bp_params *p, int64_t nside, int64_t n, const double *theta, const double *phi,
                          const double *v_los, const double *sol, const int32_t *status, const float *qtables,
                          const float *meta, float *y_map, float *b_map, float *y_comp, float *b_comp, void *ws,
                          size_t ws_bytes, size_t *ws_needed, void *stream);

/* ------------------------------------------------------------- profiling */
/* Optional timing of the library's main kernels with HIP events recorded on
 * the launch stream (for roofline measurement).  bp_profiling(1) enables it
 * and clears earlier records; bp_profile_read() waits for the recorded
 * events and returns the summed duration and number of launches of one
 * kernel since the last bp_profiling call.  Host-side only; not thread-safe
 * with respect to concurrent launches on several streams. */
enum {
    BP_PROF_ICM = 0,        /* K1 k_icm_solve */
    BP_PROF_TABLES,         /* K2 k_tables */
    BP_PROF_FLAT_PLAN,      /* K3 setup + pair emission + sort + tile ranges */
    BP_PROF_FLAT_DEPOSIT,   /* K3 k_flat_deposit */
    BP_PROF_HPX_PLAN,       /* K4 planning */
    BP_PROF_HPX_DEPOSIT,    /* K4 k_hpx_deposit */
    BP_PROF_PP_SORT,        /* K5 cell keys + radix sort + gather */
    BP_PROF_PP_KNN,         /* K6 k_pp_knn */
    BP_PROF_PP_PLAN,        /* K7 amplitudes + pair emission + sort */
    BP_PROF_PP_DEPOSIT,     /* K8 narrow + wide deposits */
    BP_PROF_MLP_FWD,        /* K10 surrogate forward */
    BP_PROF_MLP_BWD,        /* K11 surrogate backward */
    BP_PROF_SURR_APPLY,     /* K10 epilogue: tables from the network output */
    BP_PROF_FLATQ_DEPOSIT,  /* K3 deposit from surrogate tables */
    BP_PROF_HPXQ_DEPOSIT,   /* K4 deposit from surrogate tables */
    BP_PROF_PP_NEFF,        /* K6b k_pp_neff */
    BP_PROF_NGP_PLAN,       /* K13 pixel indices + tile counting sort + amplitudes */
    BP_PROF_NGP_DEPOSIT,    /* K13 k_ngp_deposit */
    BP_PROF_SPECTRUM,       /* K14 flat-sky power spectrum */
    BP_PROF_SURR_SOLVE,     /* K1 seeded by the surrogate (bp_surrogate_solve) */
    BP_PROF_NKERNELS
};
int bp_profiling(int enable);
int bp_profile_read(int kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* BP_H */
