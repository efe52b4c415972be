/*
 * fkr.h -- C ABI of the MI355X (gfx950) fast multivariate kernel regression
 * library: binned local-polynomial kernel regression on a uniform grid through
 * a type-1 non-uniform FFT, with the per-grid-point normal-equation solve,
 * Girard's Monte-Carlo degrees of freedom, GCV and the conditional-variance
 * second pass of Wang et al., "FKreg: A MATLAB toolbox for fast multivariate
 * kernel regression" (arXiv 2204.07716).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch-allocated
 *    HBM); every other pointer is host memory.  The library never allocates
 *    device memory: the caller owns all inputs, outputs and the workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is enqueued on it and is asynchronous; outputs are
 *    valid once the stream has been synchronised.  Argument errors are found on
 *    the host before anything is enqueued, and then nothing is enqueued.
 *  - Samples X are N x d, row-major (x_i0, ..., x_i,d-1 contiguous), element
 *    type FKR_F32 or FKR_F64.  They must lie inside the grid box [lo, hi]
 *    (up to a relative 1e-12 of the box width); samples outside are counted in
 *    the diagnostics and reported by fkr_get_diagnostics as FKR_E_DOMAIN.
 *  - Real responses Y are N x q row-major.  Complex responses (y_complex = 1)
 *    are N x q complex numbers stored as interleaved (re, im) pairs.
 *  - Grid functions (fits, moments, variance) are laid out with the index of
 *    dimension 0 fastest: flat(k) = k_0 + M_0 (k_1 + M_1 k_2).  The grid of
 *    eq. (6) has g_k = lo + k * (hi - lo) / (M - 1) per dimension (both ends on
 *    the grid).
 *  - Bandwidths: h is the per-dimension standard deviation of the Gaussian
 *    kernel, i.e. the bandwidth matrix of eq. (2) is diag(h_j^2).  A call with
 *    nh bandwidths takes a host array of nh x d doubles.  Every h_j must lie
 *    within the plan's [h_min_j, h_max_j].
 *  - Monomials / moment channels are ordered by total degree, then by the
 *    exponent of dimension 0 descending, then dimension 1, ...: for d = 2 the
 *    design row of eq. (4)/(14) is [1, z0, z1, z0^2, z0 z1, z1^2, ...].
 *  - Nothing is printed; no exception crosses the ABI.  One plan serves one
 *    stream at a time (calls on one plan must not overlap).
 */
#ifndef FKR_H
#define FKR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FKR_OK = 0,
    FKR_WARN_ILLPOSED = 1,   /* some grid points had no well-posed solve (NaN) */
    FKR_E_ARG = -1,          /* invalid argument (host-detected, nothing enqueued) */
    FKR_E_DOMAIN = -2,       /* samples outside [lo, hi] (device-detected) */
    FKR_E_WORKSPACE = -3,    /* workspace missing or too small */
    FKR_E_DEVICE = -4,       /* a HIP runtime call failed */
    FKR_E_UNSUPPORTED = -5,  /* a valid request this library does not implement */
    FKR_E_STATE = -6         /* call order violated (e.g. no points set) */
} fkr_status;

enum { FKR_F32 = 0, FKR_F64 = 1 };             /* element types */
enum { FKR_KERNEL_ES = 0, FKR_KERNEL_GAUSS = 1 }; /* spreading (gridding) kernel */
enum { FKR_VAR_LOG = 0, FKR_VAR_DIRECT = 1 };   /* variance estimator */
enum { FKR_TP_SAME = 0, FKR_TP_F32 = 1, FKR_TP_F64 = 2 }; /* transform precision */
enum { FKR_SIG_SCALAR = 0, FKR_SIG_GRID = 1 };   /* error variance of fkr_interval */
/* Regression kernel K of eq. (2) (Table 1 kernel_type).  The Gaussian is the
 * standard normal density and h its standard deviation; the compact kernels
 * live on |u| <= 1 with h the half-width of their support (K_h(u) =
 * K(u / h) / h per dimension): box 1/2, triangle 1 - |u|, Epanechnikov
 * 3/4 (1 - u^2), biweight 15/16 (1 - u^2)^2, triweight 35/32 (1 - u^2)^3. */
enum { FKR_REG_GAUSS = 0, FKR_REG_BOX = 1, FKR_REG_TRIANGLE = 2, FKR_REG_EPANECHNIKOV = 3,
       FKR_REG_BIWEIGHT = 4, FKR_REG_TRIWEIGHT = 5 };

#define FKR_MAX_D 3
#define FKR_MAX_ORDER 2
#define FKR_MAX_H 64        /* bandwidths per call */

/* Support of the DF, RSS and GCV sums (fkr_cv, fkr_dof, fkr_gcv).  A grid
 * point is *resolved* when its solve is well-posed and every Cholesky pivot
 * of its bandwidth-equilibrated moment matrix exceeds FKR_RESOLVE times the
 * matching diagonal entry: pivot_c / A_cc is one minus the uncentred R^2 of
 * design column c on the earlier columns (the reciprocal of its variance
 * inflation factor), so resolved points have a local design with VIF <= 1000
 * in every direction.  A sample is *supported* when all 2^d corners of its
 * interpolation cell are resolved; the Girard ratios, the RSS and N in eq.
 * (22) run over the N_I supported samples only, and N_I is reported.  A
 * sample whose cell touches a grid point this library leaves NaN (see
 * fkr_fit) is left out as well. */
#define FKR_RESOLVE 1e-3

typedef struct fkr_plan fkr_plan;

/* Plan description; mirrors the options of Table 1 that concern the fast
 * path.  Zero-initialise and fill in the fields you need. */
typedef struct {
    int d;                  /* dimension, 1..3 */
    int order;              /* local polynomial order l (eq. 2), 0..2 */
    int64_t M[FKR_MAX_D];   /* grid points per dimension, >= 2 (Table 1 "M") */
    double lo[FKR_MAX_D];   /* grid box; both ends are grid points (eq. 6) */
    double hi[FKR_MAX_D];
    double h_min[FKR_MAX_D];/* bandwidth range the plan must serve; sets the */
    double h_max[FKR_MAX_D];/* spectral band (h_min) and the zero padding (h_max) */
    double eps;             /* requested relative accuracy of the moment sums,
                               in (0, 1) (replaces Table 1 "accuracy") */
    int precision;          /* FKR_F64 or FKR_F32: spreading (kernel values and
                               LDS accumulation) and, unless transform_precision
                               says otherwise, FFTs and channel grids; the
                               normal-equation solves are always FP64 */
    int spread_kernel;      /* FKR_KERNEL_ES (default) or FKR_KERNEL_GAUSS (the
                               paper's fast Gaussian gridding, Sec. 1.2) */
    double sigma;           /* fine-grid oversampling over the spectral band;
                               0 selects 4 for d <= 2 and 2 for d = 3 (eq. 17
                               uses M_r = 2 L) */
    int64_t n_max;          /* largest N passed to fkr_set_points */
    int max_weights;        /* largest number of real weight vectors one call
                               spreads, counting the density: 1 + q (real y) or
                               1 + 2q (complex y), plus Np probes for DF calls */
    int max_h;              /* largest nh per call, 1..FKR_MAX_H */
    int transform_precision;/* FKR_TP_SAME (follow `precision`), FKR_TP_F32 or
                               FKR_TP_F64: element type of the fine grid, the
                               FFTs, the spectra and the channel grids; with
                               precision FKR_F32 and FKR_TP_F64 the spreading
                               runs in FP32 and everything after it in FP64 */
    int reg_kernel;         /* FKR_REG_GAUSS (0, default) or a compact kernel:
                               then the moments are the binned approximation of
                               eq. (11)-(13), the kernel sampled at the grid
                               offsets and its discrete transform applied to
                               every mode of the period (no spectral cut), so
                               they differ from the exact kernel sums by the
                               kernel's aliasing, which shrinks with
                               (delta / h)^(s+1) for a kernel with s
                               continuous derivatives; the calls taking a
                               full H need the Gaussian
                               (FKR_E_UNSUPPORTED otherwise) */
} fkr_plan_desc;

/* Geometry chosen by the planner (read-only). */
typedef struct {
    int d, order;
    int n_s, n_t;            /* moment channels: C(d+2l, 2l) and P = C(d+l, l) */
    int64_t M[FKR_MAX_D];
    int64_t L[FKR_MAX_D];    /* periodic length in grid steps (zero padding, eq. 18) */
    int64_t K[FKR_MAX_D];    /* retained modes n = -K..K per dimension */
    int64_t Mr[FKR_MAX_D];   /* fine (spreading) grid length per dimension */
    int64_t tile[FKR_MAX_D]; /* spreading tile edge, fine cells */
    double delta[FKR_MAX_D]; /* grid spacing */
    double period[FKR_MAX_D];/* T_j = L_j * delta_j */
    int w;                   /* spreading kernel width, fine cells */
    double kparam;           /* ES beta, or the Gaussian's exp coefficient per cell^2 */
    int64_t n_tiles;
    size_t workspace_bytes;
} fkr_geometry;

typedef struct {
    int64_t n_points;        /* N of the last fkr_set_points */
    int64_t out_of_domain;   /* samples outside [lo, hi] */
    int64_t ill_posed;       /* grid-point solves reported as NaN (last call) */
    int64_t n_jobs;          /* spreading work items of the last fkr_set_points */
    int64_t max_tile_count;  /* most samples in one tile */
} fkr_diag;

/* Create a plan: grid geometry, spectral band, spreading kernel and tables
 * (Sec. 4 fkreg_create; Table 1).  Host only.  Errors: FKR_E_ARG for d, order,
 * M, box, bandwidth range, eps or sizes out of range; FKR_E_UNSUPPORTED when a
 * transform or a spreading tile would not fit the LDS of one workgroup (very
 * small h_min relative to the box, very large M, or a wide kernel in 3-D
 * FP64).  *out is owned by the caller and released with fkr_plan_destroy. */
fkr_status fkr_plan_create(const fkr_plan_desc* desc, fkr_plan** out);
void fkr_plan_destroy(fkr_plan* plan);
fkr_status fkr_plan_geometry(const fkr_plan* plan, fkr_geometry* out);

/* Device workspace: size in bytes for the plan's maxima, then bind a buffer
 * of at least that size (256-byte aligned).  fkr_set_workspace uploads the
 * plan's constant tables with a synchronous copy. */
fkr_status fkr_workspace_size(const fkr_plan* plan, size_t* bytes);
fkr_status fkr_set_workspace(fkr_plan* plan, void* ws_dev, size_t bytes);

/* Bin and sort the samples by spreading tile (part of the O(N) gridding of
 * Sec. 1.2, eq. 16-17); reused by every later call until the next
 * fkr_set_points.  X_dev: N x d of type x_type.  N may be 0. */
fkr_status fkr_set_points(fkr_plan* plan, int64_t N, const void* X_dev, int x_type,
                          void* stream);

/* Type-1 NUFFT stage (eq. 16-20): for nw real weight vectors W (N x nw,
 * row-major, type w_type; NULL with nw = 1 means the unit weights of the
 * delta train), the deconvolved spectrum
 *     c(n) = sum_i w_i exp(-i sum_j 2 pi n_j (x_ij - lo_j) / T_j)
 * for n_j = -K_j..K_j.  out_dev: complex128 array (re, im interleaved) of
 * shape [nw][2K_{d-1}+1]...[2K_0+1]. */
fkr_status fkr_spectrum(fkr_plan* plan, int nw, const void* W_dev, int w_type,
                        double* out_dev, void* stream);

/* Moment sums of eq. (9) on the grid, through spreading, FFT, deconvolution,
 * multiplication by the kernel-moment spectra and inverse FFT (eq. 12-13,
 * 16-21).  Channels are equilibrated by the bandwidth: S_dev receives
 * s_a(g) / h^a for |a| <= 2l ([nh][n_s][M^d] doubles) and T_dev receives
 * t_{w,b}(g) / h^b for |b| <= l ([nh][nw][n_t][M^d] doubles); either may be
 * NULL.  W as in fkr_spectrum (NULL with nw = 0 gives only S). */
fkr_status fkr_moments(fkr_plan* plan, int nh, const double* h, int nw, const void* W_dev,
                       int w_type, double* S_dev, double* T_dev, void* stream);

/* Binned local-polynomial fit of eq. (11): per grid point the P x P system
 * A_bc = s_{b+c}, rhs_b = t_b, solved in FP64 (Cholesky of the
 * bandwidth-equilibrated matrix); mhat = intercept.  Y: N x q (real or
 * complex).  mhat_dev: [nh][q][M^d] doubles (complex: [nh][q][M^d][2]).
 * s0_dev (optional, [nh][M^d] doubles): s_0, the unnormalised KDE of eq. (8).
 * Grid points whose system the fast moments cannot resolve get NaN and are
 * counted: some Cholesky pivot c of the equilibrated matrix (s_0 is the
 * first) is at most max(r A_cc, e N K_h(0)), with K_h(0) = prod_j 1 / (h_j
 * sqrt(2 pi)), r = max(64 unit round-offs of the spreading precision,
 * 10 eps) (the moments are known to about that fraction of their local size)
 * and e = max(16 unit round-offs of the transform precision, 1e-5 eps) (the
 * transforms' global error).  This is a property of the fast path, not a
 * reading of the method: the plain definition leaves every non-singular
 * system well-posed. */
fkr_status fkr_fit(fkr_plan* plan, int nh, const double* h, int q, int y_complex,
                   const void* Y_dev, int y_type, double* mhat_dev, double* s0_dev,
                   void* stream);

/* fkr_set_points followed by fkr_fit, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): the
 * workspace is an array the library holds on each device for the life of the
 * process, FKR_STATIC_WORKSPACE_BYTES long, instead of a caller buffer bound
 * with fkr_set_workspace.  Calls no hipMalloc / hipFree.  The plan must need
 * at most that much (fkr_workspace_size), else FKR_E_WORKSPACE and nothing
 * is enqueued; arguments as in fkr_set_points and fkr_fit (N <= n_max).  The
 * plan stays bound to the array, so later calls on it use the array too.
 * Every call on a device shares that device's array and keeps the last
 * call's contents: the plan's tables are uploaded and the counters cleared,
 * ordered on `stream`, at the start of each call.  Calls on one device that
 * can overlap (other streams, other host threads, other plans) race on the
 * array; serialise them. */
#define FKR_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
fkr_status fkr_fit_noalloc(fkr_plan* plan, int64_t N, const void* X_dev, int x_type, int nh,
                           const double* h, int q, int y_complex, const void* Y_dev, int y_type,
                           double* mhat_dev, double* s0_dev, void* stream);

/* Moments and fits with a full bandwidth matrix (eq. 2: K_H(u) =
 * |H|^{-1/2} K(H^{-1/2} u), K the standard Gaussian density), nh matrices H
 * (host, nh x d x d doubles, row-major, symmetric positive definite).  The
 * transform of u^a K_H(u) is (-i)^{|a|} He_a(w) exp(-w^T H w / 2), with the
 * multivariate Hermite polynomials of H (He_0 = 1, He_{b+e_j} = (H w)_j He_b
 * - sum_k b_k H_jk He_{b-e_k}), evaluated per retained mode; everything
 * else is the path of fkr_moments / fkr_fit.  Channels are equilibrated by
 * s^a, s_j = sqrt(H_jj).  Each H must have s_j <= h_max_j (the padding holds
 * the kernel's reach along axis j) and 1 / sqrt((H^-1)_jj) >= h_min_j (the
 * band holds its spectrum along frequency axis j), else FKR_E_ARG; the
 * ill-posedness floor uses K_H(0).  Layouts as fkr_moments and fkr_fit. */
fkr_status fkr_moments_full(fkr_plan* plan, int nh, const double* H, int nw, const void* W_dev, int w_type,
                            double* S_dev, double* T_dev, void* stream);
fkr_status fkr_fit_full(fkr_plan* plan, int nh, const double* H, int q, int y_complex, const void* Y_dev,
                        int y_type, double* mhat_dev, double* s0_dev, void* stream);
/* fkr_cv (fits, Monte-Carlo DF, RSS and GCV of eq. 22, Sec. 2.1) over a
 * list of nh full bandwidth matrices H (as fkr_fit_full), for choosing H by
 * GCV; arguments and outputs as fkr_cv with H in place of h. */
fkr_status fkr_cv_full(fkr_plan* plan, int nh, const double* H, int q, int y_complex, const void* Y_dev,
                       int y_type, int Np, uint64_t seed, const void* probes_dev, double* mhat_dev,
                       double* rho_dev, double* rss_dev, double* gcv_dev, double* nused_dev, void* stream);

/* Multilinear interpolation (the linear griddedInterpolant of Sec. 1.1/5) of
 * nv grid functions G_dev ([nv][M^d] doubles) at Nq query points Xq_dev
 * (Nq x d, type x_type) -> out_dev ([nv][Nq] doubles).  The cell of a point
 * is floor((x - lo)/delta) clamped to [0, M-2]. */
fkr_status fkr_interp(fkr_plan* plan, int nv, const double* G_dev, int64_t Nq,
                      const void* Xq_dev, int x_type, double* out_dev, void* stream);

/* Fast Monte-Carlo DF (Sec. 2.1, Girard): Np Gaussian probes w_p pushed
 * through the grid smoother (moments -> solve -> interpolation to the
 * samples).  rho_dev: [nh][Np] doubles, rho_p = sum_I w_p (w_p - w_hat_p) /
 * sum_I w_p^2 over the supported samples I (see FKR_RESOLVE); their mean
 * estimates (1/N_I) tr((I - S_h)_II), and DF = N_I (1 - mean).  nused_dev
 * (optional, [nh] doubles) receives N_I.  Probes come from probes_dev
 * (N x Np, type w_type) or, when it is NULL, from the Philox4x32-10
 * generator: sample i, probe 4g + r uses word r of the Box-Muller transform of
 * the block with counter (i mod 2^32, floor(i / 2^32), g, 0) and key
 * (seed mod 2^32, floor(seed / 2^32)); uniforms u = (floor(x / 2^8) + 1/2)
 * 2^-24; normals sqrt(-2 ln u_0) (cos, sin)(2 pi u_1) from words (0, 1) and
 * likewise from (2, 3), in FP64 for FP64 plans and with the hardware
 * log / sqrt / sin / cos for FP32 plans. */
fkr_status fkr_dof(fkr_plan* plan, int nh, const double* h, int Np, uint64_t seed,
                   const void* probes_dev, int w_type, double* rho_dev, double* nused_dev,
                   void* stream);

/* Batched cross-validation (Sec. 2 and Fig. 3, cv_fkreg): for every h, the
 * fit of all q responses and the DF from Np probes share one spreading and
 * one forward FFT of every weight vector.  Outputs (any may be NULL):
 * mhat_dev as in fkr_fit; rho_dev [nh][Np] as in fkr_dof; rss_dev [nh][q] =
 * sum_I |y_i - yhat(x_i)|^2 over the supported samples; gcv_dev [nh][q] =
 * (rss / N_I) / mean_p(rho_p)^2 (eq. 22; needs Np >= 1); nused_dev [nh] =
 * N_I. */
fkr_status fkr_cv(fkr_plan* plan, int nh, const double* h, int q, int y_complex,
                  const void* Y_dev, int y_type, int Np, uint64_t seed,
                  const void* probes_dev, double* mhat_dev, double* rho_dev,
                  double* rss_dev, double* gcv_dev, double* nused_dev, void* stream);

/* GCV of eq. (22) for responses Y against a DF computed earlier (Sec. 2.1:
 * the DF does not depend on y): rho_dev holds the [nh][Np] Girard ratios of
 * fkr_dof (or fkr_cv) for the same points and bandwidths.  Fits density and
 * Y at every h, interpolates the fits to the samples and sums the squared
 * residuals over the supported samples I on the device; gcv_dev [nh][q] =
 * (rss / N_I) / mean_p(rho_p)^2.  mhat_dev, rss_dev and nused_dev are
 * optional (as in fkr_cv).  FKR_E_ARG for q < 1, Np < 1 or missing rho_dev
 * or gcv_dev. */
fkr_status fkr_gcv(fkr_plan* plan, int nh, const double* h, int q, int y_complex,
                   const void* Y_dev, int y_type, int Np, const double* rho_dev,
                   double* mhat_dev, double* rss_dev, double* gcv_dev, double* nused_dev,
                   void* stream);

/* Conditional-variance second pass (Sec. 3) at one bandwidth h (d doubles):
 * residuals r_i = |y_i - mhat(x_i)|^2 from the mean fit's grid mhat_dev
 * (output of fkr_fit for this Y, one column: [M^d] doubles, or [M^d][2] for
 * complex y), then
 *   FKR_VAR_LOG (eq. 24-26): v = fit of log(r_i + 1/N); kappa =
 *       [mean_i r_i exp(-v(x_i))]^-1; sigma^2(g) = exp(v(g)) / kappa;
 *   FKR_VAR_DIRECT (eq. 23): sigma^2(g) = fit of r_i.
 * Samples whose residual is undefined (NaN mean fit at a corner of their
 * cell) are left out of the second fit and of kappa, whose mean runs over the
 * samples where r_i exp(-v(x_i)) is defined.  The fit uses the plan's order.
 * sigma2_dev: [M^d] doubles; vhat_dev (optional, FKR_VAR_LOG) [M^d];
 * kappa_dev (optional) 1 double.  The density moments s_alpha of the second
 * fit equal those of the first (same points, same h, no sample left out):
 * when C(d+2l, 2l) is even and the channel buffer still holds them from the
 * plan's last fkr_fit, fkr_cv, fkr_gcv, fkr_moments or fkr_variance call at
 * a bitwise equal h on the same points, the call transforms only the moments
 * t_alpha of the new weights.  The check runs on the device, so a captured
 * graph replays correctly after any preceding call. */
fkr_status fkr_variance(fkr_plan* plan, const double* h, int y_complex, const void* Y_dev,
                        int y_type, const double* mhat_dev, int mode, double* sigma2_dev,
                        double* vhat_dev, double* kappa_dev, void* stream);
/* fkr_variance with the second fit at a full bandwidth matrix H (host,
 * d x d, as fkr_fit_full; Gaussian kernel); mhat_dev is the fit at H
 * (fkr_fit_full).  Nothing is kept between calls: the density moments under
 * K_H are made again. */
fkr_status fkr_variance_full(fkr_plan* plan, const double* H, int y_complex, const void* Y_dev,
                             int y_type, const double* mhat_dev, int mode, double* sigma2_dev,
                             double* vhat_dev, double* kappa_dev, void* stream);

/* Gradient of the GCV criterion of eq. (22) with respect to log h (Sec. 2.1:
 * bandwidth selection minimises GCV over h) and to the response, for one
 * response Y (N x 1, type y_type; complex interleaved when y_complex, with
 * |.|^2 in the RSS) and Np Philox probes (as fkr_cv with that seed).  The fits
 * are m_hat = e_0^T A^{-1} t with the bandwidth-equilibrated moments A, t of
 * eq. (11); their derivative in theta_j = log h_j is
 * e_0^T A^{-1} (dt - dA A^{-1} t), where dA, dt come from the same type-1
 * spectra multiplied by the derivative of the Gaussian moment multipliers,
 * d/dtheta_j [He_a(u) exp(-u^2/2)] = -u He_{a+1}(u) exp(-u^2/2), u = h_j w_j
 * (a compact kernel: the transform of the derivative of its sampled moment
 * kernel, -((1 + a) K(v) + v K'(v)) v^a / h_j, v = u / h_j, K' = 0 inside
 * the box kernel's support.  The binned box fit weighs the same window
 * equally for every h between the bandwidths where a grid offset crosses
 * the support's edge, so its GCV is piecewise constant there and its log-h
 * gradient zero up to rounding; at those bandwidths GCV jumps).
 * With the supported set I held fixed, dRSS = -2 sum_I r_i d yhat_i and
 * d rho_p = -sum_I w_pi d what_pi / sum_I w_pi^2, so
 * d GCV / d theta_j = GCV (dRSS / RSS - 2 d rho_bar / rho_bar).
 * The gradient in y (the DF does not depend on y) is
 * d GCV / dy = 2 / (N_I rho_bar^2) (r - S^T r), r_i = y_i - yhat_i on the
 * supported samples and 0 elsewhere, with the adjoint of the smoother
 * (S^T r)_l = sum_g sum_b u(g) c_b(g) k_b(x_l - g): u the residuals scattered
 * to the grid by the interpolation weights, c = A^{-1} e_0 and k_b the
 * equilibrated moment kernels; the sum over g runs as a type-2 transform
 * (the adjoint of the spread: forward FFT of the zero-padded grid functions,
 * conjugate moment multipliers, inverse FFT to the fine grid, the spreading
 * kernel at each sample).
 * gcv_dev (optional, 1 double): GCV at h; dlogh_dev [d] doubles: the
 * gradient in log h; dy_dev (optional, [N] doubles in the order of Y, or
 * [N][2] for complex y): the gradient in y, for complex y
 * d GCV / d Re y + i d GCV / d Im y (the convention of PyTorch for a real
 * function of complex inputs); dfit_dev [d][ny + Np][M^d] doubles
 * (caller-owned; ny = 1, or 2 for complex y): d m_hat / d log h_j of the
 * response parts and of each probe fit, NaN where the fit is not
 * resolved.  The plan needs room for the channels of 1 + ny + Np weights
 * twice (see below).
 * The plan's channel buffer holds the channels at h and their derivatives
 * side by side: FKR_E_ARG unless 2 ceil((n_s + n_t (ny + Np)) / 2) <=
 * ceil((n_s + n_t (max_weights - 1)) / 2) (max_weights >= 2 (1 + ny + Np)
 * + n_s / n_t suffices). */
fkr_status fkr_gcv_grad(fkr_plan* plan, const double* h, int y_complex, const void* Y_dev, int y_type, int Np,
                        uint64_t seed, double* gcv_dev, double* dlogh_dev, double* dy_dev, double* dfit_dev,
                        void* stream);
/* fkr_gcv_grad at a full bandwidth matrix H (host, d x d, as fkr_fit_full;
 * Gaussian kernel): GCV and its gradient in the entries H_pq, p <= q, in
 * row-major upper-triangle order (dH_dev: d (d + 1) / 2 doubles; an
 * off-diagonal entry moves H_pq and H_qp together).  The multipliers'
 * derivative follows the Hermite recurrence of fkr_fit_full forward, with
 * the Gaussian factor and the equilibration by sqrt(diag H); dy_dev
 * (optional) as in fkr_gcv_grad, its adjoint with the full-H multipliers;
 * dfit_dev [d (d + 1) / 2][ny + Np][M^d] as in fkr_gcv_grad. */
fkr_status fkr_gcv_grad_full(fkr_plan* plan, const double* H, int y_complex, const void* Y_dev, int y_type,
                             int Np, uint64_t seed, double* gcv_dev, double* dH_dev, double* dy_dev,
                             double* dfit_dev, void* stream);

/* Variance of the fit and pointwise confidence band (Sec. 4.2, eq. 27-28;
 * Sec. 4 fkreg_interval) at one bandwidth h (d doubles).  The fit of eq. (3)
 * is linear in y, m_hat(g) = sum_i S_gi y_i, so for independent errors of
 * variance sigma_i^2 its variance is Sigma(g) = sum_i S_gi^2 sigma_i^2 =
 * r^T Q r, with r = A(g)^{-1} e_1 and Q_bc = sum_i K_h(x_i - g)^2 (x_i -
 * g)^{b+c} sigma_i^2.  The squared Gaussian kernel is K_{h/sqrt2} times
 * prod_j 1 / (2 sqrt(pi) h_j), so Q comes from one more pass of the moment
 * path at h / sqrt 2, which must lie within the plan's bandwidth range
 * (create the plan with h_min <= h / sqrt 2), else FKR_E_ARG.  With a
 * compact reg_kernel the squared kernel prod_j (K(u_j / h_j)^2 / h_j) /
 * h_j is sampled at h like the kernel (the binned approximation of both
 * A and Q; exact for samples on grid nodes).
 *   sig_kind FKR_SIG_SCALAR: sigma_i^2 = sigma2 (homoscedastic model);
 *   FKR_SIG_GRID: sigma_i^2 = multilinear interpolation at x_i of the grid
 *   sigma2_dev ([M^d] doubles, e.g. fkr_variance's output); samples where it
 *   is undefined (NaN at a corner of their cell) are left out of the sum.
 * Sigma_dev [M^d] doubles receives Sigma (NaN where the fit is ill-posed, as
 * in fkr_fit).  lower_dev / upper_dev (optional, [M^d]) receive
 * mhat -/+ z_{1-alpha/2} sqrt(max(Sigma, 0)) for the real fit mhat_dev ([M^d]
 * doubles) and 0 < alpha < 1; z is found on the host from the C library's
 * erfc.  The call spreads and transforms the density (and, for
 * FKR_SIG_GRID, the interpolated sigma^2); it needs points set. */
fkr_status fkr_interval(fkr_plan* plan, const double* h, int sig_kind, double sigma2,
                        const double* sigma2_dev, const double* mhat_dev, double alpha,
                        double* Sigma_dev, double* lower_dev, double* upper_dev, void* stream);
/* fkr_interval at a full bandwidth matrix H (host, d x d, as fkr_fit_full;
 * Gaussian kernel): K_H^2 = K_{H/2} (4 pi)^{-d/2} |H|^{-1/2}, so Q comes from
 * one more pass at H / 2, which must lie within the plan's bandwidth range
 * (the conditions of fkr_fit_full for H / 2), else FKR_E_ARG.  Arguments
 * and outputs as fkr_interval. */
fkr_status fkr_interval_full(fkr_plan* plan, const double* H, int sig_kind, double sigma2,
                             const double* sigma2_dev, const double* mhat_dev, double alpha,
                             double* Sigma_dev, double* lower_dev, double* upper_dev, void* stream);

/* Prediction at new points by tensor-product cubic spline interpolation of
 * grid functions (Sec. 4 fkreg_compact / fkreg_predict; Table 1 y_grid_opt:
 * Method 'spline', ExtrapolationMethod 'linear').  Along each dimension the
 * spline is the not-a-knot cubic interpolant of the M_j grid values (the
 * parabola for M_j = 3, the line for M_j = 2); beyond the box it continues
 * along the tangent at the nearer end, dimension by dimension.  NaN grid
 * values make the spline NaN along every grid line through them.
 *   fkr_spline: coef_dev ([nv][2^d][M^d] doubles, caller-owned, must not
 *   overlap G_dev) receives, per grid function of G_dev ([nv][M^d]), the
 *   function itself and its mixed second derivatives d^2|S| f /
 *   prod_{j in S} dk_j^2 in grid-index units, for every nonempty subset S of
 *   the dimensions (array index = bit mask of S).
 *   fkr_predict: the spline value at Nq points Xq_dev (Nq x d, type x_type)
 *   -> out_dev [nv][Nq] doubles; NaN for non-finite coordinates.
 * Neither call needs points or the workspace, only the plan's grid. */
fkr_status fkr_spline(fkr_plan* plan, int nv, const double* G_dev, double* coef_dev, void* stream);
fkr_status fkr_predict(fkr_plan* plan, int nv, const double* coef_dev, int64_t Nq, const void* Xq_dev,
                       int x_type, double* out_dev, void* stream);

/* Batches of independent regressions (Sec. 2.1 and Fig. 3: the cross-
 * validation loop of one regression; Sec. 4.3: many responses): R
 * regressions of uneven size on one plan geometry (the same grid, order,
 * bandwidth range and precision), each run as fkr_set_points + fkr_cv.  A
 * batch owns n_lanes plans, each with a HIP stream of its own (default
 * priority, created by fkr_batch_create) and a slice of one caller-owned
 * workspace.  fkr_batch_cv records an event on `stream`, lets the lanes wait
 * on it, runs the regressions on the lanes, largest first, each to the lane
 * with the least estimated work so far (N + 4 M^d sample equivalents per
 * regression), and makes `stream` wait for every lane, so the whole batch is
 * ordered on `stream` and can be captured into one HIP graph by capturing
 * `stream`.
 *   offsets: host array of R + 1 sample offsets (offsets[0] = 0,
 *   nondecreasing, each regression at most desc.n_max samples); regression
 *   r owns rows offsets[r] .. offsets[r+1] - 1 of X_dev (x_type) and Y_dev
 *   (y_type, q columns, complex interleaved when y_complex) -- the layouts of
 *   fkr_set_points and fkr_cv.  Its probes are those of fkr_cv with seed
 *   `seed + r` (generated; Np >= 1).
 *   Outputs (each optional), regression-major: mhat_dev [R][nh][q][M^d]
 *   (complex: [..][2]), rho_dev [R][nh][Np], rss_dev and gcv_dev [R][nh][q],
 *   nused_dev [R][nh].  A regression without samples gets NaN fits, ratios
 *   and GCV and zero RSS and N_I.
 * Errors: FKR_E_ARG for a bad offset list, sizes beyond the plan's maxima or
 * bandwidths outside its range, all found before anything is enqueued. */
typedef struct fkr_batch fkr_batch;
fkr_status fkr_batch_create(const fkr_plan_desc* desc, int n_lanes, fkr_batch** out);
void fkr_batch_destroy(fkr_batch* batch);
fkr_status fkr_batch_workspace_size(const fkr_batch* batch, size_t* bytes);
fkr_status fkr_batch_set_workspace(fkr_batch* batch, void* ws_dev, size_t bytes);
fkr_status fkr_batch_cv(fkr_batch* batch, int R, const int64_t* offsets, const void* X_dev, int x_type,
                        int nh, const double* h, int q, int y_complex, const void* Y_dev, int y_type,
                        int Np, uint64_t seed, double* mhat_dev, double* rho_dev, double* rss_dev,
                        double* gcv_dev, double* nused_dev, void* stream);

/* Autotuner for a batch: runs the given batch (as fkr_batch_cv, outputs
 * discarded) once to warm up and `reps` times timed with HIP events, for
 * every lane count 1, 2, 4, .., n_lanes and, in 1-D and 2-D, for spreading
 * jobs of 1, 2 and 4 times the plan's chunk of samples per tile piece; keeps
 * the fastest configuration in the batch for later calls and reports it
 * (lanes, chunk, ms per batch; each output may be NULL).  Synchronises
 * `stream`; FKR_E_STATE when `stream` is being captured.  The outputs of
 * fkr_batch_cv do not depend on the configuration beyond the order of
 * floating-point sums.  fkr_batch_config sets a configuration directly
 * (chunk 0 keeps the current one; chunks below the plan's own, or any chunk
 * change in 3-D, are FKR_E_ARG). */
fkr_status fkr_batch_tune(fkr_batch* batch, int R, const int64_t* offsets, const void* X_dev, int x_type,
                          int nh, const double* h, int q, int y_complex, const void* Y_dev, int y_type,
                          int Np, uint64_t seed, int reps, int* lanes, int64_t* chunk, double* ms,
                          void* stream);
fkr_status fkr_batch_config(fkr_batch* batch, int lanes, int64_t chunk);

/* Bandwidth candidates (Sec. 4, get_hList), host only: n values from a to b
 * inclusive, log-spaced (kind 0, a > 0) or linearly spaced (kind 1). */
fkr_status fkr_hlist(int n, double a, double b, int kind, double* out);

/* Relaxed GCV selection (Table 1, dstd), host only: the largest index k with
 * gcv[k] <= min(gcv) + dstd * std(gcv) (std normalised by nh - 1; dstd = 0 is
 * the argmin with ties going to the later, larger bandwidth).  NaN entries are
 * skipped; FKR_E_ARG if all are NaN. */
fkr_status fkr_select_bandwidth(int nh, const double* gcv, double dstd, int* index);

/* Stage timing, for measurement (no part of the method).  While enabled, every
 * launch of a stage is bracketed by a pair of HIP events recorded on the
 * stream of the call that launches it.  fkr_profile_read waits for the
 * recorded events of one stage, returns their summed device time (ms) and
 * the number of bracketed launches since the previous read, and forgets
 * them.  FKR_STAGE_SPREAD brackets exactly one kernel per launch (the tiled
 * spread); the others may bracket a few.  Disabling drops unread records.
 * Events are created on first use and destroyed with the plan. */
typedef enum {
    FKR_STAGE_SORT = 0,      /* set_points: bin, scan, two-level scatter    */
    FKR_STAGE_WEIGHTS = 1,   /* weights gathered into sorted order          */
    FKR_STAGE_SPREAD = 2,    /* spreading onto tile subgrids (eq. 16-17)    */
    FKR_STAGE_FOLD = 3,      /* 3-D: the subgrids summed into the fine grid; 1-D and 2-D do this inside the first forward FFT pass (FKR_STAGE_FFT_FWD) */
    FKR_STAGE_FFT_FWD = 4,   /* forward FFT passes + deconvolution (eq. 19-20) */
    FKR_STAGE_EXPAND = 5,    /* kept for numbering: the channel spectra kernel is timed with the inverse passes (FKR_STAGE_FFT_INV) */
    FKR_STAGE_FFT_INV = 6,   /* inverse FFT passes + crop (eq. 21)          */
    FKR_STAGE_SOLVE = 7,     /* per-grid-point solves (eq. 3 / 11), and fkr_interval's variance of the fit */
    FKR_STAGE_REDUCE = 8,    /* interpolation + DF/RSS/variance reductions  */
    FKR_N_STAGES = 9
} fkr_stage;
fkr_status fkr_profile_enable(fkr_plan* plan, int on);
fkr_status fkr_profile_read(fkr_plan* plan, int stage, double* ms, int64_t* launches);

/* Synchronises the stream of the last call and reports the device-side
 * counters.  Returns FKR_E_STATE if a call since the last fkr_set_points
 * found other points sorted on the device than the plan's last
 * fkr_set_points left there (a replayed graph that sorted other points: the
 * call did nothing; call fkr_set_points again), FKR_E_DOMAIN if samples were
 * outside the box, FKR_WARN_ILLPOSED if the last solve produced NaN points,
 * else FKR_OK. */
fkr_status fkr_get_diagnostics(fkr_plan* plan, fkr_diag* out);

const char* fkr_status_string(fkr_status s);

#ifdef __cplusplus
}
#endif
#endif /* FKR_H */
