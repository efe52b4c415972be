// Launch interfaces of the device kernels (kernels.hip), used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "fkr_internal.h"

namespace fkr {

constexpr int kMaxPairsPerSpread = 8;
constexpr int kRedBlocks = 1024;      // fixed grid of the two-stage reductions
constexpr int kRedYCols = 1;          // response columns per fused cv reduction launch
constexpr int kRedProbes = 16;        // probes per fused cv reduction launch
constexpr int kGradCols = 32;         // response parts + probes of one GCV gradient call
constexpr int kSortChunk = 4096;      // samples per block in the binning kernels
constexpr int kSortThreads = 1024;    // threads per binning block
constexpr int kLdsHistMax = 16384;    // tiles counted in LDS (else global atomics)
constexpr int kSpreadBlock = 256;     // threads per spreading workgroup

struct Geo {                          // geometry passed by value to kernels
    int d, w;
    int64_t M[3], Mr[3], ts[3], nt[3], pe[3], B[3], K[3];
    double lo[3], hi[3], delta[3], inv_delta[3], inv_hf[3], tol[3];
    int64_t n_tiles, Psub, Mtot, Btot, Mrtot;
    int tsp, ncell;                   // tile pitch for cell ids, cells per tile
    double kparam;
    int chunk;
};

// One real weight vector for spreading / reductions.
// W_ARRAY is indexed by the original sample index, W_SORTED by the sorted position.
enum : int { W_ZERO = 0, W_ONE = 1, W_ARRAY = 2, W_PHILOX = 3, W_SORTED = 4 };
struct WSrc {
    int kind;
    int type;          // FKR_F32 / FKR_F64 for arrays
    const void* ptr;
    int64_t stride;    // element stride between samples
    int64_t col;       // element offset of this vector
    uint64_t seed;
    int probe;         // probe index (Philox)
    // W_SORTED: 0 for rows (column c of sample s at s stride + c); else the
    // columns in groups of four, [group][sample][4]: (c / 4) gstride + s stride + c % 4
    int64_t gstride;
};

struct SpreadSrc {
    int npairs;
    WSrc w[2 * kMaxPairsPerSpread];
    // optional device flag: when nonzero the first column's spread is not
    // needed (its moments are kept); the 3-D spread of one pair then spreads
    // only the second column (other paths spread both)
    const long long* keep_first;
};

struct ExpandArgs {
    int d, n_s, n_t, nreal, ncp, npairs;
    int c0;                  // first channel pair expanded (row pair c is channel pair c0 + c)
    int64_t B[3], K[3], Btot;
    double h[3], T[3];       // bandwidth and period per dimension
    unsigned long long* ill_clear;   // cleared by the launch when given
    int deriv_dim;           // >= 0: the multipliers' derivative in log h of this dimension
    const double* ktab;      // compact kernels: per dim [kdeg][B_j] multipliers (else null: the Gaussian)
    int kdeg;                // degrees in ktab (2 l + 1)
    int cpr;                 // channel pairs per workgroup row (set by the launcher)
};

// Moment multipliers of the Gaussian with a full bandwidth matrix H: the
// transform of u^a K_H(u) is (-i)^{|a|} He_a(w) exp(-w^T H w / 2) with the
// multivariate Hermite polynomials of H, He_0 = 1 and
// He_{b + e_j} = z_j He_b - sum_k b_k H_jk He_{b - e_k}, z = H w.  Per
// s-channel c (graded order) with |a_c| >= 1: the dimension j it is built
// along, the channel of b = a_c - e_j, and per k the channel of b - e_k (-1
// when b_k = 0); channels are divided by s^a, s_j = sqrt(H_jj).
struct FullH {
    double H[9];
    double s[3];
    int rj[kMaxChannels], rb[kMaxChannels], rbk[kMaxChannels][3];
    // deriv != 0: the multipliers' derivative along the symmetric direction
    // dH (the channels d/dtheta of the equilibrated moments, H + theta dH)
    int deriv;
    double dH[9];
};

// Derivative of the fits in log h_j (one dimension per launch), per grid
// point from the equilibrated channels at h (A, t) and their derivatives
// (dA, dt): d m_hat = e_0^T A^{-1} (dt - dA A^{-1} t).
struct DSolveArgs {
    int P, n_s, n_t, ncp, nr;      // nr real weights incl. the density
    int64_t Mtot;
    const float* sup;              // [M] 0 where resolved (the base solve), NaN elsewhere
    double* out;                   // [nr - 1][M]; NaN where not resolved
};

// Sums over the supported samples for the log-h gradient of GCV: columns
// c < ny sum r_ic d yhat_ic (r = y - yhat, response part c of ny = 1 real or
// 2 complex parts), column ny + p sum w_pi d what_pi, for the derivative
// grids of one dimension.
struct GradSumArgs {
    int64_t N;
    int x_type;
    const void* X;                 // sorted coordinates
    const void* wsorted;           // staged weights: 1, y, probes
    int w_type, wstride;
    int64_t wgstride;
    int ny;                        // response parts (1 real, 2 complex)
    const double* yfit;            // [M][ny] the base fit of y
    const double* dfit;            // [d][ny + Np][M] derivative grids
    const float* sup;              // [M]
    int ncol;                      // columns per dimension: ny + Np
    int col0, nall;                // columns (over all dimensions) of this launch: col0 .. col0 + nall - 1 (nall <= 32)
    double* partial;               // [slot][kRedBlocks]
};

// What a fold needs: the fine cell (c_0, .., c_{d-1}) of pair p is the sum
// over the padded tiles that cover it and the jobs of each such tile.
struct FoldArgs {
    const int32_t* cover;    // per dim: Mr_j entries of (1 + 2 kCoverSlots) int32
    const int32_t* job_off;  // [n_tiles + 1]
    const void* subgrid;     // [job][pair][Psub][re, im], spreading precision
    int64_t Psub;
    int np;                  // pairs of the launch
    int64_t nt0, nt1, pe0, pe1;
    int64_t Mr[3];
};

struct FftPass {
    int64_t rows;      // number of rows
    int64_t n_in;      // input row length
    int64_t F;         // transform length
    int64_t n_out;     // outputs per row
    int64_t K;         // band half-width (band input/output modes)
    int64_t out_estride, out_roff;
    int64_t out_rdiv, out_rmul;   // output row map: (r / rdiv) * rmul + r % rdiv
    // input element e of row r at (r / in_rdiv) in_rmul + r % in_rdiv +
    // e in_estride (in_rdiv = 0: contiguous rows of n_in)
    int64_t in_estride, in_rdiv, in_rmul;
    int in_band;       // input row holds modes -K..K (zero-padded to F)
    int out_band;      // output = modes -K..K (else indices 0..n_out-1)
    int nfac;
    int fac[kMaxFactors];
    const double* tw;  // exp(-2 pi i k / F), FP64 pairs
    const double* fac_out;  // optional real factor per output element
    int rows_per_block;
    // forward first pass only: the input rows are folded from the subgrids
    // (row = pair * rest + (c_1 + Mr_1 c_2), element = c_0) instead of read
    int fold_d;                   // 0: read `in`; else the dimension count
    int fold_f64;                 // subgrid element type
    int64_t fold_rest;            // Mr_1 Mr_2
    int fold_split;               // two threads per element (set by the launcher)
    FoldArgs fold;
    // rows below skip_rows are neither read nor written when *skip_flag is
    // nonzero (density channel pairs kept from an earlier call)
    const long long* skip_flag;
    int64_t skip_rows;
};


struct SolveArgs {
    int P, n_s, n_t, ncp, nr;      // nr real weights incl. density
    int ny, y_cplx;                // real weights 1..ny are responses
    int64_t Mtot;
    // A point is ill-posed (NaN) when a Cholesky pivot of the equilibrated
    // matrix (s_0 first) is at most max(rel_floor A_cc, abs_floor), and
    // unresolved when it is ill-posed or a pivot is at most resolve A_cc.
    double abs_floor, rel_floor, resolve;
    double* y_out;                 // [q][M][(2)] per bandwidth (may be null); NaN where ill-posed
    void* probe_out;               // [M][probe_stride], FP32 or FP64 (may be null); NaN where unresolved
    int probe_f32, probe_stride;
    int rows_with_y;               // the y fits go to the rows too: column r - 1 for weight r
    int wpg;                       // weights per thread (set by the launcher)
    double* s0_out;                // [M] (may be null)
    double* r0_out;                // [P][M] row 0 of the equilibrated inverse (may be null); NaN where ill-posed
    float* sup_out;                // [M] 0 where resolved, NaN elsewhere (may be null)
    unsigned long long* ill_count;
};

// Variance of the fit (eq. 27) per grid point from row 0 of the
// equilibrated inverse at h and the s-channels of the weights sigma_i^2 at
// h / sqrt 2 (the squared Gaussian kernel): Sigma = scale sum_bc r0_b r0_c
// fac_bc s_{b+c}, fac_bc = 2^(-|b+c|/2) re-equilibrates the channels to h.
struct IntervalArgs {
    int P;
    int64_t Mtot;
    const double* r0;              // [P][M]
    int sidx[kMaxP * kMaxP];       // s-channel of b + c
    double fac[kMaxP * kMaxP];
    double scale;                  // prod_j 1 / (2 sqrt(pi) h_j), times sigma^2 when it is a constant
    const double* mhat;            // [M] (needed for the band)
    double z;                      // z_{1 - alpha / 2}
    double* sigma;                 // [M]
    double* lower;                 // [M] (may be null)
    double* upper;                 // [M] (may be null)
};

struct ReduceCvArgs {
    int64_t N;
    int x_type;                   // element type of the sorted coordinates
    const void* X;                // sorted coordinates [N][d]
    const void* wsorted;          // staged weights: 1, y parts, probes (layout of WSrc W_SORTED)
    int w_type, wstride;
    int64_t wgstride;             // 0: rows [N][wstride]; else [group of 4][N][4], groups wgstride apart
    int ny_cols, y_cplx;          // response columns (complex: re, im parts)
    const double* yfit;           // [q][M] or [q][M][2]
    int np;                       // probes
    const void* pfit;             // [M][pstride], element type w_type
    int pstride;
    int yrow;                     // one real response whose fit is column 0 of the rows (FP32)
    int y0, ny_launch;            // response columns of this launch (<= kRedYCols)
    int p0, np_launch;            // probes of this launch (<= kRedProbes)
    const float* sup;             // [M] 0 / NaN resolved flags (read when yrow == 0)
    int count_slot;               // slot of the supported-sample count (< 0: not written)
    double* partial;              // [slot][kRedBlocks]; items: y columns, then probes, then the count
};

// Device-side record of the sorted points, checked by every kernel that
// reads a caller's per-sample array through the sort permutation.  Slots of
// the diagnostics block: kDiagN / kDiagEpoch are written by the sort (the
// point count and the host's set_points counter); a kernel launched for other
// points sets kDiagStale and does nothing (a HIP graph replay can leave the
// device with points the host did not set last).
constexpr int kDiagN = 6, kDiagEpoch = 7, kDiagStale = 8;
// Density-channel tag: the epoch and bandwidth (bit patterns) of the density
// moments in the channel buffer, and the reuse flag computed from it.
constexpr int kDiagChanEpoch = 9, kDiagChanH = 10, kDiagReuse = 13;
// Set by the variance pass's residual kernel when it leaves samples out (the
// second fit's density then differs from the first fit's: no reuse).
constexpr int kDiagResidExcl = 14;
struct PointsCheck {
    int64_t n;
    long long epoch;
    long long* diag;
};

void launch_bin_count(const Geo& g, int x_type, const void* X, int64_t N, int32_t* counts, int32_t* bhist,
                      int32_t* obuf, hipStream_t s);
void launch_scan(const Geo& g, int64_t N, long long epoch, int32_t* counts, int32_t* tile_off, int32_t* job_off,
                 int32_t* jobs, int32_t* cursor, long long* diag, const int32_t* obuf, hipStream_t s);
void launch_sort_cells(const Geo& g, int prec, int x_type, const void* X, int64_t N, int64_t n_jobs_max,
                       const int32_t* tile_off, int32_t* cursor, const int32_t* jobs, const int32_t* bhist,
                       void* trec, uint32_t* loc, void* frac, int32_t* perm, void* xs, hipStream_t s);
size_t tile_record_bytes(int d, int prec);   // bytes of one tile-ordered sample record
void launch_spread(const Geo& g, int prec, int kernel, const SpreadSrc& src, const uint32_t* loc,
                   const void* frac, const int32_t* perm, const int32_t* jobs, int64_t n_jobs_max,
                   void* subgrid, hipStream_t s);
FoldArgs fold_args(const Geo& g, int npairs, const int32_t* cover, const int32_t* job_off, const void* subgrid);
// Channel spectra [pair][band index] (pairs c_keep .. when *skip_flag is set,
// else all ncp) from the pair spectra `spec` (the forward transforms' output).
void launch_expand(int prec, const ExpandArgs& a, const int* es, const int* et, const void* spec, void* out,
                   const long long* skip_flag, int64_t c_keep, hipStream_t s);
// 3-D: the fine grid [pair][Mr^d] (transform precision) of the launch's
// pairs folded from the subgrids; the first forward pass then reads its rows.
// two_covers: no fine cell is covered by more than two padded tiles in any dimension.
void launch_fold_grid(int prec, int tprec, const Geo& g, const FoldArgs& fa, int npairs, bool two_covers,
                      void* grid, hipStream_t s);
void launch_fft(int prec, bool inverse, const FftPass& f, const void* in, void* out,
                hipStream_t s);
void launch_solve2(int prec, const SolveArgs& a, const int* pidx, const void* chan, hipStream_t s);
void launch_unpack_spec(int prec, int64_t Btot, const int64_t* B, int d, int npairs, int nw,
                        const void* spec, double* out, hipStream_t s);
void launch_chan_out(int prec, int64_t Mtot, int ncp, int n_s, int n_t, int nw, const void* chan,
                     double* S, double* T, hipStream_t s);
void launch_reduce_cv(const Geo& g, const ReduceCvArgs& a, hipStream_t s);
void launch_reduce_final(const double* partial, int nslots, double* out, hipStream_t s);
void launch_interp(const Geo& g, int nv, const double* G, int64_t Nq, const void* X,
                   int x_type, double* out, hipStream_t s);
// DF / RSS / GCV of one bandwidth from the reduced sums; the Girard mean
// comes from the probes of the sums, or from rho_in ([nh][Np]) when given.
void launch_finalize_cv(int nh_index, int Np, int q, const double* red, int n_items,
                        int ny_cols, const double* rho_in, double* rho_out, double* rss_out,
                        double* gcv_out, double* nused_out, hipStream_t s);
// residuals r_out[s] and the staged rows (1, z) of the variance pass, of
// resid_row_stride elements each (2 or 4; unused elements zero)
int resid_row_stride(const Geo& g, int prec);
// (samples whose residual is undefined get the row (0, 0) and r = NaN)
void launch_resid(const Geo& g, int prec, int mode, const PointsCheck& pc, int x_type, const void* xs,
                  const int32_t* perm, int y_type, const void* Y, int y_cplx, const double* mhat, double* r_out,
                  void* rows, hipStream_t s);
// partial sums of r exp(-v) (slot 0) and of their count (slot 1) over the
// samples where the term is defined
void launch_kappa_partial(const Geo& g, int64_t N, int x_type, const void* xs, const int32_t* perm,
                          const double* vhat, const double* r, double* partial, hipStream_t s);
void launch_sigma2(int64_t Mtot, const double* vhat, const double* kappa_sums, double* sigma2,
                   double* kappa_out, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
void launch_dsolve(int prec, const DSolveArgs& a, const int* pidx, const void* chan_base, const void* chan_der,
                   hipStream_t s);
void launch_grad_sums(const Geo& g, const GradSumArgs& a, hipStream_t s);
void launch_finalize_grad(int d, int ny, int Np, const double* red, const double* gred, double* gcv, double* dlogh,
                          hipStream_t s);
void launch_adj_scatter(const Geo& g, int64_t N, int prec, const void* X, const void* W, int wstride,
                        int64_t wgstride, int ny, const double* yfit, const float* sup, double* u, hipStream_t s);
void launch_adj_pack(int prec, int P, int64_t Mtot, const double* u, const double* c, int cplx, void* out,
                     hipStream_t s);
void launch_adj_combine(int prec, const ExpandArgs& a, int P, int cplx, const int* et, const double* fac,
                        const void* spec, void* out, hipStream_t s);
// k_adj_combine with the multipliers of a full bandwidth matrix fh (es, pidx:
// the s-channel exponents and the t-to-s channel map)
void launch_adj_combine_full(int prec, const ExpandArgs& a, const FullH& fh, int P, int cplx, const int* es,
                             const int* pidx, const double* fac, const void* spec, void* out, hipStream_t s);
void launch_adj_gather(const Geo& g, int prec, int tprec, int kernel, int Np, int64_t n_jobs_max,
                       const int32_t* jobs, const uint32_t* loc, const void* frac, const void* X,
                       const int32_t* perm, const void* fgrid, int ny, int part, const double* yfit, const float* sup,
                       const void* W, int wstride, int64_t wgstride, const double* red, double* grad, hipStream_t s);
// The library-held workspace of the current device (fkr_fit_noalloc):
// kStaticScratchBytes, 256-byte aligned.
constexpr size_t kStaticScratchBytes = FKR_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(void** ptr);
// gstride 0: rows [N][nr]; else columns in groups of four, [group][N][4] with
// groups gstride elements apart (FP32 only).
void launch_stage_weights(int prec, const SpreadSrc& src, int nsrc, int r0, int nr, int64_t gstride, const PointsCheck& pc,
                          const int32_t* perm, void* out, hipStream_t s);
void launch_ktab(const ExpandArgs& a, const double* delta, int reg_kernel, int square, double* ktab, hipStream_t s);
void launch_expand_full(int prec, const ExpandArgs& a, const FullH& fh, const int* es, const int* pidx,
                        const void* spec, void* out, hipStream_t s);
void launch_chan_tag(long long* diag, const double* h, int d, hipStream_t s);
void launch_chan_untag(long long* diag, hipStream_t s);
void launch_stage_grid(const Geo& g, int prec, const PointsCheck& pc, const void* xs, const double* G, void* rows,
                       hipStream_t s);
void launch_interval(int prec, const IntervalArgs& a, const void* chan, hipStream_t s);
void launch_spline(const Geo& g, int nv, const double* G, double* coef, hipStream_t s);
void launch_spline_eval(const Geo& g, int nv, const double* coef, int64_t Nq, const void* X, int x_type,
                        double* out, hipStream_t s);
void launch_chan_reuse(long long* diag, const double* h, int d, hipStream_t s);

}  // namespace fkr
