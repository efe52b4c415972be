// C ABI of the fast kernel-regression library: argument checks, workspace
// binding and the order of device stages for each call (declared in fkr.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fkr_internal.h"
#include "kernels.h"

using namespace fkr;

namespace {

#define FKR_HIP(call)                                      \
    do {                                                   \
        if ((call) != hipSuccess) return FKR_E_DEVICE;     \
    } while (0)

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

template <typename P> P* at(fkr_plan* p, size_t off) { return reinterpret_cast<P*>(p->ws + off); }

// Stage timing: an event pair around the launches of one scope.
hipEvent_t record_event(fkr_plan* p, hipStream_t s) {
    hipEvent_t e = nullptr;
    if (!p->ev_free.empty()) {
        e = p->ev_free.back();
        p->ev_free.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    if (hipEventRecord(e, s) != hipSuccess) {
        p->ev_free.push_back(e);
        return nullptr;
    }
    return e;
}

struct StageTimer {
    fkr_plan* p;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageTimer(fkr_plan* p_, int stage_, hipStream_t s_) : p(p_), stage(stage_), s(s_) {
        if (p->prof_on) a = record_event(p, s);
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = record_event(p, s);
        if (b) p->ev_pairs[stage].emplace_back(a, b);
        else p->ev_free.push_back(a);
    }
};

Geo make_geo(const fkr_plan* p) {
    Geo g{};
    g.d = p->d;
    g.w = p->w;
    for (int j = 0; j < 3; ++j) {
        g.M[j] = p->M[j]; g.Mr[j] = p->Mr[j]; g.ts[j] = p->ts[j]; g.nt[j] = p->nt[j];
        g.pe[j] = p->pe[j]; g.B[j] = p->B[j]; g.K[j] = p->K[j];
        g.lo[j] = p->lo[j]; g.hi[j] = p->hi[j]; g.delta[j] = p->delta[j];
        g.inv_delta[j] = j < p->d ? 1.0 / p->delta[j] : 1.0;
        g.inv_hf[j] = p->inv_hf[j];
        g.tol[j] = j < p->d ? 1e-12 * (p->hi[j] - p->lo[j]) : 0.0;
    }
    g.n_tiles = p->n_tiles; g.Psub = p->Psub; g.Mtot = p->Mtot; g.Btot = p->Btot; g.Mrtot = p->Mrtot;
    g.kparam = p->kparam;
    g.chunk = p->chunk;
    g.tsp = p->tsp;
    g.ncell = p->ncell;
    return g;
}

bool valid_type(int t) { return t == FKR_F32 || t == FKR_F64; }

fkr_status check_h(const fkr_plan* p, int nh, const double* h) {
    if (nh < 1 || nh > p->max_h || !h) return FKR_E_ARG;
    for (int q = 0; q < nh; ++q)
        for (int j = 0; j < p->d; ++j) {
            const double v = h[q * p->d + j];
            if (!(v >= p->h_min[j] * (1 - 1e-12) && v <= p->h_max[j] * (1 + 1e-12))) return FKR_E_ARG;
        }
    return FKR_OK;
}

fkr_status ready(const fkr_plan* p) {
    if (!p) return FKR_E_ARG;
    if (!p->ws_ready) return FKR_E_WORKSPACE;
    if (!p->points_set) return FKR_E_STATE;
    return FKR_OK;
}

WSrc src_one() { WSrc w{}; w.kind = W_ONE; return w; }
WSrc src_zero() { WSrc w{}; w.kind = W_ZERO; return w; }
WSrc src_array(const void* ptr, int type, int64_t stride, int64_t col) {
    WSrc w{}; w.kind = W_ARRAY; w.type = type; w.ptr = ptr; w.stride = stride; w.col = col; return w;
}
WSrc src_philox(uint64_t seed, int probe) { WSrc w{}; w.kind = W_PHILOX; w.seed = seed; w.probe = probe; return w; }

const int* dev_es(fkr_plan* p) { return at<int>(p, p->lay.consts + 64); }
const int* dev_et(fkr_plan* p) { return at<int>(p, p->lay.consts + 64 + 512); }
const int* dev_pidx(fkr_plan* p) { return at<int>(p, p->lay.consts + 64 + 1024); }
unsigned long long* ill_ctr(fkr_plan* p) { return at<unsigned long long>(p, p->lay.diag + 2 * 8); }
long long* diag_ptr(fkr_plan* p) { return at<long long>(p, p->lay.diag); }
PointsCheck points_check(fkr_plan* p) { return PointsCheck{p->N, p->epoch, diag_ptr(p)}; }

// The staged weights are grouped by four columns, [group][N][4], where the
// 3-D FP32 w = 8 spread reads them: each of its passes takes one group, so it
// streams exactly the 16 bytes per sample it uses.  Elsewhere they are rows.
bool grouped_weights(const fkr_plan* p) { return p->d == 3 && p->prec == FKR_F32 && p->w == 8; }

// Every fine cell is covered by its own padded tile and at most the previous
// one in each dimension (no padded tile wider than the period, so none covers
// a cell twice): the fold's workgroups then share their covering tiles.
bool fold_two_covers(const fkr_plan* p) {
    if (p->max_cover > 2) return false;
    for (int j = 0; j < p->d; ++j)
        if (p->pe[j] > p->Mr[j]) return false;
    return true;
}

// Every weight vector of a call, constants included, gathered once into
// sorted sample order: `stride` = nr rounded up to 4 columns (16-byte loads;
// padding columns are zero), as rows [N][stride] or as column groups.
std::vector<WSrc> stage_weights(fkr_plan* p, const std::vector<WSrc>& srcs, hipStream_t s) {
    const int nr = (int)srcs.size();
    const int stride = (nr + 3) & ~3;
    const int64_t gstride = grouped_weights(p) ? 4 * p->N : 0;
    std::vector<WSrc> all(srcs);
    all.resize(stride, src_zero());
    void* buf = p->ws + p->lay.wsort;
    for (int r0 = 0; r0 < stride; r0 += 2 * kMaxPairsPerSpread) {
        SpreadSrc chunk{};
        const int n = std::min(2 * kMaxPairsPerSpread, stride - r0);
        for (int q = 0; q < n; ++q) chunk.w[q] = all[r0 + q];
        StageTimer t(p, FKR_STAGE_WEIGHTS, s);
        launch_stage_weights(p->prec, chunk, n, r0, stride, gstride, points_check(p), at<int32_t>(p, p->lay.perm),
                             buf, s);
    }
    std::vector<WSrc> out(stride);
    for (int r = 0; r < stride; ++r) {
        WSrc w{};
        w.kind = W_SORTED; w.type = p->prec; w.ptr = buf; w.stride = gstride ? 4 : stride; w.col = r;
        w.gstride = gstride;
        out[r] = w;
    }
    return out;
}

// Spread + fold + forward FFT of every weight pair -> spec [band][npairs].
// With staged = true the sources already are columns of the staged rows.
fkr_status run_spectra(fkr_plan* p, const std::vector<WSrc>& srcs_in, hipStream_t s, bool staged,
                       const long long* keep_first = nullptr) {
    const std::vector<WSrc> srcs = staged ? srcs_in : stage_weights(p, srcs_in, s);   // padded to a multiple of 4
    const Geo g = make_geo(p);
    const int nr = (int)srcs_in.size();
    const int npairs = (nr + 1) / 2;
    if (npairs > p->npairs_max) return FKR_E_ARG;
    const size_t csz = 2 * elem_size(p->prec);
    for (int p0 = 0; p0 < npairs; p0 += p->pairs_per_spread) {
        const int gp = std::min(p->pairs_per_spread, npairs - p0);
        SpreadSrc src{};
        src.npairs = gp;
        src.keep_first = p0 == 0 ? keep_first : nullptr;
        for (int q = 0; q < gp; ++q) {
            const int r0 = 2 * (p0 + q), r1 = r0 + 1;
            src.w[2 * q] = srcs[r0];
            src.w[2 * q + 1] = srcs[r1];   // column nr (odd nr) is staged as zeros
        }
        {
            StageTimer t(p, FKR_STAGE_SPREAD, s);
            launch_spread(g, p->prec, p->kernel, src, at<uint32_t>(p, p->lay.loc), p->ws + p->lay.frac,
                          at<int32_t>(p, p->lay.perm), at<int32_t>(p, p->lay.jobs), p->n_jobs_max,
                          p->ws + p->lay.subgrid, s);
        }
        // In 1-D and 2-D the first forward pass folds its rows from the
        // subgrids itself; in 3-D the fold writes the fine grid first, one
        // workgroup per tile (the subgrids are read once, in runs).
        const void* in = nullptr;
        const bool grid_fold = p->d == 3;
        if (grid_fold) {
            StageTimer tg(p, FKR_STAGE_FOLD, s);
            launch_fold_grid(p->prec, p->tprec, g,
                             fold_args(g, gp, at<int32_t>(p, p->lay.cover), at<int32_t>(p, p->lay.job_off),
                                       p->ws + p->lay.subgrid),
                             gp, fold_two_covers(p), p->ws + p->lay.fftB, s);
            in = p->ws + p->lay.fftB;
        }
        StageTimer tf(p, FKR_STAGE_FFT_FWD, s);
        int64_t done_B = 1;
        for (int j = 0; j < p->d; ++j) {
            FftPass f{};
            int64_t rest = 1;
            for (int i = j + 1; i < p->d; ++i) rest *= p->Mr[i];
            f.rows = done_B * gp * rest;
            f.n_in = p->Mr[j];
            f.F = p->Mr[j];
            f.n_out = p->B[j];
            f.K = p->K[j];
            f.in_band = 0;
            f.out_band = 1;
            if (j == 0 && !grid_fold) {
                f.fold_d = p->d;
                f.fold_f64 = p->prec == FKR_F64 ? 1 : 0;
                f.fold_rest = rest;
                f.fold = fold_args(g, gp, at<int32_t>(p, p->lay.cover), at<int32_t>(p, p->lay.job_off),
                                   p->ws + p->lay.subgrid);
            }
            f.nfac = p->fMr[j].nfac;
            for (int q = 0; q < p->fMr[j].nfac; ++q) f.fac[q] = p->fMr[j].fac[q];
            f.tw = at<double>(p, p->fMr[j].tw_off);
            size_t doff = p->lay.deconv;
            for (int i = 0; i < j; ++i) doff += p->B[i] * 8;
            f.fac_out = at<double>(p, doff);
            void* out;
            if (j == p->d - 1) {
                out = p->ws + p->lay.spec;
                f.out_estride = done_B * npairs;
                f.out_roff = p0;
                f.out_rdiv = gp;
                f.out_rmul = npairs;
            } else {
                out = p->ws + ((j % 2 == 0) ? p->lay.fftA : p->lay.fftB);
                f.out_estride = f.rows;
                f.out_roff = 0;
                f.out_rdiv = f.rows;
                f.out_rmul = 0;
            }
            launch_fft(p->tprec, false, f, in, out, s);
            in = out;
            done_B *= p->B[j];
        }
        (void)csz;
    }
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

// Channels at one bandwidth h: expansion + inverse FFT -> chan [pair][M][re, im].
// Weight 0 of the spectra is the density in every caller, so afterwards the
// first n_s / 2 pairs hold its moments s_alpha at h, and (when n_s is even) a
// device tag records the points epoch and h they belong to.  With reuse, the
// passes skip those pairs when the tag already matches (the density moments
// depend on the points and h only); the decision is taken on the device, so a
// captured graph stays valid whatever ran before its replay.
// tag: 1 records the density tag (weight 0 is the unit density), 0 clears
// it (weight 0 is not the density), 2 leaves it (the call writes only pairs
// above the density moments).  deriv_dim >= 0 expands the derivatives of the
// channels in log h of that dimension; pair_off places the channels that
// many pairs up in the channel buffer.  ksq (compact kernels): the moments
// of the squared kernel prod_j K(u_j / h_j)^2 / h_j (the caller untags).
fkr_status run_channels(fkr_plan* p, const double* h, int nr, unsigned long long* ill_clear, hipStream_t s,
                        bool reuse = false, int tag = 1, int deriv_dim = -1, int64_t pair_off = 0,
                        const FullH* full = nullptr, bool ksq = false) {
    const int nreal = p->n_s + p->n_t * (nr - 1);
    const int ncp = (nreal + 1) / 2;
    if (ncp + pair_off > p->ncp_max) return FKR_E_ARG;
    if (pair_off > 0 && reuse) return FKR_E_ARG;
    const bool even = p->n_s % 2 == 0;
    reuse = reuse && even;
    const int64_t c_keep = reuse ? p->n_s / 2 : 0;   // pairs a matching tag lets the passes skip
    if (reuse) launch_chan_reuse(diag_ptr(p), h, p->d, s);
    const long long* skip_flag = reuse ? diag_ptr(p) + kDiagReuse : nullptr;
    ExpandArgs a{};
    a.d = p->d; a.n_s = p->n_s; a.n_t = p->n_t; a.nreal = nreal; a.ncp = ncp;
    a.c0 = 0;
    a.npairs = (nr + 1) / 2;
    for (int j = 0; j < 3; ++j) { a.B[j] = p->B[j]; a.K[j] = p->K[j]; }
    for (int j = 0; j < p->d; ++j) { a.h[j] = h[j]; a.T[j] = p->T[j]; }
    a.Btot = p->Btot;
    a.ill_clear = ill_clear;
    a.deriv_dim = deriv_dim;
    if (p->reg_kernel && !full) {
        a.kdeg = 2 * p->order + 1;
        a.ktab = at<double>(p, p->lay.ktab);
        launch_ktab(a, p->delta, p->reg_kernel, ksq ? 1 : 0, at<double>(p, p->lay.ktab), s);
    }
    // the first inverse pass expands its rows from the pair spectra itself
    StageTimer tf(p, FKR_STAGE_FFT_INV, s);
    void* chan_out = p->ws + p->lay.chan + (size_t)pair_off * p->Mtot * 2 * elem_size(p->tprec);
    auto pass = [&](int j) {
        FftPass f{};
        f.n_in = p->B[j];
        f.F = p->L[j];
        f.n_out = p->M[j];
        f.K = p->K[j];
        f.in_band = 1;
        f.out_band = 0;
        f.nfac = p->fL[j].nfac;
        for (int q = 0; q < p->fL[j].nfac; ++q) f.fac[q] = p->fL[j].fac[q];
        f.tw = at<double>(p, p->fL[j].tw_off);
        f.fac_out = nullptr;
        f.skip_flag = skip_flag;
        return f;
    };
    // The channel spectra [pair][band index e_0 + B_0 e_1 + ..] first, then
    // dimensions d-1 .. 0.  Before the pass along dimension j the rows are
    // (pair, e_{j-1} .. e_0, m_{d-1} .. m_{j+1}) with the pair outermost and
    // e_0 fastest among the band indices, m_{j+1} fastest among the grid
    // ones; the pass reads element e_j at row stride R (the other indices'
    // extent) and writes each row's M_j outputs contiguously, so every pass
    // stores whole rows and the last one leaves the channels pair-major,
    // [pair][M^d][re, im] with m_0 fastest.
    if (full)
        launch_expand_full(p->tprec, a, *full, dev_es(p), dev_pidx(p), p->ws + p->lay.spec, p->ws + p->lay.fftB, s);
    else
        launch_expand(p->tprec, a, dev_es(p), dev_et(p), p->ws + p->lay.spec, p->ws + p->lay.fftB, skip_flag, c_keep,
                      s);
    const void* in = p->ws + p->lay.fftB;
    for (int j = p->d - 1; j >= 0; --j) {
        FftPass f = pass(j);
        int64_t R = 1;
        for (int i = 0; i < j; ++i) R *= p->B[i];
        for (int i = j + 1; i < p->d; ++i) R *= p->M[i];
        f.rows = ncp * R;
        f.skip_rows = c_keep * R;
        f.in_rdiv = R;
        f.in_rmul = p->B[j] * R;
        f.in_estride = R;
        f.out_estride = 1;
        f.out_roff = 0;
        f.out_rdiv = 1;
        f.out_rmul = p->M[j];
        void* out;
        if (j == 0) out = chan_out;
        else out = p->ws + (in == p->ws + p->lay.fftA ? p->lay.fftB : p->lay.fftA);   // fftA first
        launch_fft(p->tprec, true, f, in, out, s);
        in = out;
    }
    if (tag == 0) launch_chan_untag(diag_ptr(p), s);
    else if (tag == 1 && even) launch_chan_tag(diag_ptr(p), h, p->d, s);
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

// Ill-posedness floors of the solve.  The moments are known to about a
// relative 1e-6 of their local size with FP32 spreading (the spreading
// kernel's values carry FP32 round-off; the LDS sums are FP64) and to about
// the requested accuracy eps otherwise (the spreading kernel is sized for
// eps / 10), so a pivot below rel_floor A_cc = max(64 unit round-offs,
// 10 eps) A_cc cannot be told from a singular direction.  Globally the transforms add an error of
// about the transform round-off (16 units) or 1e-5 of the requested accuracy
// times N K_h(0), the largest value s_0 can take; a pivot below that absolute
// floor is noise.  (Measured on the workloads: relative errors of 3e-7 to
// 8e-6 with FP32 spreading, absolute errors below 3.1e-12 N K_h(0) with FP64
// transforms and below 2e-7 N K_h(0) with FP32 transforms.)
double abs_floor(const fkr_plan* p, const double* h) {
    // the kernel's peak K_h(0) = prod_j K(0) / h_j
    static const double k_peak[] = {0.0, 0.5, 1.0, 0.75, 0.9375, 1.09375};
    const double kz = p->reg_kernel ? k_peak[p->reg_kernel] : 1.0 / std::sqrt(2.0 * M_PI);
    double k0 = 1.0;
    for (int j = 0; j < p->d; ++j) k0 *= kz / h[j];
    const double u32 = 5.9604644775390625e-08, u64 = 1.1102230246251565e-16;
    const double ut = p->tprec == FKR_F64 ? u64 : u32;
    const double e = std::max(16.0 * ut, 1e-5 * p->eps);
    return std::max(1e-300, e * (double)std::max<int64_t>(p->N, 1) * k0);
}

double rel_floor(const fkr_plan* p) {
    const double u32 = 5.9604644775390625e-08, u64 = 1.1102230246251565e-16;
    return std::max(64.0 * (p->prec == FKR_F64 ? u64 : u32), 10.0 * p->eps);
}

SolveArgs solve_args(fkr_plan* p, int nr, int ny, int y_cplx, const double* h) {
    SolveArgs a{};
    a.P = p->n_t; a.n_s = p->n_s; a.n_t = p->n_t;
    a.ncp = (p->n_s + p->n_t * (nr - 1) + 1) / 2;
    a.nr = nr; a.ny = ny; a.y_cplx = y_cplx;
    a.Mtot = p->Mtot;
    a.abs_floor = abs_floor(p, h);
    a.rel_floor = rel_floor(p);
    a.resolve = FKR_RESOLVE;
    a.ill_count = at<unsigned long long>(p, p->lay.diag + 2 * 8);
    return a;
}

// Response sources: each real column (or re/im of complex columns).
void add_response_sources(std::vector<WSrc>* v, int q, int y_cplx, const void* Y, int y_type) {
    const int cpl = y_cplx ? 2 : 1;
    for (int c = 0; c < q; ++c)
        for (int part = 0; part < cpl; ++part) v->push_back(src_array(Y, y_type, (int64_t)q * cpl, c * cpl + part));
}

void add_probe_sources(std::vector<WSrc>* v, int Np, uint64_t seed, const void* probes, int w_type) {
    for (int pr = 0; pr < Np; ++pr)
        v->push_back(probes ? src_array(probes, w_type, Np, pr) : src_philox(seed, pr));
}

fkr_status common_fit_checks(fkr_plan* p, int nh, const double* h, int q, int y_complex, const void* Y,
                             int y_type) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if ((st = check_h(p, nh, h)) != FKR_OK) return st;
    if (q < 0 || (q > 0 && !Y && p->N > 0) || (y_complex != 0 && y_complex != 1)) return FKR_E_ARG;
    if (q > 0 && !valid_type(y_type)) return FKR_E_ARG;
    return FKR_OK;
}

// Fits, DF and RSS of a bandwidth list (the batched loop of Sec. 2 and
// Fig. 3).  With rho_in the DF is given (fkr_gcv): no probes are spread and
// the GCV uses the given Girard ratios.  With fh (and heff) the list is one
// of full bandwidth matrices: the channels of matrix hi use fh[hi], the
// solve heff[3 hi ..].
fkr_status cv_impl(fkr_plan* p, int nh, const double* h, int q, int y_complex, const void* Y, int y_type, int Np,
                   uint64_t seed, const void* probes, const double* rho_in, double* mhat, double* rho, double* rss,
                   double* gcv, double* nused, hipStream_t s, const FullH* fh = nullptr,
                   const double* heff = nullptr) {
    fkr_status st;
    const int cpl = y_complex ? 2 : 1;
    const int ny = q * cpl;
    const int Ns = rho_in ? 0 : Np;   // probes that are spread
    const int ptype = y_type;
    std::vector<WSrc> srcs{src_one()};
    add_response_sources(&srcs, q, y_complex, Y, y_type);
    add_probe_sources(&srcs, Ns, seed, probes, ptype);
    if ((st = run_spectra(p, srcs, s, false)) != FKR_OK) return st;
    const Geo g = make_geo(p);
    const int nr = (int)srcs.size();
    double* internal = at<double>(p, p->lay.mhat);
    // probe fits [M][pstride] in the spreading precision (they only feed the
    // DF reduction), 16-byte aligned rows for FP32
    const bool pf32 = p->prec == FKR_F32;
    // one real response and all probes in one reduction launch: the y fit
    // rides in column 0 of the FP32 rows, so the reduction gathers one row
    // (NaN rows mark the corners that are not resolved)
    const bool yrow = pf32 && q == 1 && !y_complex && Ns <= kRedProbes;
    const int pstride = pf32 ? ((yrow ? 1 : 0) + Ns + 3) & ~3 : std::max(Ns, 1);
    void* pfit = p->ws + p->lay.mhat + (((size_t)ny * p->Mtot * 8 + 15) & ~(size_t)15);
    double* red = at<double>(p, p->lay.red);
    double* partial = at<double>(p, p->lay.partial);
    float* sup = at<float>(p, p->lay.sup);
    const int n_items = q + Ns;
    for (int hi = 0; hi < nh; ++hi) {
        unsigned long long* ill = hi == 0 ? ill_ctr(p) : nullptr;
        // full H: channels under K_H (no density tag: they are not the
        // moments of a diagonal bandwidth)
        st = fh ? run_channels(p, fh[hi].s, nr, ill, s, false, 0, -1, 0, &fh[hi])
                : run_channels(p, h + hi * p->d, nr, ill, s);
        if (st != FKR_OK) return st;
        SolveArgs a = solve_args(p, nr, ny, y_complex, fh ? heff + 3 * hi : h + hi * p->d);
        double* yfit = mhat ? mhat + (int64_t)hi * ny * p->Mtot : internal;
        a.y_out = yfit;
        a.probe_out = (yrow || Ns > 0) ? pfit : nullptr;
        a.probe_f32 = pf32 ? 1 : 0;
        a.probe_stride = pstride;
        a.rows_with_y = yrow ? 1 : 0;
        a.sup_out = sup;
        {
            StageTimer t(p, FKR_STAGE_SOLVE, s);
            launch_solve2(p->tprec, a, dev_pidx(p), p->ws + p->lay.chan, s);
        }
        ReduceCvArgs r{};
        r.N = p->N; r.x_type = p->prec; r.X = p->ws + p->lay.xs;
        r.wsorted = p->ws + p->lay.wsort; r.w_type = p->prec;
        r.wgstride = grouped_weights(p) ? 4 * p->N : 0;
        r.wstride = r.wgstride ? 4 : (nr + 3) & ~3;
        r.ny_cols = q; r.y_cplx = y_complex; r.yfit = yfit;
        r.np = Ns; r.pfit = pfit; r.pstride = pstride; r.yrow = yrow ? 1 : 0;
        r.sup = sup;
        r.partial = partial;
        StageTimer t(p, FKR_STAGE_REDUCE, s);
        // probes per launch: at most kRedProbes, spread evenly over the launches
        const int nlp = (Ns + kRedProbes - 1) / kRedProbes;
        const int pper = nlp > 0 ? (Ns + nlp - 1) / nlp : 0;
        const int nlaunch = std::max(std::max((q + kRedYCols - 1) / kRedYCols, nlp), 1);
        for (int li = 0; li < nlaunch; ++li) {
            r.y0 = li * kRedYCols;
            r.ny_launch = std::max(0, std::min(kRedYCols, q - r.y0));
            r.p0 = li * pper;
            r.np_launch = std::max(0, std::min(pper, Ns - r.p0));
            r.count_slot = li == 0 ? 2 * n_items : -1;   // every launch counts the same samples
            launch_reduce_cv(g, r, s);
        }
        launch_reduce_final(partial, 2 * n_items + 1, red, s);
        launch_finalize_cv(hi, Np, q, red, n_items, q, rho_in, rho, rss, gcv, nused, s);
    }
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

// The plan's constant tables (periods, channel exponents, pair index,
// deconvolution factors, twiddles, tile cover lists) as (workspace offset,
// bytes) blobs.
std::vector<std::pair<size_t, std::vector<unsigned char>>> constant_tables(const fkr_plan* p) {
    std::vector<std::pair<size_t, std::vector<unsigned char>>> out;
    auto add = [&](size_t off, const void* data, size_t n) {
        const unsigned char* c = static_cast<const unsigned char*>(data);
        out.emplace_back(off, std::vector<unsigned char>(c, c + n));
    };
    std::vector<unsigned char> consts(4096, 0);
    double* per = reinterpret_cast<double*>(consts.data());
    for (int j = 0; j < p->d; ++j) per[j] = p->T[j];
    int* es = reinterpret_cast<int*>(consts.data() + 64);
    int* et = reinterpret_cast<int*>(consts.data() + 64 + 512);
    int* pi = reinterpret_cast<int*>(consts.data() + 64 + 1024);
    for (int c = 0; c < p->n_s; ++c) for (int j = 0; j < 3; ++j) es[3 * c + j] = p->es[c][j];
    for (int c = 0; c < p->n_t; ++c) for (int j = 0; j < 3; ++j) et[3 * c + j] = p->et[c][j];
    for (int b = 0; b < kMaxP; ++b) for (int c = 0; c < kMaxP; ++c) pi[b * kMaxP + c] = p->pair_index[b][c];
    add(p->lay.consts, consts.data(), consts.size());
    size_t off = p->lay.deconv;
    for (int j = 0; j < p->d; ++j) {
        add(off, p->deconv[j].data(), p->deconv[j].size() * 8);
        off += p->deconv[j].size() * 8;
        std::vector<double> tw;
        twiddle_table(p->Mr[j], &tw);
        add(p->fMr[j].tw_off, tw.data(), tw.size() * 8);
        twiddle_table(p->L[j], &tw);
        add(p->fL[j].tw_off, tw.data(), tw.size() * 8);
    }
    off = p->lay.cover;
    for (int j = 0; j < p->d; ++j) {
        add(off, p->cover[j].data(), p->cover[j].size() * 4);
        off += p->cover[j].size() * 4;
    }
    return out;
}

// A full bandwidth matrix (d x d, row-major): symmetric, positive definite,
// its marginal standard deviations s_j = sqrt(H_jj) within the plan's h_max
// (the zero padding covers the kernel's reach along each axis) and its
// spectrum's reach along each frequency axis, 1 / sqrt((H^-1)_jj), at least
// the plan's h_min (the band holds it).  Fills the Hermite recurrence tables
// and heff, per-dimension widths with prod heff = sqrt(det H) (the kernel's
// peak, for the ill-posedness floor).
fkr_status build_full(const fkr_plan* p, const double* H, FullH* fh, double* heff) {
    const int d = p->d;
    *fh = FullH{};
    double A[3][3] = {};
    for (int j = 0; j < d; ++j)
        for (int k = 0; k < d; ++k) {
            const double v = H[j * d + k];
            if (!std::isfinite(v)) return FKR_E_ARG;
            A[j][k] = v;
            fh->H[3 * j + k] = v;
        }
    for (int j = 0; j < d; ++j)
        for (int k = 0; k < j; ++k)
            if (std::fabs(A[j][k] - A[k][j]) > 1e-12 * std::sqrt(std::fabs(A[j][j] * A[k][k]))) return FKR_E_ARG;
    // Cholesky H = L L^T
    double L[3][3] = {};
    double det = 1.0;
    for (int c = 0; c < d; ++c) {
        double v = A[c][c];
        for (int q = 0; q < c; ++q) v -= L[c][q] * L[c][q];
        if (!(v > 0.0)) return FKR_E_ARG;
        L[c][c] = std::sqrt(v);
        det *= v;
        for (int b = c + 1; b < d; ++b) {
            double u = A[b][c];
            for (int q = 0; q < c; ++q) u -= L[b][q] * L[c][q];
            L[b][c] = u / L[c][c];
        }
    }
    // (H^-1)_jj = || L^-1 e_j ||^2
    for (int j = 0; j < d; ++j) {
        double y[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < d; ++b) {
            double v = b == j ? 1.0 : 0.0;
            for (int q = 0; q < b; ++q) v -= L[b][q] * y[q];
            y[b] = v / L[b][b];
        }
        double ii = 0.0;
        for (int b = 0; b < d; ++b) ii += y[b] * y[b];
        const double sj = std::sqrt(A[j][j]);
        fh->s[j] = sj;
        if (sj > p->h_max[j] * (1 + 1e-12)) return FKR_E_ARG;
        if (1.0 / std::sqrt(ii) < p->h_min[j] * (1 - 1e-12)) return FKR_E_ARG;
    }
    double sprod = 1.0;
    for (int j = 0; j < d; ++j) sprod *= fh->s[j];
    const double shrink = std::pow(std::sqrt(det) / sprod, 1.0 / d);
    for (int j = 0; j < d; ++j) heff[j] = fh->s[j] * shrink;
    auto find = [&](const int* e) {
        for (int c = 0; c < p->n_s; ++c) {
            bool eq = true;
            for (int k = 0; k < d; ++k) eq &= p->es[c][k] == e[k];
            if (eq) return c;
        }
        return -1;
    };
    for (int c = 1; c < p->n_s; ++c) {
        int j = 0;
        while (p->es[c][j] == 0) ++j;
        int b[3] = {p->es[c][0], p->es[c][1], p->es[c][2]};
        b[j] -= 1;
        fh->rj[c] = j;
        fh->rb[c] = find(b);
        for (int k = 0; k < 3; ++k) {
            fh->rbk[c][k] = -1;
            if (k < d && b[k] > 0) {
                int bk[3] = {b[0], b[1], b[2]};
                bk[k] -= 1;
                fh->rbk[c][k] = find(bk);
            }
        }
    }
    return FKR_OK;
}

// z with Phi(z) = 1 - alpha / 2 (the quantile of eq. 28): bisection on the
// decreasing upper tail Q(z) = erfc(z / sqrt 2) / 2 until the bracket stops
// shrinking, so z is as accurate as the library's erfc.
double upper_quantile(double alpha) {
    double lo = 0.0, hi = 40.0;
    const double target = 0.5 * alpha;
    for (int it = 0; it < 256; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (0.5 * std::erfc(mid / std::sqrt(2.0)) > target) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// The argument checks of fkr_fit that do not need points on the device.
fkr_status st_check_fit(const fkr_plan* p, int nh, const double* h, int q, int y_complex, const void* Y,
                        int y_type, const double* mhat) {
    if (check_h(p, nh, h) != FKR_OK) return FKR_E_ARG;
    if (q < 1 || !mhat || !Y || (y_complex != 0 && y_complex != 1) || !valid_type(y_type)) return FKR_E_ARG;
    if (1 + q * (y_complex ? 2 : 1) > p->max_weights) return FKR_E_ARG;
    return FKR_OK;
}

}  // namespace

extern "C" {

const char* fkr_status_string(fkr_status s) {
    switch (s) {
        case FKR_OK: return "ok";
        case FKR_WARN_ILLPOSED: return "some grid points are ill-posed (NaN)";
        case FKR_E_ARG: return "invalid argument";
        case FKR_E_DOMAIN: return "samples outside the grid box";
        case FKR_E_WORKSPACE: return "workspace missing or too small";
        case FKR_E_DEVICE: return "HIP runtime error";
        case FKR_E_UNSUPPORTED: return "unsupported configuration";
        case FKR_E_STATE: return "call order violated (no points set)";
    }
    return "unknown status";
}

fkr_status fkr_plan_create(const fkr_plan_desc* desc, fkr_plan** out) {
    if (!desc || !out) return FKR_E_ARG;
    *out = nullptr;
    fkr_plan* p = new (std::nothrow) fkr_plan();
    if (!p) return FKR_E_ARG;
    const fkr_status st = build_plan(desc, p);
    if (st != FKR_OK) {
        delete p;
        return st;
    }
    *out = p;
    return FKR_OK;
}

void fkr_plan_destroy(fkr_plan* p) { delete p; }

fkr_status fkr_plan_geometry(const fkr_plan* p, fkr_geometry* g) {
    if (!p || !g) return FKR_E_ARG;
    std::memset(g, 0, sizeof(*g));
    g->d = p->d; g->order = p->order; g->n_s = p->n_s; g->n_t = p->n_t;
    for (int j = 0; j < FKR_MAX_D; ++j) {
        const bool on = j < p->d;
        g->M[j] = on ? p->M[j] : 1; g->L[j] = on ? p->L[j] : 1; g->K[j] = on ? p->K[j] : 0;
        g->Mr[j] = on ? p->Mr[j] : 1; g->tile[j] = on ? p->ts[j] : 1;
        g->delta[j] = on ? p->delta[j] : 0; g->period[j] = on ? p->T[j] : 0;
    }
    g->w = p->w;
    g->kparam = p->kparam;
    g->n_tiles = p->n_tiles;
    g->workspace_bytes = p->lay.total;
    return FKR_OK;
}

fkr_status fkr_workspace_size(const fkr_plan* p, size_t* bytes) {
    if (!p || !bytes) return FKR_E_ARG;
    *bytes = p->lay.total;
    return FKR_OK;
}

fkr_status fkr_set_workspace(fkr_plan* p, void* ws, size_t bytes) {
    if (!p || !ws) return FKR_E_ARG;
    if (bytes < p->lay.total || (reinterpret_cast<uintptr_t>(ws) & 255u)) return FKR_E_WORKSPACE;
    p->ws = static_cast<unsigned char*>(ws);
    p->ws_bytes = bytes;
    p->ws_ready = false;
    p->points_set = false;
    for (const auto& blob : constant_tables(p))
        FKR_HIP(hipMemcpy(p->ws + blob.first, blob.second.data(), blob.second.size(), hipMemcpyHostToDevice));
    FKR_HIP(hipMemset(p->ws + p->lay.diag, 0, 16 * 8));
    FKR_HIP(hipDeviceSynchronize());
    p->ws_ready = true;
    return FKR_OK;
}

fkr_status fkr_fit_noalloc(fkr_plan* p, int64_t N, const void* X, int x_type, int nh, const double* h, int q,
                           int y_complex, const void* Y, int y_type, double* mhat, double* s0, void* stream) {
    if (!p) return FKR_E_ARG;
    if (p->lay.total > kStaticScratchBytes) return FKR_E_WORKSPACE;   // the plan needs more than the array holds
    if (N < 0 || N > p->n_max || (N > 0 && !X) || !valid_type(x_type)) return FKR_E_ARG;
    if ((st_check_fit(p, nh, h, q, y_complex, Y, y_type, mhat)) != FKR_OK) return FKR_E_ARG;
    void* ws = nullptr;
    if (static_scratch(&ws) != hipSuccess) return FKR_E_DEVICE;
    const hipStream_t s = S(stream);
    // Bind the plan to the device's array.  Its contents are whatever the
    // last call on this device left: the plan's tables are uploaded again
    // (ordered on the stream, after any earlier call queued there) and the
    // counters are cleared.
    p->ws = static_cast<unsigned char*>(ws);
    p->ws_bytes = kStaticScratchBytes;
    p->points_set = false;
    if (p->const_blobs.empty()) p->const_blobs = constant_tables(p);
    for (const auto& blob : p->const_blobs)
        FKR_HIP(hipMemcpyAsync(p->ws + blob.first, blob.second.data(), blob.second.size(), hipMemcpyHostToDevice, s));
    launch_zero(p->ws + p->lay.diag, 16 * 8, s);
    if (hipGetLastError() != hipSuccess) return FKR_E_DEVICE;
    p->ws_ready = true;
    fkr_status st = fkr_set_points(p, N, X, x_type, stream);
    if (st != FKR_OK) return st;
    return fkr_fit(p, nh, h, q, y_complex, Y, y_type, mhat, s0, stream);
}

fkr_status fkr_set_points(fkr_plan* p, int64_t N, const void* X, int x_type, void* stream) {
    if (!p) return FKR_E_ARG;
    if (!p->ws_ready) return FKR_E_WORKSPACE;
    if (N < 0 || N > p->n_max || (N > 0 && !X) || !valid_type(x_type)) return FKR_E_ARG;
    const hipStream_t s = S(stream);
    const long long epoch = p->epoch + 1;
    const Geo g = make_geo(p);
    StageTimer t(p, FKR_STAGE_SORT, s);
    // the tile counts need clearing only where the binning adds to them with
    // global atomics (more tiles than the LDS histogram holds) or does not run
    if (p->n_tiles > kLdsHistMax || N == 0) launch_zero(p->ws + p->lay.counts, (p->n_tiles + 1) * 4, s);
    launch_bin_count(g, x_type, X, N, at<int32_t>(p, p->lay.counts), at<int32_t>(p, p->lay.bhist),
                     at<int32_t>(p, p->lay.obuf), s);
    launch_scan(g, N, epoch, at<int32_t>(p, p->lay.counts), at<int32_t>(p, p->lay.tile_off),
                at<int32_t>(p, p->lay.job_off), at<int32_t>(p, p->lay.jobs), at<int32_t>(p, p->lay.cursor),
                diag_ptr(p), at<int32_t>(p, p->lay.obuf), s);
    launch_sort_cells(g, p->prec, x_type, X, N, p->n_jobs_max, at<int32_t>(p, p->lay.tile_off),
                      at<int32_t>(p, p->lay.cursor), at<int32_t>(p, p->lay.jobs), at<int32_t>(p, p->lay.bhist),
                      p->ws + p->lay.trec, at<uint32_t>(p, p->lay.loc), p->ws + p->lay.frac,
                      at<int32_t>(p, p->lay.perm), p->ws + p->lay.xs, s);
    if (hipGetLastError() != hipSuccess) return FKR_E_DEVICE;
    p->N = N;
    p->epoch = epoch;
    p->points_set = true;
    p->last_stream = stream;
    return FKR_OK;
}

fkr_status fkr_spectrum(fkr_plan* p, int nw, const void* W, int w_type, double* out, void* stream) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if (nw < 1 || nw > p->max_weights || !out) return FKR_E_ARG;
    if (!W && nw != 1) return FKR_E_ARG;
    if (W && !valid_type(w_type)) return FKR_E_ARG;
    std::vector<WSrc> srcs;
    for (int r = 0; r < nw; ++r) srcs.push_back(W ? src_array(W, w_type, nw, r) : src_one());
    const hipStream_t s = S(stream);
    if ((st = run_spectra(p, srcs, s, false)) != FKR_OK) return st;
    launch_unpack_spec(p->tprec, p->Btot, p->B, p->d, (nw + 1) / 2, nw, p->ws + p->lay.spec, out, s);
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_moments(fkr_plan* p, int nh, const double* h, int nw, const void* W, int w_type,
                       double* Sout, double* Tout, void* stream) {
    fkr_status st = common_fit_checks(p, nh, h, nw, 0, W, w_type);
    if (st != FKR_OK) return st;
    if (1 + nw > p->max_weights) return FKR_E_ARG;
    const hipStream_t s = S(stream);
    std::vector<WSrc> srcs{src_one()};
    for (int r = 0; r < nw; ++r) srcs.push_back(src_array(W, w_type, nw, r));
    if ((st = run_spectra(p, srcs, s, false)) != FKR_OK) return st;
    const int nr = 1 + nw;
    const int ncp = (p->n_s + p->n_t * nw + 1) / 2;
    for (int hi = 0; hi < nh; ++hi) {
        if ((st = run_channels(p, h + hi * p->d, nr, nullptr, s)) != FKR_OK) return st;
        launch_chan_out(p->tprec, p->Mtot, ncp, p->n_s, p->n_t, nw, p->ws + p->lay.chan,
                        Sout ? Sout + (int64_t)hi * p->n_s * p->Mtot : nullptr,
                        Tout ? Tout + (int64_t)hi * nw * p->n_t * p->Mtot : nullptr, s);
    }
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_fit(fkr_plan* p, int nh, const double* h, int q, int y_complex, const void* Y, int y_type,
                   double* mhat, double* s0, void* stream) {
    fkr_status st = common_fit_checks(p, nh, h, q, y_complex, Y, y_type);
    if (st != FKR_OK) return st;
    if (q < 1 || !mhat) return FKR_E_ARG;
    const int ny = q * (y_complex ? 2 : 1);
    if (1 + ny > p->max_weights) return FKR_E_ARG;
    const hipStream_t s = S(stream);
    std::vector<WSrc> srcs{src_one()};
    add_response_sources(&srcs, q, y_complex, Y, y_type);
    if ((st = run_spectra(p, srcs, s, false)) != FKR_OK) return st;
    const int nr = (int)srcs.size();
    for (int hi = 0; hi < nh; ++hi) {
        if ((st = run_channels(p, h + hi * p->d, nr, hi == 0 ? ill_ctr(p) : nullptr, s)) != FKR_OK) return st;
        SolveArgs a = solve_args(p, nr, ny, y_complex, h + hi * p->d);
        a.y_out = mhat + (int64_t)hi * ny * p->Mtot;
        a.s0_out = s0 ? s0 + (int64_t)hi * p->Mtot : nullptr;
        {
            StageTimer t(p, FKR_STAGE_SOLVE, s);
            launch_solve2(p->tprec, a, dev_pidx(p), p->ws + p->lay.chan, s);
        }
    }
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_fit_full(fkr_plan* p, int nh, const double* H, int q, int y_complex, const void* Y, int y_type,
                        double* mhat, double* s0, void* stream) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if (nh < 1 || nh > p->max_h || !H || q < 1 || !mhat || (p->N > 0 && !Y) || (y_complex != 0 && y_complex != 1) ||
        !valid_type(y_type))
        return FKR_E_ARG;
    const int ny = q * (y_complex ? 2 : 1);
    if (1 + ny > p->max_weights) return FKR_E_ARG;
    if (p->reg_kernel) return FKR_E_UNSUPPORTED;
    const int dd = p->d * p->d;
    std::vector<FullH> fh(nh);
    std::vector<double> heff(3 * nh, 0.0);
    for (int hi = 0; hi < nh; ++hi)
        if ((st = build_full(p, H + hi * dd, &fh[hi], &heff[3 * hi])) != FKR_OK) return st;
    const hipStream_t s = S(stream);
    std::vector<WSrc> srcs{src_one()};
    add_response_sources(&srcs, q, y_complex, Y, y_type);
    if ((st = run_spectra(p, srcs, s, false)) != FKR_OK) return st;
    const int nr = (int)srcs.size();
    for (int hi = 0; hi < nh; ++hi) {
        if ((st = run_channels(p, fh[hi].s, nr, hi == 0 ? ill_ctr(p) : nullptr, s, false, 0, -1, 0, &fh[hi])) !=
            FKR_OK)
            return st;
        SolveArgs a = solve_args(p, nr, ny, y_complex, &heff[3 * hi]);
        a.y_out = mhat + (int64_t)hi * ny * p->Mtot;
        a.s0_out = s0 ? s0 + (int64_t)hi * p->Mtot : nullptr;
        StageTimer t(p, FKR_STAGE_SOLVE, s);
        launch_solve2(p->tprec, a, dev_pidx(p), p->ws + p->lay.chan, s);
    }
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_cv_full(fkr_plan* p, int nh, const double* H, int q, int y_complex, const void* Y, int y_type, int Np,
                       uint64_t seed, const void* probes, double* mhat, double* rho, double* rss, double* gcv,
                       double* nused, void* stream) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if (nh < 1 || nh > p->max_h || !H) return FKR_E_ARG;
    if (q < 0 || (q > 0 && !Y && p->N > 0) || (y_complex != 0 && y_complex != 1)) return FKR_E_ARG;
    if (q > 0 && !valid_type(y_type)) return FKR_E_ARG;
    if (Np < 0 || (q == 0 && Np == 0)) return FKR_E_ARG;
    if (gcv && (Np < 1 || q < 1)) return FKR_E_ARG;
    const int ny = q * (y_complex ? 2 : 1);
    if (1 + ny + Np > p->max_weights) return FKR_E_ARG;
    if (probes && !valid_type(y_type)) return FKR_E_ARG;
    if (p->reg_kernel) return FKR_E_UNSUPPORTED;
    const int dd = p->d * p->d;
    std::vector<FullH> fh(nh);
    std::vector<double> heff(3 * nh, 0.0);
    for (int hi = 0; hi < nh; ++hi)
        if ((st = build_full(p, H + hi * dd, &fh[hi], &heff[3 * hi])) != FKR_OK) return st;
    st = cv_impl(p, nh, nullptr, q, y_complex, Y, y_type, Np, seed, probes, nullptr, mhat, rho, rss, gcv, nused,
                 S(stream), fh.data(), heff.data());
    p->last_stream = stream;
    return st;
}

fkr_status fkr_moments_full(fkr_plan* p, int nh, const double* H, int nw, const void* W, int w_type, double* Sout,
                            double* Tout, void* stream) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if (nh < 1 || nh > p->max_h || !H || nw < 0 || (nw > 0 && p->N > 0 && !W) || 1 + nw > p->max_weights) return FKR_E_ARG;
    if (nw > 0 && !valid_type(w_type)) return FKR_E_ARG;
    if (p->reg_kernel) return FKR_E_UNSUPPORTED;
    const int dd = p->d * p->d;
    std::vector<FullH> fh(nh);
    std::vector<double> heff(3 * nh, 0.0);
    for (int hi = 0; hi < nh; ++hi)
        if ((st = build_full(p, H + hi * dd, &fh[hi], &heff[3 * hi])) != FKR_OK) return st;
    const hipStream_t s = S(stream);
    std::vector<WSrc> srcs{src_one()};
    for (int r = 0; r < nw; ++r) srcs.push_back(src_array(W, w_type, nw, r));
    if ((st = run_spectra(p, srcs, s, false)) != FKR_OK) return st;
    const int nr = 1 + nw;
    const int ncp = (p->n_s + p->n_t * nw + 1) / 2;
    for (int hi = 0; hi < nh; ++hi) {
        if ((st = run_channels(p, fh[hi].s, nr, nullptr, s, false, 0, -1, 0, &fh[hi])) != FKR_OK) return st;
        launch_chan_out(p->tprec, p->Mtot, ncp, p->n_s, p->n_t, nw, p->ws + p->lay.chan,
                        Sout ? Sout + (int64_t)hi * p->n_s * p->Mtot : nullptr,
                        Tout ? Tout + (int64_t)hi * nw * p->n_t * p->Mtot : nullptr, s);
    }
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_interp(fkr_plan* p, int nv, const double* G, int64_t Nq, const void* Xq, int x_type,
                      double* out, void* stream) {
    if (!p) return FKR_E_ARG;
    if (nv < 1 || !G || Nq < 0 || (Nq > 0 && (!Xq || !out)) || !valid_type(x_type)) return FKR_E_ARG;
    launch_interp(make_geo(p), nv, G, Nq, Xq, x_type, out, S(stream));
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_cv(fkr_plan* p, int nh, const double* h, int q, int y_complex, const void* Y, int y_type,
                  int Np, uint64_t seed, const void* probes, double* mhat, double* rho, double* rss,
                  double* gcv, double* nused, void* stream) {
    fkr_status st = common_fit_checks(p, nh, h, q, y_complex, Y, y_type);
    if (st != FKR_OK) return st;
    if (Np < 0 || (q == 0 && Np == 0)) return FKR_E_ARG;
    if (gcv && (Np < 1 || q < 1)) return FKR_E_ARG;
    const int ny = q * (y_complex ? 2 : 1);
    if (1 + ny + Np > p->max_weights) return FKR_E_ARG;
    if (probes && !valid_type(y_type)) return FKR_E_ARG;
    st = cv_impl(p, nh, h, q, y_complex, Y, y_type, Np, seed, probes, nullptr, mhat, rho, rss, gcv, nused,
                 S(stream));
    p->last_stream = stream;
    return st;
}

fkr_status fkr_gcv(fkr_plan* p, int nh, const double* h, int q, int y_complex, const void* Y, int y_type,
                   int Np, const double* rho_dev, double* mhat, double* rss, double* gcv, double* nused,
                   void* stream) {
    fkr_status st = common_fit_checks(p, nh, h, q, y_complex, Y, y_type);
    if (st != FKR_OK) return st;
    if (q < 1 || Np < 1 || !rho_dev || !gcv) return FKR_E_ARG;
    const int ny = q * (y_complex ? 2 : 1);
    if (1 + ny > p->max_weights) return FKR_E_ARG;
    st = cv_impl(p, nh, h, q, y_complex, Y, y_type, Np, 0, nullptr, rho_dev, mhat, nullptr, rss, gcv, nused,
                 S(stream));
    p->last_stream = stream;
    return st;
}

fkr_status fkr_dof(fkr_plan* p, int nh, const double* h, int Np, uint64_t seed, const void* probes,
                   int w_type, double* rho, double* nused, void* stream) {
    if (!p) return FKR_E_ARG;
    if (Np < 1 || !rho) return FKR_E_ARG;
    if (probes && !valid_type(w_type)) return FKR_E_ARG;
    // q = 0: only the density and the probes are spread.
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if ((st = check_h(p, nh, h)) != FKR_OK) return st;
    return fkr_cv(p, nh, h, 0, 0, probes, w_type, Np, seed, probes, nullptr, rho, nullptr, nullptr, nused, stream);
}

// The second pass at a diagonal bandwidth h, or (H non-null) at the full
// bandwidth matrix H.
fkr_status variance_impl(fkr_plan* p, const double* h, const double* H, int y_complex, const void* Y, int y_type,
                         const double* mhat, int mode, double* sigma2, double* vhat, double* kappa, void* stream) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if (!H && (st = check_h(p, 1, h)) != FKR_OK) return st;
    if ((!Y && p->N > 0) || (y_complex != 0 && y_complex != 1) || !valid_type(y_type)) return FKR_E_ARG;
    if (!mhat || !sigma2 || (mode != FKR_VAR_LOG && mode != FKR_VAR_DIRECT)) return FKR_E_ARG;
    if (p->max_weights < 2) return FKR_E_ARG;
    FullH fh{};
    double heff[3] = {0.0, 0.0, 0.0};
    if (H) {
        if (p->reg_kernel) return FKR_E_UNSUPPORTED;
        if ((st = build_full(p, H, &fh, heff)) != FKR_OK) return st;
    }
    const hipStream_t s = S(stream);
    const Geo g = make_geo(p);
    double* wbuf = at<double>(p, p->lay.wbuf);
    {
        // residuals, and the staged rows (1, z) of the second fit, in sorted order
        StageTimer t(p, FKR_STAGE_REDUCE, s);
        launch_resid(g, p->prec, mode, points_check(p), p->prec, p->ws + p->lay.xs, at<int32_t>(p, p->lay.perm),
                     y_type, Y, y_complex, mhat, wbuf + p->N, p->ws + p->lay.wsort, s);
    }
    std::vector<WSrc> srcs(2);
    for (int r = 0; r < 2; ++r) {
        srcs[r].kind = W_SORTED; srcs[r].type = p->prec; srcs[r].ptr = p->ws + p->lay.wsort;
        srcs[r].stride = resid_row_stride(g, p->prec); srcs[r].col = r;
    }
    // The density moments s_alpha depend on the points and h only: when the
    // channel buffer still holds them for these points at this h and the
    // residual pass left no sample out, the passes skip their pairs (decided
    // on the device), and the spread skips the density column.
    // (a full H: its channels carry no density tag, so nothing is kept)
    const bool keep = !H && p->n_s % 2 == 0;
    if (keep) launch_chan_reuse(diag_ptr(p), h, p->d, s);
    if ((st = run_spectra(p, srcs, s, true, keep ? diag_ptr(p) + kDiagReuse : nullptr)) != FKR_OK) return st;
    st = H ? run_channels(p, fh.s, 2, ill_ctr(p), s, false, 0, -1, 0, &fh) : run_channels(p, h, 2, ill_ctr(p), s, true);
    if (st != FKR_OK) return st;
    SolveArgs a = solve_args(p, 2, 1, 0, H ? heff : h);
    double* v = mode == FKR_VAR_DIRECT ? sigma2 : (vhat ? vhat : at<double>(p, p->lay.mhat));
    a.y_out = v;
    {
        StageTimer t(p, FKR_STAGE_SOLVE, s);
        launch_solve2(p->tprec, a, dev_pidx(p), p->ws + p->lay.chan, s);
    }
    if (mode == FKR_VAR_LOG) {
        StageTimer t(p, FKR_STAGE_REDUCE, s);
        double* partial = at<double>(p, p->lay.partial);
        launch_kappa_partial(g, p->N, p->prec, p->ws + p->lay.xs, at<int32_t>(p, p->lay.perm), v,
                             wbuf + p->N, partial, s);
        double* red = at<double>(p, p->lay.red);
        launch_reduce_final(partial, 2, red, s);
        launch_sigma2(p->Mtot, v, red, sigma2, kappa, s);
    }
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_variance(fkr_plan* p, const double* h, int y_complex, const void* Y, int y_type,
                        const double* mhat, int mode, double* sigma2, double* vhat, double* kappa,
                        void* stream) {
    if (!h) return FKR_E_ARG;
    return variance_impl(p, h, nullptr, y_complex, Y, y_type, mhat, mode, sigma2, vhat, kappa, stream);
}

fkr_status fkr_variance_full(fkr_plan* p, const double* H, int y_complex, const void* Y, int y_type,
                             const double* mhat, int mode, double* sigma2, double* vhat, double* kappa,
                             void* stream) {
    if (!H) return FKR_E_ARG;
    return variance_impl(p, nullptr, H, y_complex, Y, y_type, mhat, mode, sigma2, vhat, kappa, stream);
}

// The variance of the fit at a diagonal bandwidth h, or (H non-null) at
// the full bandwidth matrix H.
fkr_status interval_impl(fkr_plan* p, const double* h, const double* H, int sig_kind, double sigma2,
                         const double* sigma2_dev, const double* mhat, double alpha, double* Sigma, double* lower,
                         double* upper, void* stream) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if (!H && (st = check_h(p, 1, h)) != FKR_OK) return st;
    if (!Sigma) return FKR_E_ARG;
    if (H && p->reg_kernel) return FKR_E_UNSUPPORTED;
    if (sig_kind == FKR_SIG_SCALAR) {
        if (!(sigma2 >= 0.0) || !std::isfinite(sigma2)) return FKR_E_ARG;
    } else if (sig_kind != FKR_SIG_GRID || !sigma2_dev) {
        return FKR_E_ARG;
    }
    if ((lower || upper) && (!mhat || !(alpha > 0.0 && alpha < 1.0))) return FKR_E_ARG;
    // the squared Gaussian kernel is a Gaussian of bandwidth h / sqrt 2; a
    // compact kernel's square is sampled at h like the kernel itself
    const bool compact = p->reg_kernel != 0;
    double h2[3] = {0.0, 0.0, 0.0};
    // full H: the squared kernel is K_{H/2} (4 pi)^{-d/2} |H|^{-1/2}
    FullH fh{}, fh2{};
    double heff[3] = {0.0, 0.0, 0.0}, heff2[3] = {0.0, 0.0, 0.0};
    if (H) {
        const int dd = p->d * p->d;
        std::vector<double> Hh(dd);
        for (int k = 0; k < dd; ++k) Hh[k] = 0.5 * H[k];
        if ((st = build_full(p, H, &fh, heff)) != FKR_OK) return st;
        if (build_full(p, Hh.data(), &fh2, heff2) != FKR_OK) return FKR_E_ARG;
    } else {
        for (int j = 0; j < p->d; ++j) h2[j] = compact ? h[j] : h[j] / std::sqrt(2.0);
        if (check_h(p, 1, h2) != FKR_OK) return FKR_E_ARG;
    }
    const hipStream_t s = S(stream);
    const Geo g = make_geo(p);
    // 1. density moments at h -> row 0 of the equilibrated inverse per point
    std::vector<WSrc> dens{src_one()};
    if ((st = run_spectra(p, dens, s, false)) != FKR_OK) return st;
    st = H ? run_channels(p, fh.s, 1, ill_ctr(p), s, false, 0, -1, 0, &fh) : run_channels(p, h, 1, ill_ctr(p), s);
    if (st != FKR_OK) return st;
    SolveArgs a = solve_args(p, 1, 0, 0, H ? heff : h);
    a.r0_out = at<double>(p, p->lay.r0);
    {
        StageTimer t(p, FKR_STAGE_SOLVE, s);
        launch_solve2(p->tprec, a, dev_pidx(p), p->ws + p->lay.chan, s);
    }
    // 2. moments of the weights sigma_i^2 under the squared kernel (the
    // Gaussian at h / sqrt 2, K_h^2 = K_{h/sqrt2} prod_j 1 / (2 sqrt(pi) h_j);
    // a compact kernel: prod_j (K(u_j / h_j)^2 / h_j) prod_j 1 / h_j): the
    // same density spectra for a constant sigma^2, else the interpolated grid
    // staged as the weights of a spread
    IntervalArgs iv{};
    double scale = 1.0;
    if (H) {
        scale = std::pow(4.0 * M_PI, -0.5 * p->d);
        for (int j = 0; j < p->d; ++j) scale /= heff[j];   // prod_j heff_j = |H|^{1/2}
    } else
        for (int j = 0; j < p->d; ++j) scale *= compact ? 1.0 / h[j] : 1.0 / (2.0 * std::sqrt(M_PI) * h[j]);
    // the squared kernel's channels: at h / sqrt 2 (tagged as the density
    // moments there), at H / 2, or a compact kernel's square at h (neither
    // is a diagonal-bandwidth density moment: untagged)
    auto q_channels = [&]() {
        if (H) return run_channels(p, fh2.s, 1, nullptr, s, false, 0, -1, 0, &fh2);
        return run_channels(p, h2, 1, nullptr, s, false, compact || sig_kind != FKR_SIG_SCALAR ? 0 : 1, -1, 0,
                            nullptr, compact);
    };
    if (sig_kind == FKR_SIG_SCALAR) {
        if ((st = q_channels()) != FKR_OK) return st;
        scale *= sigma2;
    } else {
        {
            StageTimer t(p, FKR_STAGE_WEIGHTS, s);
            launch_stage_grid(g, p->prec, points_check(p), p->ws + p->lay.xs, sigma2_dev, p->ws + p->lay.wsort, s);
        }
        std::vector<WSrc> srcs(2);
        for (int r = 0; r < 2; ++r) {
            srcs[r].kind = W_SORTED; srcs[r].type = p->prec; srcs[r].ptr = p->ws + p->lay.wsort;
            srcs[r].stride = resid_row_stride(g, p->prec); srcs[r].col = r;
        }
        if ((st = run_spectra(p, srcs, s, true)) != FKR_OK) return st;
        if ((st = q_channels()) != FKR_OK) return st;
    }
    // 3. Sigma = scale r0^T Q r0, with Q re-equilibrated from h / sqrt 2 to h
    iv.P = p->n_t;
    iv.Mtot = p->Mtot;
    iv.r0 = at<double>(p, p->lay.r0);
    for (int b = 0; b < p->n_t; ++b)
        for (int c = 0; c < p->n_t; ++c) {
            int deg = 0;
            for (int j = 0; j < p->d; ++j) deg += p->et[b][j] + p->et[c][j];
            iv.sidx[b * kMaxP + c] = p->pair_index[b][c];
            iv.fac[b * kMaxP + c] = compact ? 1.0 : std::pow(2.0, -0.5 * deg);   // s / sqrt 2 -> s
        }
    iv.scale = scale;
    iv.mhat = mhat;
    iv.z = (lower || upper) ? upper_quantile(alpha) : 0.0;
    iv.sigma = Sigma;
    iv.lower = lower;
    iv.upper = upper;
    {
        StageTimer t(p, FKR_STAGE_SOLVE, s);
        launch_interval(p->tprec, iv, p->ws + p->lay.chan, s);
    }
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_interval(fkr_plan* p, const double* h, int sig_kind, double sigma2, const double* sigma2_dev,
                        const double* mhat, double alpha, double* Sigma, double* lower, double* upper,
                        void* stream) {
    if (!h) return FKR_E_ARG;
    return interval_impl(p, h, nullptr, sig_kind, sigma2, sigma2_dev, mhat, alpha, Sigma, lower, upper, stream);
}

fkr_status fkr_interval_full(fkr_plan* p, const double* H, int sig_kind, double sigma2, const double* sigma2_dev,
                             const double* mhat, double alpha, double* Sigma, double* lower, double* upper,
                             void* stream) {
    if (!H) return FKR_E_ARG;
    return interval_impl(p, nullptr, H, sig_kind, sigma2, sigma2_dev, mhat, alpha, Sigma, lower, upper, stream);
}

// Gradient of GCV in y after the base pass at h (channels at h in the first
// pairs, support flags, the fit of y, the sums): c = A^{-1} e_0, u = P^T r,
// the type-2 path of v_b = u c_b to the fine grid, the gather at the samples.
// u uses `scratch` ([M] doubles).
fkr_status grad_y(fkr_plan* p, const double* h, const FullH* fh, int Np, int nr, int ny, double* scratch,
                  double* dy, hipStream_t s) {
    const Geo g = make_geo(p);
    const int P = p->n_t;
    // a complex response runs as one complex function per b (real part:
    // the real residuals, imaginary part: the imaginary ones); a real one
    // packs two b per complex array
    const int cplx = ny == 2 ? 1 : 0;
    const int npv = cplx ? P : (P + 1) / 2;
    SolveArgs a = solve_args(p, 1, 0, 0, h);
    a.r0_out = at<double>(p, p->lay.r0);
    a.ill_count = nullptr;   // counted by the base solve
    launch_solve2(p->tprec, a, dev_pidx(p), p->ws + p->lay.chan, s);
    const int64_t wgstride = grouped_weights(p) ? 4 * p->N : 0;
    const int wstride = wgstride ? 4 : (nr + 3) & ~3;
    const double* yfit = at<double>(p, p->lay.mhat);
    const float* sup = at<float>(p, p->lay.sup);
    // u for every part of the response in one pass
    launch_fill_f64(scratch, (int64_t)ny * p->Mtot, 0.0, s);
    launch_adj_scatter(g, p->N, p->prec, p->ws + p->lay.xs, p->ws + p->lay.wsort, wstride, wgstride, ny, yfit, sup,
                       scratch, s);
    {
    void* bufs[2] = {p->ws + p->lay.fftA, p->ws + p->lay.fftB};
    int cur = 0;
    launch_adj_pack(p->tprec, P, p->Mtot, scratch, at<double>(p, p->lay.r0), cplx, bufs[cur], s);
    // grid (zero-padded to the period L) -> band, each pass moving its axis
    // to the end as the forward passes of the spread do: [band index][pair]
    int64_t done_B = 1;
    for (int j = 0; j < p->d; ++j) {
        FftPass f{};
        int64_t rest = 1;
        for (int i = j + 1; i < p->d; ++i) rest *= p->M[i];
        f.rows = done_B * npv * rest;
        f.n_in = p->M[j];
        f.F = p->L[j];
        f.n_out = p->B[j];
        f.K = p->K[j];
        f.in_band = 0;
        f.out_band = 1;
        f.nfac = p->fL[j].nfac;
        for (int q = 0; q < p->fL[j].nfac; ++q) f.fac[q] = p->fL[j].fac[q];
        f.tw = at<double>(p, p->fL[j].tw_off);
        if (j == p->d - 1) {
            f.out_estride = done_B * npv;
            f.out_rdiv = npv;
            f.out_rmul = npv;
        } else {
            f.out_estride = f.rows;
            f.out_rdiv = f.rows;
            f.out_rmul = 0;
        }
        launch_fft(p->tprec, false, f, bufs[cur], bufs[1 - cur], s);
        cur = 1 - cur;
        done_B *= p->B[j];
    }
    ExpandArgs ea{};
    ea.d = p->d;
    for (int j = 0; j < 3; ++j) { ea.B[j] = p->B[j]; ea.K[j] = p->K[j]; }
    for (int j = 0; j < p->d; ++j) { ea.h[j] = h[j]; ea.T[j] = p->T[j]; }
    ea.Btot = p->Btot;
    ea.n_s = p->n_s;
    ea.n_t = p->n_t;
    ea.deriv_dim = -1;
    if (p->reg_kernel) {   // the base pass left the kernel's tables at h
        ea.kdeg = 2 * p->order + 1;
        ea.ktab = at<double>(p, p->lay.ktab);
    }
    if (fh)
        launch_adj_combine_full(p->tprec, ea, *fh, P, cplx, dev_es(p), dev_pidx(p), at<double>(p, p->lay.deconv),
                                bufs[cur], bufs[1 - cur], s);
    else
        launch_adj_combine(p->tprec, ea, P, cplx, dev_et(p), at<double>(p, p->lay.deconv), bufs[cur], bufs[1 - cur],
                           s);
    cur = 1 - cur;
    // band -> fine grid along dimensions d-1 .. 0 (the inverse passes of the
    // channels with the fine grid's length and no crop)
    for (int j = p->d - 1; j >= 0; --j) {
        FftPass f{};
        int64_t R = 1;
        for (int i = 0; i < j; ++i) R *= p->B[i];
        for (int i = j + 1; i < p->d; ++i) R *= p->Mr[i];
        f.rows = R;
        f.n_in = p->B[j];
        f.F = p->Mr[j];
        f.n_out = p->Mr[j];
        f.K = p->K[j];
        f.in_band = 1;
        f.out_band = 0;
        f.nfac = p->fMr[j].nfac;
        for (int q = 0; q < p->fMr[j].nfac; ++q) f.fac[q] = p->fMr[j].fac[q];
        f.tw = at<double>(p, p->fMr[j].tw_off);
        f.in_rdiv = R;
        f.in_rmul = p->B[j] * R;
        f.in_estride = R;
        f.out_estride = 1;
        f.out_rdiv = 1;
        f.out_rmul = p->Mr[j];
        launch_fft(p->tprec, true, f, bufs[cur], bufs[1 - cur], s);
        cur = 1 - cur;
    }
    launch_adj_gather(g, p->prec, p->tprec, p->kernel, Np, p->n_jobs_max, at<int32_t>(p, p->lay.jobs),
                      at<uint32_t>(p, p->lay.loc), p->ws + p->lay.frac, p->ws + p->lay.xs, at<int32_t>(p, p->lay.perm),
                      bufs[cur], ny, cplx ? -1 : 0, yfit, sup, p->ws + p->lay.wsort, wstride, wgstride,
                      at<double>(p, p->lay.red), dy, s);
    }
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

// GCV and its gradient: in log h_j at a diagonal bandwidth h (nd = d
// directions), or (H non-null) in the upper-triangle entries H_pq, p <= q,
// row-major, of a full bandwidth matrix (nd = d (d + 1) / 2; an
// off-diagonal entry moves H_pq and H_qp together).
fkr_status grad_impl(fkr_plan* p, const double* h, const double* H, int y_complex, const void* Y, int y_type,
                     int Np, uint64_t seed, double* gcv, double* dtheta, double* dy, double* dfit, void* stream) {
    fkr_status st = ready(p);
    if (st != FKR_OK) return st;
    if (!H && (st = check_h(p, 1, h)) != FKR_OK) return st;
    if ((!Y && p->N > 0) || (y_complex != 0 && y_complex != 1) || !valid_type(y_type)) return FKR_E_ARG;
    if (Np < 1 || !dtheta || !dfit) return FKR_E_ARG;
    if (H && p->reg_kernel) return FKR_E_UNSUPPORTED;   // full H: the Gaussian only
    FullH fh{};
    double heff[3] = {0.0, 0.0, 0.0};
    if (H && (st = build_full(p, H, &fh, heff)) != FKR_OK) return st;
    const int nd = H ? p->d * (p->d + 1) / 2 : p->d;
    const int ny = y_complex ? 2 : 1;
    if (ny + Np > kGradCols) return FKR_E_ARG;
    const int nr = 1 + ny + Np;
    const int ncp = (p->n_s + p->n_t * (nr - 1) + 1) / 2;
    const int n_items = 1 + Np;          // base sums: the response (|r|^2), then the probes
    const int ncol = ny + Np;            // gradient sums per direction
    const int nslot = nd * ncol;
    // the channels at h and their derivatives side by side; the gradient sums
    // after the base sums
    if (nr > p->max_weights || 2 * ncp > p->ncp_max) return FKR_E_ARG;
    if ((int64_t)nslot * kRedBlocks > p->lay.cap_partial) return FKR_E_ARG;
    if (2 * n_items + 1 + nslot > (int64_t)p->max_h * (2 * p->max_weights + 4)) return FKR_E_ARG;
    const hipStream_t s = S(stream);
    // base pass: fit, DF and GCV at h (spectra, channels in pairs [0, ncp),
    // support flags, the fit of y, the sums)
    if ((st = cv_impl(p, 1, h, 1, y_complex, Y, y_type, Np, seed, nullptr, nullptr, nullptr, nullptr, nullptr,
                      nullptr, nullptr, s, H ? &fh : nullptr, H ? heff : nullptr)) != FKR_OK)
        return st;
    if (dy) {
        StageTimer t(p, FKR_STAGE_REDUCE, s);
        if ((st = grad_y(p, H ? heff : h, H ? &fh : nullptr, Np, nr, ny, dfit, dy, s)) != FKR_OK) return st;
    }
    const Geo g = make_geo(p);
    double* red = at<double>(p, p->lay.red);
    double* gred = red + 2 * n_items + 1;
    double* partial = at<double>(p, p->lay.partial);
    const float* sup = at<float>(p, p->lay.sup);
    const size_t pair_bytes = (size_t)p->Mtot * 2 * elem_size(p->tprec);
    for (int j = 0; j < nd; ++j) {
        if (H) {
            // direction j: the j-th upper-triangle entry (pq), symmetric
            int pp = 0, qq = 0, k = j;
            while (k >= p->d - pp) { k -= p->d - pp; ++pp; }
            qq = pp + k;
            FullH fd = fh;
            fd.deriv = 1;
            for (int e = 0; e < 9; ++e) fd.dH[e] = 0.0;
            fd.dH[3 * pp + qq] = 1.0;
            fd.dH[3 * qq + pp] = 1.0;
            st = run_channels(p, fh.s, nr, nullptr, s, false, 2, -1, ncp, &fd);
        } else {
            st = run_channels(p, h, nr, nullptr, s, false, 2, j, ncp);
        }
        if (st != FKR_OK) return st;
        DSolveArgs a{};
        a.P = p->n_t; a.n_s = p->n_s; a.n_t = p->n_t; a.ncp = ncp; a.nr = nr;
        a.Mtot = p->Mtot;
        a.sup = sup;
        a.out = dfit + (int64_t)j * (nr - 1) * p->Mtot;
        {
            StageTimer t(p, FKR_STAGE_SOLVE, s);
            launch_dsolve(p->tprec, a, dev_pidx(p), p->ws + p->lay.chan, p->ws + p->lay.chan + ncp * pair_bytes, s);
        }
    }
    {
        // the sums of every dimension's columns in one pass over the samples
        StageTimer t(p, FKR_STAGE_REDUCE, s);
        for (int c0 = 0; c0 < nslot; c0 += 32) {
            GradSumArgs r{};
            r.N = p->N; r.x_type = p->prec; r.X = p->ws + p->lay.xs;
            r.wsorted = p->ws + p->lay.wsort; r.w_type = p->prec;
            r.wgstride = grouped_weights(p) ? 4 * p->N : 0;
            r.wstride = r.wgstride ? 4 : (nr + 3) & ~3;
            r.ny = ny;
            r.yfit = at<double>(p, p->lay.mhat);
            r.dfit = dfit;
            r.sup = sup;
            r.ncol = ncol;
            r.col0 = c0;
            r.nall = std::min(32, nslot - c0);
            r.partial = partial;
            launch_grad_sums(g, r, s);
        }
    }
    launch_reduce_final(partial, nslot, gred, s);
    launch_finalize_grad(nd, ny, Np, red, gred, gcv, dtheta, s);
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_gcv_grad(fkr_plan* p, const double* h, int y_complex, const void* Y, int y_type, int Np,
                        uint64_t seed, double* gcv, double* dlogh, double* dy, double* dfit, void* stream) {
    if (!h) return FKR_E_ARG;
    return grad_impl(p, h, nullptr, y_complex, Y, y_type, Np, seed, gcv, dlogh, dy, dfit, stream);
}

fkr_status fkr_gcv_grad_full(fkr_plan* p, const double* H, int y_complex, const void* Y, int y_type, int Np,
                             uint64_t seed, double* gcv, double* dH, double* dy, double* dfit, void* stream) {
    if (!H) return FKR_E_ARG;
    return grad_impl(p, nullptr, H, y_complex, Y, y_type, Np, seed, gcv, dH, dy, dfit, stream);
}

fkr_status fkr_spline(fkr_plan* p, int nv, const double* G, double* coef, void* stream) {
    if (!p) return FKR_E_ARG;
    if (nv < 1 || !G || !coef) return FKR_E_ARG;
    const size_t blk = (size_t)p->Mtot << p->d;
    const char* gb = reinterpret_cast<const char*>(G);
    const char* cb = reinterpret_cast<const char*>(coef);
    if (gb < cb + blk * nv * 8 && cb < gb + (size_t)p->Mtot * nv * 8) return FKR_E_ARG;   // overlap
    launch_spline(make_geo(p), nv, G, coef, S(stream));
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_predict(fkr_plan* p, int nv, const double* coef, int64_t Nq, const void* Xq, int x_type,
                       double* out, void* stream) {
    if (!p) return FKR_E_ARG;
    if (nv < 1 || !coef || Nq < 0 || (Nq > 0 && (!Xq || !out)) || !valid_type(x_type)) return FKR_E_ARG;
    launch_spline_eval(make_geo(p), nv, coef, Nq, Xq, x_type, out, S(stream));
    p->last_stream = stream;
    return hipGetLastError() == hipSuccess ? FKR_OK : FKR_E_DEVICE;
}

fkr_status fkr_hlist(int n, double a, double b, int kind, double* out) {
    if (n < 1 || !out || !std::isfinite(a) || !std::isfinite(b) || (kind != 0 && kind != 1)) return FKR_E_ARG;
    if (kind == 0 && !(a > 0.0 && b > 0.0)) return FKR_E_ARG;
    for (int k = 0; k < n; ++k) {
        const double t = n == 1 ? 1.0 : (double)k / (double)(n - 1);
        if (kind == 0) out[k] = std::pow(10.0, std::log10(a) + t * (std::log10(b) - std::log10(a)));
        else out[k] = a + t * (b - a);
    }
    out[0] = a;
    if (n > 1) out[n - 1] = b;
    return FKR_OK;
}

fkr_status fkr_select_bandwidth(int nh, const double* gcv, double dstd, int* index) {
    if (nh < 1 || !gcv || !index || !(dstd >= 0.0)) return FKR_E_ARG;
    double mn = INFINITY, sum = 0.0;
    int cnt = 0;
    for (int k = 0; k < nh; ++k)
        if (std::isfinite(gcv[k])) { mn = std::min(mn, gcv[k]); sum += gcv[k]; ++cnt; }
    if (cnt == 0) return FKR_E_ARG;
    double thr = mn;
    if (dstd > 0.0 && cnt > 1) {
        const double mean = sum / cnt;
        double ss = 0.0;
        for (int k = 0; k < nh; ++k)
            if (std::isfinite(gcv[k])) ss += (gcv[k] - mean) * (gcv[k] - mean);
        thr += dstd * std::sqrt(ss / (cnt - 1));
    }
    int best = -1;
    for (int k = 0; k < nh; ++k)
        if (std::isfinite(gcv[k]) && gcv[k] <= thr) best = k;
    *index = best;
    return FKR_OK;
}

fkr_status fkr_profile_enable(fkr_plan* p, int on) {
    if (!p || (on != 0 && on != 1)) return FKR_E_ARG;
    if (!on) {
        for (auto& v : p->ev_pairs) {
            for (auto& e : v) {
                (void)hipEventSynchronize(e.second);
                p->ev_free.push_back(e.first);
                p->ev_free.push_back(e.second);
            }
            v.clear();
        }
    }
    p->prof_on = on != 0;
    return FKR_OK;
}

fkr_status fkr_profile_read(fkr_plan* p, int stage, double* ms, int64_t* launches) {
    if (!p || stage < 0 || stage >= FKR_N_STAGES || !ms || !launches) return FKR_E_ARG;
    double total = 0.0;
    fkr_status st = FKR_OK;
    auto& v = p->ev_pairs[stage];
    for (auto& e : v) {
        float t = 0.0f;
        if (hipEventSynchronize(e.second) != hipSuccess ||
            hipEventElapsedTime(&t, e.first, e.second) != hipSuccess)
            st = FKR_E_DEVICE;
        total += (double)t;
        p->ev_free.push_back(e.first);
        p->ev_free.push_back(e.second);
    }
    *ms = total;
    *launches = (int64_t)v.size();
    v.clear();
    return st;
}

fkr_status fkr_get_diagnostics(fkr_plan* p, fkr_diag* out) {
    if (!p || !out) return FKR_E_ARG;
    std::memset(out, 0, sizeof(*out));
    if (!p->ws_ready) return FKR_E_WORKSPACE;
    FKR_HIP(hipStreamSynchronize(S(p->last_stream)));
    long long d[16];
    FKR_HIP(hipMemcpy(d, p->ws + p->lay.diag, sizeof(d), hipMemcpyDeviceToHost));
    out->n_points = p->N;
    out->out_of_domain = d[1];
    out->ill_posed = d[2];
    out->n_jobs = d[3];
    out->max_tile_count = d[4];
    if (d[5] != 0) return FKR_E_DEVICE;
    if (d[kDiagStale] != 0) return FKR_E_STATE;
    if (d[1] != 0) return FKR_E_DOMAIN;
    if (d[2] != 0) return FKR_WARN_ILLPOSED;
    return FKR_OK;
}

}  // extern "C"
