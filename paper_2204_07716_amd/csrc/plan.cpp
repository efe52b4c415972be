// Host planner: grid geometry, spectral band, spreading kernel, tiles and the
// workspace layout.  Pure host code (no HIP calls).
//
// Geometry per dimension j (Sec. 1.2 and Sec. 4 fkreg_create):
//   delta_j = (hi_j - lo_j) / (M_j - 1)                    grid spacing, eq. (6)
//   L_j     >= M_j - 1 + U_x h_max / delta_j, 2^a 3^b 5^c    zero padding, eq. (18):
//             the period T_j = L_j delta_j exceeds the data span plus the reach
//             of the widest kernel, so the circular convolution of eq. (19)-(21)
//             does not wrap at accuracy eps
//   K_j     = ceil(U_w / h_min * T_j / (2 pi))             retained modes |n| <= K_j:
//             beyond U_w / h the Gaussian moment spectra (Hermite form) fall
//             below eps, so higher modes never reach the output (when the
//             band is wider than L_j, modes are folded modulo L_j before the
//             inverse transform, which is exact on the grid points)
//   Mr_j    = smooth(sigma * (2 K_j + 1))                  fine spreading grid, the
//             oversampled grid of eq. (17) (sigma = 2 is M_r = 2 L of the paper
//             applied to the retained band)
// The spreading kernel is the exponential of semicircle (Barnett, Magland and
// af Klinteberg 2019) or the paper's Gaussian (Dutt-Rokhlin / Greengard-Lee,
// eq. 17 and 20); its width follows from eps.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fkr_internal.h"
#include "kernels.h"

namespace fkr {

size_t elem_size(int type) { return type == FKR_F64 ? 8 : 4; }

int64_t smooth_up(int64_t n) {
    if (n < 1) n = 1;
    for (;; ++n) {
        int64_t m = n;
        for (int p : {2, 3, 5})
            while (m % p == 0) m /= p;
        if (m == 1) return n;
    }
}

bool factorise(int64_t n, FftLen* out) {
    out->n = n;
    out->nfac = 0;
    int64_t m = n;
    while (m % 4 == 0 && out->nfac < kMaxFactors) { out->fac[out->nfac++] = 4; m /= 4; }
    for (int p : {2, 3, 5})
        while (m % p == 0 && out->nfac < kMaxFactors) { out->fac[out->nfac++] = p; m /= p; }
    return m == 1;
}

void twiddle_table(int64_t n, std::vector<double>* t) {
    // exp(-2 pi i k / n), k = 0..n-1, evaluated in long double from the
    // reduced angle so every entry is correctly rounded to FP64.
    t->resize(2 * (size_t)n);
    const long double two_pi = 6.283185307179586476925286766559L;
    for (int64_t k = 0; k < n; ++k) {
        long double a = -two_pi * (long double)k / (long double)n;
        (*t)[2 * k] = (double)cosl(a);
        (*t)[2 * k + 1] = (double)sinl(a);
    }
}

// Probabilists' Hermite polynomial He_a(u).
static double hermite_e(int a, double u) {
    if (a == 0) return 1.0;
    double hm = 1.0, h = u;
    for (int k = 1; k < a; ++k) {
        double hn = u * h - k * hm;
        hm = h;
        h = hn;
    }
    return h;
}

// Smallest u such that for every t >= u and every degree a <= maxdeg both
// t^a exp(-t^2/2) and |He_a(t)| exp(-t^2/2) are <= tol.
static double gaussian_tail(int maxdeg, double tol) {
    const double step = 1e-3;
    double u = 40.0;
    for (double t = 40.0; t >= 0.0; t -= step) {
        double e = std::exp(-0.5 * t * t);
        double worst = 0.0;
        for (int a = 0; a <= maxdeg; ++a) {
            worst = std::max(worst, std::pow(t, a) * e);
            worst = std::max(worst, std::fabs(hermite_e(a, t)) * e);
        }
        if (worst > tol) return u;
        u = t;
    }
    return 0.0;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
static void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w) {
    x->resize(n);
    w->resize(n);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        (*x)[i] = -z;
        (*x)[n - 1 - i] = z;
        (*w)[i] = (*w)[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// Fourier transform of the ES kernel psi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1))
// on |t| < w/2 (t in fine cells), at xi radians per cell, by Gauss-Legendre
// quadrature of 2 * int_0^{w/2} psi(t) cos(xi t) dt.
double es_kernel_hat(double xi, int w, double beta) {
    static thread_local std::vector<double> gx, gw;
    const int nq = 200 + 20 * w;
    if ((int)gx.size() != nq) gauss_legendre(nq, &gx, &gw);
    const double half = 0.5 * w;
    double acc = 0.0;
    for (int q = 0; q < nq; ++q) {
        double t = 0.5 * half * (gx[q] + 1.0);
        double s = t / half;
        double psi = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - s * s)) - 1.0));
        acc += gw[q] * 0.5 * half * psi * std::cos(xi * t);
    }
    return 2.0 * acc;
}

static int64_t binom(int n, int k) {
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// Exponent tuples of total degree <= deg; degree ascending, then the exponent
// of dimension 0 descending, then dimension 1, ...
static int enumerate(int d, int deg, int (*out)[kMaxD]) {
    int n = 0;
    for (int t = 0; t <= deg; ++t) {
        if (d == 1) {
            out[n][0] = t; out[n][1] = out[n][2] = 0; ++n;
        } else if (d == 2) {
            for (int a = t; a >= 0; --a) { out[n][0] = a; out[n][1] = t - a; out[n][2] = 0; ++n; }
        } else {
            for (int a = t; a >= 0; --a)
                for (int b = t - a; b >= 0; --b) { out[n][0] = a; out[n][1] = b; out[n][2] = t - a - b; ++n; }
        }
    }
    return n;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void layout(fkr_plan* p) {
    Layout& L = p->lay;
    const size_t sz = elem_size(p->prec), csz = 2 * sz;      // spreading side
    const size_t tcsz = 2 * elem_size(p->tprec);              // transform side
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + std::max<size_t>(bytes, 1)); return o; };
    size_t nB = 0, nTw = 0, nCov = 0;
    for (int j = 0; j < p->d; ++j) {
        nB += p->B[j];
        nCov += (size_t)p->Mr[j] * (1 + 2 * kCoverSlots);
    }
    L.consts = take(4096);
    L.deconv = take(nB * 8);
    for (int j = 0; j < p->d; ++j) {
        p->fMr[j].tw_off = take((size_t)p->fMr[j].n * 16);
        p->fL[j].tw_off = take((size_t)p->fL[j].n * 16);
        nTw += p->fMr[j].n + p->fL[j].n;
    }
    (void)nTw;
    L.cover = take(nCov * 4);
    L.diag = take(16 * 8);
    const int64_t N = std::max<int64_t>(p->n_max, 1);
    L.trec = take(N * tile_record_bytes(p->d, p->prec));
    // block x tile counts of the binning pass (when the tiles fit the LDS histogram)
    const int64_t nbins = (N + kSortChunk - 1) / kSortChunk;
    L.bhist = take(p->n_tiles <= kLdsHistMax ? (size_t)nbins * p->n_tiles * 4 : 4);
    L.obuf = take((size_t)nbins * 4);   // per-block counts of samples outside [lo, hi]
    L.counts = take((p->n_tiles + 1) * 4);
    L.tile_off = take((p->n_tiles + 1) * 4);
    L.cursor = take(p->n_tiles * 4);
    L.job_off = take((p->n_tiles + 1) * 4);
    L.cap_jobs = p->n_jobs_max;
    L.jobs = take((p->n_jobs_max * 4 + 4) * 4);
    L.loc = take(N * 4);
    L.frac = take(N * p->d * sz);
    L.perm = take(N * 4);
    L.xs = take(N * p->d * sz);
    L.subgrid = take((size_t)p->n_jobs_max * p->Psub * p->pairs_per_spread * csz);
    // FFT intermediates (complex elements)
    int64_t cap = 0;
    {
        int64_t g = p->pairs_per_spread;
        if (p->d == 3) cap = std::max(cap, g * p->Mr[0] * p->Mr[1] * p->Mr[2]);   // the folded fine grid
        // one complex fine grid and the band-to-fine-grid intermediates of the
        // gradient in y (the adjoint of the moment path)
        for (int j = 0; j < p->d; ++j) {
            int64_t e = 1;
            for (int i = 0; i < j; ++i) e *= p->B[i];
            for (int i = j; i < p->d; ++i) e *= p->Mr[i];
            cap = std::max(cap, e);
        }
        for (int j = 0; j < p->d; ++j) {
            int64_t e = g;
            for (int i = 0; i <= j; ++i) e *= p->B[i];
            for (int i = j + 1; i < p->d; ++i) e *= p->Mr[i];
            cap = std::max(cap, e);
        }
        int64_t c = p->ncp_max;
        cap = std::max(cap, c * p->Btot);
        // inverse transforms run dimensions d-1 .. 0: after the pass along
        // dimension j, [pair][B_{j-1} .. B_0][M_{d-1} .. M_j]
        for (int j = p->d - 1; j >= 0; --j) {
            int64_t e = c;
            for (int i = 0; i < j; ++i) e *= p->B[i];
            for (int i = j; i < p->d; ++i) e *= p->M[i];
            cap = std::max(cap, e);
        }
    }
    L.cap_fft = cap;
    L.fftA = take(cap * tcsz);
    L.fftB = take(cap * tcsz);
    L.cap_spec = p->Btot * p->npairs_max;
    L.spec = take(L.cap_spec * tcsz);
    L.cap_chan = p->Mtot * p->ncp_max;
    L.chan = take(L.cap_chan * tcsz);
    L.cap_mhat = p->Mtot * (int64_t)p->max_weights;
    L.mhat = take(L.cap_mhat * 8 + 64);   // + alignment and row padding of the FP32 probe fits
    L.cap_partial = kRedBlocks * (int64_t)(2 * p->max_weights + 2);
    L.partial = take(L.cap_partial * 8);
    L.cap_wbuf = 2 * N;
    L.wbuf = take(L.cap_wbuf * 8);
    L.wsort = take((size_t)N * ((p->max_weights + 3) & ~3) * sz + 256);   // slack: row loads may read 16 past the last row
    L.red = take((size_t)p->max_h * (2 * p->max_weights + 4) * 8);
    L.sup = take((size_t)p->Mtot * 4);
    L.r0 = take((size_t)p->Mtot * p->n_t * 8);
    int64_t nb = 0, nbmax = 0;
    for (int j = 0; j < p->d; ++j) { nb += p->B[j]; nbmax = std::max<int64_t>(nbmax, p->B[j]); }
    L.ktab = take((size_t)(2 * p->order + 1) * (nb + nbmax) * 8);   // + one derivative block
    L.total = off;
}

fkr_status build_plan(const fkr_plan_desc* desc, fkr_plan* p) {
    const fkr_plan_desc& D = *desc;
    if (D.d < 1 || D.d > kMaxD || D.order < 0 || D.order > FKR_MAX_ORDER) return FKR_E_ARG;
    if (!(D.eps > 0.0 && D.eps < 1.0)) return FKR_E_ARG;
    if (D.precision != FKR_F32 && D.precision != FKR_F64) return FKR_E_ARG;
    if (D.transform_precision != 0 && D.transform_precision != FKR_TP_F32 &&
        D.transform_precision != FKR_TP_F64) return FKR_E_ARG;
    if (D.spread_kernel != FKR_KERNEL_ES && D.spread_kernel != FKR_KERNEL_GAUSS) return FKR_E_ARG;
    if (D.reg_kernel < FKR_REG_GAUSS || D.reg_kernel > FKR_REG_TRIWEIGHT) return FKR_E_ARG;
    if (D.n_max < 0 || D.n_max > INT32_MAX - 1) return FKR_E_ARG;
    if (D.max_weights < 1 || D.max_weights > 1024) return FKR_E_ARG;
    if (D.max_h < 1 || D.max_h > FKR_MAX_H) return FKR_E_ARG;
    if (!(D.sigma == 0.0 || (D.sigma >= 1.25 && D.sigma <= 4.0))) return FKR_E_ARG;
    p->desc = D;
    p->d = D.d;
    p->order = D.order;
    p->prec = D.precision;
    p->tprec = D.transform_precision == FKR_TP_F64 ? FKR_F64
             : D.transform_precision == FKR_TP_F32 ? FKR_F32 : D.precision;
    p->kernel = D.spread_kernel;
    p->reg_kernel = D.reg_kernel;
    p->eps = D.eps;
    // Default oversampling: 4 in 1-D and 2-D (narrower kernel, sparser fine
    // cells; the fine grid stays small), 2 in 3-D.
    p->sigma = D.sigma == 0.0 ? (D.d <= 2 ? 4.0 : 2.0) : D.sigma;
    p->n_max = D.n_max;
    p->max_weights = D.max_weights;
    p->max_h = D.max_h;
    for (int j = 0; j < D.d; ++j) {
        if (D.M[j] < 2 || D.M[j] > (1 << 20)) return FKR_E_ARG;
        if (!std::isfinite(D.lo[j]) || !std::isfinite(D.hi[j]) || !(D.hi[j] > D.lo[j])) return FKR_E_ARG;
        if (!(D.h_min[j] > 0.0) || !(D.h_max[j] >= D.h_min[j]) || !std::isfinite(D.h_max[j])) return FKR_E_ARG;
    }

    // Channels (eq. 12-13): s for |a| <= 2l, t for |b| <= l.
    p->n_s = enumerate(p->d, 2 * p->order, p->es);
    p->n_t = enumerate(p->d, p->order, p->et);
    if (p->n_s != binom(p->d + 2 * p->order, 2 * p->order) || p->n_t != binom(p->d + p->order, p->order))
        return FKR_E_ARG;
    for (int b = 0; b < p->n_t; ++b)
        for (int c = 0; c < p->n_t; ++c) {
            int idx = -1;
            for (int s = 0; s < p->n_s; ++s) {
                bool eq = true;
                for (int j = 0; j < p->d; ++j) eq &= p->es[s][j] == p->et[b][j] + p->et[c][j];
                if (eq) { idx = s; break; }
            }
            p->pair_index[b][c] = idx;
        }

    // Tolerances: the tails of the moment kernels in space and in frequency
    // are cut at eps / 10; the spreading kernel is sized for eps / 10 too.
    const double tol = 0.1 * p->eps;
    p->U_space = gaussian_tail(2 * p->order, tol);
    p->U_spec = p->U_space;
    const double tol_k = std::max(tol, p->prec == FKR_F32 ? 1e-9 : 1e-16);

    if (p->kernel == FKR_KERNEL_ES) {
        // ES width for oversampling sigma (Barnett, Magland, af Klinteberg):
        // w = ceil(ln(1/tol) / (pi sqrt(1 - 1/sigma))), i.e. digits + 1 at sigma = 2.
        p->w = (int)std::ceil(-std::log(tol_k) / (M_PI * std::sqrt(1.0 - 1.0 / p->sigma)));
        p->w = std::min(std::max(p->w, 2), 16);
        p->kparam = 0.97 * M_PI * (1.0 - 0.5 / p->sigma) * p->w;
    } else {
        // Gaussian gridding: error ~ exp(-pi Msp (R-1)/(R-0.5)); w = 2 Msp.
        const double R = p->sigma;
        int msp = (int)std::ceil(-std::log(tol_k) * (R - 0.5) / (M_PI * (R - 1.0)));
        msp = std::min(std::max(msp, 2), 12);
        p->w = 2 * msp;
        p->kparam = M_PI * (R - 0.5) / (R * msp);   // psi(t) = exp(-a t^2), t in cells
    }
    {   // round up to a compiled width
        int wr = -1;
        for (int cand : kWidths)
            if (cand >= p->w) { wr = cand; break; }
        if (wr < 0) return FKR_E_UNSUPPORTED;
        p->w = wr;
    }

    p->Mtot = p->Btot = p->Mrtot = 1;
    for (int j = 0; j < p->d; ++j) {
        p->M[j] = D.M[j];
        p->lo[j] = D.lo[j];
        p->hi[j] = D.hi[j];
        p->h_min[j] = D.h_min[j];
        p->h_max[j] = D.h_max[j];
        p->delta[j] = (D.hi[j] - D.lo[j]) / (double)(D.M[j] - 1);
        // the zero padding holds the kernel's reach at h_max: the Gaussian's
        // tail down to the tolerance, a compact kernel's support
        const double reach = (p->reg_kernel ? 1.0 : p->U_space) * D.h_max[j] / p->delta[j] + (p->reg_kernel ? 1.0 : 0.0);
        if (reach > 4.0 * (1 << 20)) return FKR_E_ARG;
        p->L[j] = smooth_up((int64_t)std::ceil((double)(D.M[j] - 1) + reach) + 1);
        p->T[j] = (double)p->L[j] * p->delta[j];
        const double omega = p->U_spec / D.h_min[j];
        // a compact kernel keeps every mode of the period (eq. 12-13: the
        // discrete convolution with the sampled kernel); for even L the
        // modes +-L/2 share the Nyquist term, each with half its weight
        int64_t K = p->reg_kernel ? p->L[j] / 2 : (int64_t)std::ceil(omega * p->T[j] / (2.0 * M_PI));
        p->K[j] = K;
        p->B[j] = 2 * K + 1;
        int64_t mr = smooth_up((int64_t)std::ceil(p->sigma * (double)p->B[j]));
        mr = std::max<int64_t>(mr, smooth_up(p->w + 2));
        p->Mr[j] = mr;
        p->hf[j] = p->T[j] / (double)mr;
        p->inv_hf[j] = (double)mr / p->T[j];
        if (!factorise(p->Mr[j], &p->fMr[j]) || !factorise(p->L[j], &p->fL[j])) return FKR_E_UNSUPPORTED;
        // One FFT row and its ping-pong copy live in 64 KB of LDS.
        if ((int64_t)2 * std::max(p->Mr[j], p->L[j]) * 2 * (int64_t)elem_size(p->tprec) > 65536)
            return FKR_E_UNSUPPORTED;
        p->Mtot *= p->M[j];
        p->Btot *= p->B[j];
        p->Mrtot *= p->Mr[j];
    }

    // Deconvolution factors 1 / psi_hat(2 pi n / Mr) (eq. 20), n = -K..K.
    for (int j = 0; j < p->d; ++j) {
        p->deconv[j].resize(p->B[j]);
        for (int64_t n = -p->K[j]; n <= p->K[j]; ++n) {
            const double xi = 2.0 * M_PI * (double)n / (double)p->Mr[j];
            double ph;
            if (p->kernel == FKR_KERNEL_ES) ph = es_kernel_hat(xi, p->w, p->kparam);
            else ph = std::sqrt(M_PI / p->kparam) * std::exp(-xi * xi / (4.0 * p->kparam));
            p->deconv[j][n + p->K[j]] = 1.0 / ph;
        }
    }

    // Spreading tiles: a tile of TS fine cells per dimension (fewer when the
    // fine grid is shorter); the subgrid of a job has pitch PE = TS + w - 1.
    const int TS = spread_tile_edge(p->d, p->w);
    if (TS <= 0) return FKR_E_UNSUPPORTED;
    p->Psub = 1;
    for (int j = 0; j < p->d; ++j) {
        p->ts[j] = std::min<int64_t>(TS, p->Mr[j]);
        p->nt[j] = (p->Mr[j] + p->ts[j] - 1) / p->ts[j];
        p->pe[j] = TS + p->w - 1;
        p->Psub *= p->pe[j];
    }
    p->pairs_per_spread = kMaxPairsInLaunch;
    p->tsp = TS;
    p->ncell = 1;
    for (int j = 0; j < p->d; ++j) p->ncell *= TS;
    p->n_tiles = 1;
    for (int j = 0; j < p->d; ++j) p->n_tiles *= p->nt[j];

    // Cover lists: for every fine cell, the (tile, offset) pairs of the padded
    // tiles that contain it (periodic in Mr).
    for (int j = 0; j < p->d; ++j) {
        const int stride = 1 + 2 * kCoverSlots;
        p->cover[j].assign((size_t)p->Mr[j] * stride, 0);
        for (int64_t b = 0; b < p->nt[j]; ++b) {
            const int64_t interior = std::min<int64_t>(p->ts[j], p->Mr[j] - b * p->ts[j]);
            for (int64_t o = 0; o < interior + p->w - 1; ++o) {
                int64_t c = (b * p->ts[j] + o) % p->Mr[j];
                int32_t* e = &p->cover[j][(size_t)c * stride];
                if (e[0] >= kCoverSlots) return FKR_E_UNSUPPORTED;
                e[1 + 2 * e[0]] = (int32_t)b;
                e[2 + 2 * e[0]] = (int32_t)o;
                e[0]++;
                p->max_cover = std::max(p->max_cover, (int)e[0]);
            }
        }
    }

    // Spreading jobs: a tile's samples, cut into near-equal pieces of at most
    // one chunk so that dense tiles do not serialise on one workgroup.  Every
    // piece costs one subgrid of (TS + W - 1)^d cells that the fold reads
    // back, which weighs more in 3-D; there the pieces are large (the column
    // spread keeps a whole (x, y) run of first cells in registers).
    // (3-D: the largest job whose records, 32 bytes each in FP32, fit the
    // LDS the per-job cell sort stages them in; a dense 8^3-cell tile of
    // ~8000 samples is two jobs)
    p->chunk = p->d <= 2 ? 1024 : (p->prec == FKR_F32 ? 4800 : 2400);
    p->chunk_min = p->chunk;
    p->n_jobs_max = p->n_tiles + (p->n_max + p->chunk - 1) / p->chunk + 1;
    p->npairs_max = (p->max_weights + 1) / 2;
    const int nreal = p->n_s + p->n_t * (p->max_weights - 1);
    p->ncp_max = (nreal + 1) / 2;
    layout(p);
    return FKR_OK;
}

}  // namespace fkr
