/*
 * FP64 direct-sum oracle for fast kernel regression -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the HIP path.
 *
 * It evaluates, by the plain O(N * G) definition and with no FFT, no gridding,
 * no blocking and no fusion:
 *
 *   orc_moments: the kernel-weighted moment sums of Sec. 1.1, eq. (9), with
 *       the displacement written as z = x_i - g (the sign convention of
 *       eq. (2)-(4)) and the scaled Gaussian kernel of eq. (2) with a diagonal
 *       bandwidth matrix H = diag(h_j^2):
 *           K(z) = prod_j exp(-z_j^2 / (2 h_j^2)) / (h_j sqrt(2 pi)),
 *           s_a(g)   = sum_i K(x_i - g) (x_i - g)^a          (|a| <= 2l),
 *           t_w,b(g) = sum_i K(x_i - g) (x_i - g)^b W[i, w]  (|b| <= l).
 *       The monomial exponent lists are passed in, so the caller decides the
 *       ordering; sums are Neumaier-compensated.  With cutoff != 0, pairs with
 *       |z_j| > h_j * sqrt(2 ln 2^64) are skipped: there each kernel factor is
 *       below 2^-64 of its peak, beneath FP64 resolution of any sum that also
 *       holds the nearby samples.
 *
 *   orc_nudft: the type-1 non-uniform discrete Fourier transform that the
 *       gridding + FFT of Sec. 1.2 (eq. 16-21) approximates:
 *           c(n) = sum_i w_i exp(-i sum_j 2 pi n_j (x_ij - lo_j) / T_j),
 *       for the modes n_j = -K_j .. K_j (n_0 fastest in the output).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC fkr_oracle.c -o libfkr_oracle.so -lm
 */
#define _GNU_SOURCE
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXD 3
#define ORC_MAXDEG 8

typedef struct { double s, c; } nsum; /* Neumaier running sum */

static inline void nadd(nsum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

int orc_moments(int d, int64_t N, const double* X, int nw, const double* W,
                const double* h, int n_s, const int* exps_s, int n_t,
                const int* exps_t, int64_t G, const double* gpts, double* S,
                double* T, int cutoff)
{
    if (d < 1 || d > ORC_MAXD || N < 0 || G < 0 || nw < 0) return -1;
    int maxdeg = 0;
    for (int m = 0; m < n_s * d; ++m) if (exps_s[m] > maxdeg) maxdeg = exps_s[m];
    for (int m = 0; m < n_t * d; ++m) if (exps_t[m] > maxdeg) maxdeg = exps_t[m];
    if (maxdeg > ORC_MAXDEG) return -2;
    const double reach = sqrt(2.0 * 64.0 * log(2.0)); /* in units of h */
    double norm = 1.0;
    for (int j = 0; j < d; ++j) norm *= 1.0 / (h[j] * sqrt(2.0 * M_PI));

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < G; ++g) {
        nsum* acc_s = (nsum*)calloc((size_t)n_s, sizeof(nsum));
        nsum* acc_t = (nsum*)calloc((size_t)n_t * (size_t)(nw > 0 ? nw : 1), sizeof(nsum));
        double pw[ORC_MAXD][ORC_MAXDEG + 1];
        for (int64_t i = 0; i < N; ++i) {
            double e = 0.0;
            int skip = 0;
            for (int j = 0; j < d; ++j) {
                double z = X[i * d + j] - gpts[g * d + j];
                double u = z / h[j];
                if (cutoff && fabs(u) > reach) { skip = 1; break; }
                e += u * u;
                pw[j][0] = 1.0;
                for (int a = 1; a <= maxdeg; ++a) pw[j][a] = pw[j][a - 1] * z;
            }
            if (skip) continue;
            double K = norm * exp(-0.5 * e);
            for (int m = 0; m < n_s; ++m) {
                double v = K;
                for (int j = 0; j < d; ++j) v *= pw[j][exps_s[m * d + j]];
                nadd(&acc_s[m], v);
            }
            for (int m = 0; m < n_t; ++m) {
                double v = K;
                for (int j = 0; j < d; ++j) v *= pw[j][exps_t[m * d + j]];
                for (int w = 0; w < nw; ++w) nadd(&acc_t[(size_t)w * n_t + m], v * W[i * nw + w]);
            }
        }
        for (int m = 0; m < n_s; ++m) S[g * n_s + m] = acc_s[m].s + acc_s[m].c;
        for (int w = 0; w < nw; ++w)
            for (int m = 0; m < n_t; ++m)
                T[(g * nw + w) * n_t + m] = acc_t[(size_t)w * n_t + m].s + acc_t[(size_t)w * n_t + m].c;
        free(acc_s);
        free(acc_t);
    }
    return 0;
}

/* W is N x nw complex, interleaved (re, im); out is B x nw complex with
   B = prod_j (2 K_j + 1), mode index n_0 fastest, then the weight index. */
int orc_nudft(int d, int64_t N, const double* X, const double* lo, const double* period,
              int nw, const double* W, const int* K, double* out)
{
    if (d < 1 || d > ORC_MAXD) return -1;
    int64_t B = 1;
    int64_t ext[ORC_MAXD];
    for (int j = 0; j < d; ++j) { ext[j] = 2 * (int64_t)K[j] + 1; B *= ext[j]; }

#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t b = 0; b < B; ++b) {
        int64_t rem = b;
        double om[ORC_MAXD];
        for (int j = 0; j < d; ++j) {
            int64_t n = rem % ext[j] - K[j];
            rem /= ext[j];
            om[j] = 2.0 * M_PI * (double)n / period[j];
        }
        for (int w = 0; w < nw; ++w) {
            nsum re = {0, 0}, im = {0, 0};
            for (int64_t i = 0; i < N; ++i) {
                double ph = 0.0;
                for (int j = 0; j < d; ++j) ph += om[j] * (X[i * d + j] - lo[j]);
                double c = cos(ph), s = -sin(ph);
                double wr = W[(i * nw + w) * 2], wi = W[(i * nw + w) * 2 + 1];
                nadd(&re, wr * c - wi * s);
                nadd(&im, wr * s + wi * c);
            }
            out[(b * nw + w) * 2] = re.s + re.c;
            out[(b * nw + w) * 2 + 1] = im.s + im.c;
        }
    }
    return 0;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_threads(void) { return omp_get_max_threads(); }
