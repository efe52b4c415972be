// Device kernels of the fast kernel-regression path for gfx950 (CDNA4, wave64).
//
// Stages (Sec. 1.2 and Sec. 2 of the paper):
//   bin / scan / scatter   sort samples by spreading tile (once per X)
//   spread                 gridding of eq. (16)-(17): every sample adds its
//                          kernel footprint into an LDS copy of its padded tile
//                          (no global atomics)
//   fft pass               mixed-radix Stockham FFT along one axis in LDS,
//                          forward (eq. 19, keeping the retained band and
//                          dividing by the gridding kernel's transform, eq. 20)
//                          or inverse (eq. 21, zero-padded band -> grid rows).
//                          The first forward pass folds its rows (the padded
//                          tiles summed into the periodic fine grid); the
//                          first inverse pass expands its rows (kernel-moment
//                          spectra x data spectrum, eq. 12-13 in the frequency
//                          domain, two real channels per complex)
//   solve                  per-grid-point FP64 normal equations (eq. 3 / 11)
//   reduce                 interpolation to the samples with the Girard and
//                          residual dot products (Sec. 2.1, eq. 22)
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "kernels.h"

namespace fkr {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }
// a * (sgn i)
template <typename C> __device__ __forceinline__ C cmuli(C a, int sgn) { C r; r.x = -sgn * a.y; r.y = sgn * a.x; return r; }

__device__ __forceinline__ double load_as_double(const void* p, int type, int64_t i) {
    return type == FKR_F64 ? static_cast<const double*>(p)[i] : (double)static_cast<const float*>(p)[i];
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) + Box-Muller probes
// ---------------------------------------------------------------------------
// Sample i, probe p = 4 g + r: counter (i lo, i hi, g, 0), key (seed lo, seed
// hi); word x gives the uniform (floor(x / 2^8) + 1/2) 2^-24, exact in float
// and double.  Box-Muller pairs (u0, u1) -> normals 0, 1 and (u2, u3) -> 2, 3.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
        const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0; k1 += W1;
    }
}

__device__ __forceinline__ void philox_block(uint64_t seed, uint64_t i, uint32_t g, uint32_t x[4]) {
    x[0] = (uint32_t)i; x[1] = (uint32_t)(i >> 32); x[2] = g; x[3] = 0u;
    philox4x32_10(x, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Four normals of one block, in double (FP64 plans) ...
__device__ __forceinline__ void box_muller4(const uint32_t x[4], double z[4]) {
    double u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = ((double)(x[k] >> 8) + 0.5) * 0x1p-24;
    const double ra = sqrt(-2.0 * log(u[0])), rb = sqrt(-2.0 * log(u[2]));
    double sn, cs;
    sincospi(2.0 * u[1], &sn, &cs);
    z[0] = ra * cs; z[1] = ra * sn;
    sincospi(2.0 * u[3], &sn, &cs);
    z[2] = rb * cs; z[3] = rb * sn;
}

// ... or in single precision with the hardware log2 / sqrt / sin / cos (the
// trigonometric units take revolutions, so 2 pi u needs no multiply).
__device__ __forceinline__ void box_muller4(const uint32_t x[4], float z[4]) {
    float u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = ((float)(x[k] >> 8) + 0.5f) * 0x1p-24f;
    const float ln2 = 0.69314718055994531f;
    const float ra = __builtin_amdgcn_sqrtf(-2.0f * ln2 * __builtin_amdgcn_logf(u[0]));
    const float rb = __builtin_amdgcn_sqrtf(-2.0f * ln2 * __builtin_amdgcn_logf(u[2]));
    z[0] = ra * __builtin_amdgcn_cosf(u[1]); z[1] = ra * __builtin_amdgcn_sinf(u[1]);
    z[2] = rb * __builtin_amdgcn_cosf(u[3]); z[3] = rb * __builtin_amdgcn_sinf(u[3]);
}

__device__ double probe_value(uint64_t seed, uint64_t i, int p) {
    uint32_t x[4];
    philox_block(seed, i, (uint32_t)(p >> 2), x);
    double z[4];
    box_muller4(x, z);
    const int r = p & 3;
    return r == 0 ? z[0] : r == 1 ? z[1] : r == 2 ? z[2] : z[3];
}

__device__ __forceinline__ double wval(const WSrc& s, int64_t i) {
    switch (s.kind) {
        case W_ONE: return 1.0;
        case W_ARRAY: return load_as_double(s.ptr, s.type, i * s.stride + s.col);
        case W_PHILOX: return probe_value(s.seed, (uint64_t)i, s.probe);
        default: return 0.0;
    }
}

// ---------------------------------------------------------------------------
// Sample binning (once per X)
// ---------------------------------------------------------------------------
struct Binned {
    int c0[3];        // first footprint cell, wrapped into [0, Mr)
    double frac[3];   // u - first cell, in [w/2 - 1, w/2)
    int tile;
    int cell;         // first cell within the tile, pitch g.tsp
    bool outside;
};

template <int D>
__device__ __forceinline__ Binned bin_sample(const Geo& g, int x_type, const void* X, int64_t i) {
    Binned b;
    b.outside = false;
    int tile = 0, stride = 1, cell = 0, cstride = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double x = load_as_double(X, x_type, i * D + j);
        if (!(x >= g.lo[j] - g.tol[j] && x <= g.hi[j] + g.tol[j])) b.outside = true;
        x = fmin(fmax(x, g.lo[j]), g.hi[j]);
        const double u = (x - g.lo[j]) * g.inv_hf[j];
        const double cf = floor(u - 0.5 * g.w) + 1.0;
        b.frac[j] = u - cf;
        // 32-bit integer arithmetic: 0 <= u < Mr, so cf lies in [1 - w/2, Mr)
        // and one conditional add wraps it
        const int mr = (int)g.Mr[j], ts = (int)g.ts[j];
        int c0 = (int)cf;
        c0 = c0 < 0 ? c0 + mr : (c0 >= mr ? c0 - mr : c0);
        b.c0[j] = c0;
        const int tj = (int)((unsigned)c0 / (unsigned)ts);
        tile += tj * stride;
        stride *= (int)g.nt[j];
        cell += (c0 - tj * ts) * cstride;
        cstride *= g.tsp;
    }
    b.tile = tile;
    b.cell = cell;
    return b;
}

// Tile histogram: per-block LDS counts, then one global add per touched tile.
template <int D>
__global__ __launch_bounds__(kSortThreads) void k_bin_count(Geo g, int x_type, const void* X, int64_t N,
                                                   int32_t* counts, int32_t* bhist, int32_t* obuf) {
    extern __shared__ int32_t hist[];   // n_tiles entries when use_lds
    const bool use_lds = g.n_tiles <= kLdsHistMax;
    if (use_lds)
        for (int64_t t = threadIdx.x; t < g.n_tiles; t += blockDim.x) hist[t] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * kSortChunk;
    const int64_t end = min<int64_t>(N, beg + kSortChunk);
    __shared__ int32_t n_out;
    if (threadIdx.x == 0) n_out = 0;
    __syncthreads();
    int outside = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        Binned b = bin_sample<D>(g, x_type, X, i);
        if (use_lds) atomicAdd(&hist[b.tile], 1);
        else atomicAdd(&counts[b.tile], 1);
        outside += b.outside ? 1 : 0;
    }
    if (outside) atomicAdd(&n_out, outside);
    __syncthreads();
    if (threadIdx.x == 0) obuf[blockIdx.x] = n_out;   // summed by k_scan (no clearing needed)
    if (use_lds)   // this block's row of the block x tile count matrix (no atomics)
        for (int64_t t = threadIdx.x; t < g.n_tiles; t += blockDim.x)
            bhist[(int64_t)blockIdx.x * g.n_tiles + t] = hist[t];
}

// Column prefix of the block x tile count matrix: for tile t, bhist[b][t]
// becomes the number of samples of t in blocks before b and counts[t] the
// total, so each binning block owns a fixed, ordered range of every tile.
// A workgroup takes 64 consecutive tiles, one per lane, so every row of the
// matrix is read and written as one contiguous run; its 16 waves take
// consecutive ranges of rows and start from the totals of the ranges before.
__global__ __launch_bounds__(1024) void k_tile_prefix(int64_t n_tiles, int nblocks, int32_t* bhist,
                                                      int32_t* counts) {
    __shared__ int32_t part[16][64];
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * 64 + lane;
    const bool ok = t < n_tiles;
    const int per = (nblocks + 15) / 16;
    const int b0 = min(nblocks, seg * per), b1 = min(nblocks, b0 + per);
    int sum = 0;
    if (ok) {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) sum += bhist[(int64_t)b * n_tiles + t];
    }
    part[seg][lane] = sum;
    __syncthreads();
    int run = 0;
    for (int q = 0; q < seg; ++q) run += part[q][lane];
    if (ok) {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) {
            const int64_t at = (int64_t)b * n_tiles + t;
            const int v = bhist[at];
            bhist[at] = run;
            run += v;
        }
        if (seg == 15) counts[t] = run;
    }
}

// Single-block exclusive scans of the tile counts and of the job counts;
// writes tile_off, job_off, the job table and resets the scatter cursors.
__global__ __launch_bounds__(1024) void k_scan(int64_t n_tiles, int chunk, int64_t N, long long epoch,
                                               int32_t* counts, int32_t* tile_off, int32_t* job_off,
                                               int32_t* jobs, int32_t* cursor, long long* diag,
                                               const int32_t* obuf, int nbins) {
    __shared__ int64_t sa[1024], sb[1024];
    __shared__ int64_t smax[1024];
    const int t = threadIdx.x;
    const int64_t per = (n_tiles + 1023) / 1024;
    const int64_t beg = min<int64_t>(n_tiles, t * per), end = min<int64_t>(n_tiles, beg + per);
    int64_t a = 0, b = 0, mx = 0;
    for (int64_t k = beg; k < end; ++k) {
        const int64_t c = counts[k];
        a += c;
        b += (c + chunk - 1) / chunk;
        mx = c > mx ? c : mx;
    }
    sa[t] = a; sb[t] = b; smax[t] = mx;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t va = t >= off ? sa[t - off] : 0, vb = t >= off ? sb[t - off] : 0;
        int64_t vm = t >= off ? smax[t - off] : 0;
        __syncthreads();
        sa[t] += va; sb[t] += vb; smax[t] = vm > smax[t] ? vm : smax[t];
        __syncthreads();
    }
    int64_t ra = sa[t] - a, rb = sb[t] - b;
    for (int64_t k = beg; k < end; ++k) {
        const int64_t c = counts[k];
        tile_off[k] = (int32_t)ra;
        job_off[k] = (int32_t)rb;
        ra += c;
        rb += (c + chunk - 1) / chunk;
    }
    {   // samples outside [lo, hi]: sum of the binning pass's per-block counts
        __shared__ unsigned long long n_out;
        if (t == 0) n_out = 0;
        __syncthreads();
        unsigned long long o = 0;
        for (int b = t; b < nbins; b += 1024) o += (unsigned long long)obuf[b];
        if (o) atomicAdd(&n_out, o);
        __syncthreads();
        if (t == 0) diag[1] = (long long)n_out;
    }
    if (t == 0) {   // the device's record of the points (see PointsCheck)
        diag[kDiagN] = (long long)N;
        diag[kDiagEpoch] = epoch;
        diag[kDiagStale] = 0;
    }
    if (t == 1023) {
        tile_off[n_tiles] = (int32_t)sa[1023];
        job_off[n_tiles] = (int32_t)sb[1023];
        jobs[0] = (int32_t)sb[1023];   // job count in the table header
        diag[3] = sb[1023];
        diag[4] = smax[1023];
    }
    __syncthreads();
    // job table entries: (tile, start, end, order) at jobs[4 + 4 * job].
    // Processing order (field 3 of entry b = the job that workgroup b of a
    // spread takes): jobs bucketed by size, largest first, so the workgroups
    // that the dispatcher hands out last are the short ones.  The order
    // within a bucket is arbitrary; every job writes its own subgrid.
    __shared__ int32_t bcnt[8];
    if (t < 8) bcnt[t] = 0;
    __syncthreads();
    auto bucket = [&](int64_t sz) { return min(7, (int)(((int64_t)chunk - sz) * 8 / chunk)); };
    for (int64_t k = t; k < n_tiles; k += 1024) {
        const int64_t c = counts[k];
        const int64_t nj = (c + chunk - 1) / chunk;
        const int64_t j0 = job_off[k], s0 = tile_off[k];
        for (int64_t q = 0; q < nj; ++q) {
            int32_t* e = jobs + 4 + 4 * (j0 + q);
            // nj near-equal pieces of at most one chunk each
            const int64_t a0 = s0 + q * c / nj, a1 = s0 + (q + 1) * c / nj;
            e[0] = (int32_t)k;
            e[1] = (int32_t)a0;
            e[2] = (int32_t)a1;
            atomicAdd(&bcnt[bucket(a1 - a0)], 1);
        }
        cursor[k] = 0;
    }
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int b = 0; b < 8; ++b) { const int c = bcnt[b]; bcnt[b] = run; run += c; }
    }
    __syncthreads();
    for (int64_t k = t; k < n_tiles; k += 1024) {
        const int64_t c = counts[k];
        const int64_t nj = (c + chunk - 1) / chunk;
        const int64_t j0 = job_off[k];
        for (int64_t q = 0; q < nj; ++q) {
            const int64_t sz = (q + 1) * c / nj - q * c / nj;   // the piece sizes of the loop above
            jobs[4 + 4 * atomicAdd(&bcnt[bucket(sz)], 1) + 3] = (int32_t)(j0 + q);
        }
    }
}

// Tile-ordered sample record: original index, packed first cell relative to
// the tile (10 bits per dimension), fractions and clamped coordinates, padded
// to a multiple of 16 bytes so it moves with vector stores and loads.
template <int D, typename T>
struct TileRec {
    static constexpr int BYTES = 8 + 2 * D * (int)sizeof(T);
    static constexpr int WORDS = ((BYTES + 15) / 16) * 4;   // 32-bit words
    uint32_t w[WORDS];
    __device__ __forceinline__ T& at(int k) { return reinterpret_cast<T*>(w + 2)[k]; }
    __device__ __forceinline__ const T& at(int k) const { return reinterpret_cast<const T*>(w + 2)[k]; }
};

// Scatter into tile order: each block ranks its samples per tile in LDS,
// reserves a range per touched tile with one global add, and writes the
// sample's record at its tile-ordered position.  The binning is evaluated
// twice (the second time from the cached coordinates) rather than kept in
// registers.
template <int D, typename T>
__global__ __launch_bounds__(kSortThreads) void k_scatter_tiles(Geo g, int x_type, const void* X, int64_t N,
                                                       const int32_t* tile_off, int32_t* cursor,
                                                       const int32_t* bhist, TileRec<D, T>* trec) {
    extern __shared__ int32_t lcount[];   // [n_tiles] local counts, then bases
    const bool use_lds = g.n_tiles <= kLdsHistMax;
    if (use_lds)
        for (int64_t t = threadIdx.x; t < g.n_tiles; t += blockDim.x) lcount[t] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * kSortChunk;
    const int64_t end = min<int64_t>(N, beg + kSortChunk);
    constexpr int kPer = kSortChunk / kSortThreads;
    int rank[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t i = beg + threadIdx.x + (int64_t)q * kSortThreads;
        rank[q] = 0;
        if (i < end) {
            const int t = bin_sample<D>(g, x_type, X, i).tile;
            rank[q] = use_lds ? atomicAdd(&lcount[t], 1) : atomicAdd(&cursor[t], 1);
        }
    }
    __syncthreads();
    if (use_lds)   // this block's range of every tile, from the column prefix
        for (int64_t t = threadIdx.x; t < g.n_tiles; t += blockDim.x)
            lcount[t] = bhist[(int64_t)blockIdx.x * g.n_tiles + t];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t i = beg + threadIdx.x + (int64_t)q * kSortThreads;
        if (i >= end) continue;
        const Binned b = bin_sample<D>(g, x_type, X, i);
        const int t = b.tile;
        const int64_t pos = tile_off[t] + (use_lds ? lcount[t] : 0) + rank[q];
        if (pos >= tile_off[t + 1]) continue;
        TileRec<D, T> r;
#pragma unroll
        for (int k = 0; k < TileRec<D, T>::WORDS; ++k) r.w[k] = 0u;
        r.w[0] = (uint32_t)i;
        uint32_t l = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int ts = (int)g.ts[j];
            const int tj = (int)((unsigned)b.c0[j] / (unsigned)ts);
            l |= (uint32_t)(b.c0[j] - tj * ts) << (10 * j);
            r.at(j) = (T)b.frac[j];
            const double x = load_as_double(X, x_type, i * D + j);
            r.at(D + j) = (T)fmin(fmax(x, g.lo[j]), g.hi[j]);
        }
        r.w[1] = l;
        uint4* dst = reinterpret_cast<uint4*>(trec + pos);
#pragma unroll
        for (int k = 0; k < TileRec<D, T>::WORDS / 4; ++k)
            dst[k] = make_uint4(r.w[4 * k], r.w[4 * k + 1], r.w[4 * k + 2], r.w[4 * k + 3]);
    }
}

// Local cell (pitch g.tsp) of a packed first-cell record: the sort key of
// the samples within a job.  In 3-D the key is (x, y) major and z minor, so
// the samples of one (x, y) column of first cells are contiguous with z
// ascending (the 3-D column spread keeps such a run in registers).
template <int D>
__device__ __forceinline__ int local_cell(const Geo& g, uint32_t l) {
    const int x = (int)(l & 1023);
    if (D == 1) return x;
    const int y = (int)((l >> 10) & 1023);
    if (D == 2) return x + g.tsp * y;
    const int z = (int)((l >> 20) & 1023);
    return z + g.tsp * (x + g.tsp * y);
}

// Per job (a tile-ordered range of at most one chunk): order the job's
// records by first cell within the job's own range, writing the packed first
// cell, fractions, clamped coordinates and original index.  Counts per cell
// in LDS, an exclusive scan over the cells, then LDS-atomic ranks.  The jobs
// keep the ranges the tile scatter gave them, so a tile's samples end up in
// (job, cell) order and no job needs another job's counts.  When the records
// fit the LDS budget they are placed there first and leave as one contiguous
// run.
template <int D, typename T, int NT>
__global__ __launch_bounds__(NT) void k_cell_sort(Geo g, const int32_t* jobs, const TileRec<D, T>* trec,
                                                  int stage, uint32_t* loc, T* frac, int32_t* perm, T* xs) {
    // [ncell] counts, then cursors; [NT] scan scratch; staged records
    extern __shared__ int32_t cur[];
    const int job = blockIdx.x;
    if (job >= jobs[0]) return;
    const int32_t* jd = jobs + 4 + 4 * job;
    const int s0 = jd[1], s1 = jd[2], n = s1 - s0;
    int32_t* scan = cur + g.ncell;
    uint32_t* sl_loc = reinterpret_cast<uint32_t*>(scan + NT);
    int32_t* sl_perm = reinterpret_cast<int32_t*>(sl_loc + g.chunk);
    T* sl_frac = reinterpret_cast<T*>(sl_perm + g.chunk);
    T* sl_xs = sl_frac + (int64_t)g.chunk * D;
    for (int c = threadIdx.x; c < g.ncell; c += blockDim.x) cur[c] = 0;
    __syncthreads();
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) atomicAdd(&cur[local_cell<D>(g, trec[s].w[1])], 1);
    __syncthreads();
    // exclusive scan of the counts: thread t owns cells [t per, (t + 1) per),
    // block scan of the thread sums
    const int per = (g.ncell + NT - 1) / NT;
    const int c_beg = min(g.ncell, (int)threadIdx.x * per), c_end = min(g.ncell, c_beg + per);
    int sum = 0;
    for (int c = c_beg; c < c_end; ++c) sum += cur[c];
    scan[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {
        const int v = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    int run = scan[threadIdx.x] - sum;
    for (int c = c_beg; c < c_end; ++c) {
        const int v = cur[c];
        cur[c] = run;
        run += v;
    }
    __syncthreads();
    for (int s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        TileRec<D, T> r;
        const uint4* src = reinterpret_cast<const uint4*>(trec + s);
#pragma unroll
        for (int k = 0; k < TileRec<D, T>::WORDS / 4; ++k) {
            const uint4 v = src[k];
            r.w[4 * k] = v.x; r.w[4 * k + 1] = v.y; r.w[4 * k + 2] = v.z; r.w[4 * k + 3] = v.w;
        }
        const uint32_t l = r.w[1];
        const int k = atomicAdd(&cur[local_cell<D>(g, l)], 1);
        if (k >= n) continue;   // never taken: the ranks are a permutation of 0 .. n-1
        if (stage) {
            sl_loc[k] = l;
            sl_perm[k] = (int32_t)r.w[0];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                sl_frac[k * D + j] = r.at(j);
                sl_xs[k * D + j] = r.at(D + j);
            }
        } else {
            const int64_t pos = (int64_t)s0 + k;
            loc[pos] = l;
            perm[pos] = (int32_t)r.w[0];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                frac[pos * D + j] = r.at(j);
                xs[pos * D + j] = r.at(D + j);
            }
        }
    }
    if (!stage) return;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        loc[s0 + k] = sl_loc[k];
        perm[s0 + k] = sl_perm[k];
    }
    for (int k = threadIdx.x; k < n * D; k += blockDim.x) {
        frac[(int64_t)s0 * D + k] = sl_frac[k];
        xs[(int64_t)s0 * D + k] = sl_xs[k];
    }
}

// ---------------------------------------------------------------------------
// Spreading into LDS tiles (eq. 16-17)
// ---------------------------------------------------------------------------
// Spreading kernel value at distance t (fine cells).  FP32 uses the hardware
// exp2 / sqrt approximations (about 1 ulp), FP64 the accurate library ones.
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double fast_exp(double x) { return exp(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }

template <typename T, int KER>
__device__ __forceinline__ T kernel_value(T t, int w, T kp) {
    if (KER == FKR_KERNEL_ES) {
        const T s = t * ((T)2 / (T)w);
        const T q = (T)1 - s * s;
        return q > (T)0 ? fast_exp(kp * (fast_sqrt(q) - (T)1)) : (T)0;
    } else {
        return fast_exp(-kp * t * t);
    }
}

// A weight read from memory or a constant (the spreading reads weights that
// k_stage_weights has put in sorted order; generated probes never reach it).
__device__ __forceinline__ double wval_mem(const WSrc& s, int64_t sp, int64_t i) {
    switch (s.kind) {
        case W_ONE: return 1.0;
        case W_ARRAY: return load_as_double(s.ptr, s.type, i * s.stride + s.col);
        case W_SORTED:
            return load_as_double(s.ptr, s.type,
                                  s.gstride ? (s.col >> 2) * s.gstride + sp * s.stride + (s.col & 3)
                                            : sp * s.stride + s.col);
        default: return 0.0;
    }
}

// Kernel values psi(k - f), k = 0..W-1, of one dimension.
template <int W, typename T, int KER>
__device__ __forceinline__ void kernel_row(T f, T kp, T (&kv)[W]) {
#pragma unroll
    for (int k = 0; k < W; ++k) kv[k] = kernel_value<T, KER>((T)k - f, W, kp);
}

// One job = a range of at most one chunk of samples of one tile, sorted by
// first footprint cell.  The job is cut into equal
// segments of consecutive samples; segment NWAVE * l + v goes to lane l of
// wave v, so the lanes of a wave hold segments far apart and rarely share a
// cell.  With ACC (1-D, and 2-D FP32 with W^2 <= 64) a thread sums the
// footprints of consecutive samples that share a first cell in registers and
// adds them to the tile when the cell changes; otherwise every sample's
// footprint is added directly.  The tile accumulates in FP64 in LDS (LDS FP64
// atomics are an order of magnitude faster than FP32 ones on gfx950) with the
// compile-time pitch PE = TS + W - 1 and is written out in the element type T,
// one pair of weight vectors at a time.
template <int D, int W, typename T, int KER>
__global__ __launch_bounds__(kSpreadBlock) void k_spread(Geo g, SpreadSrc src, const uint32_t* loc,
                                                         const T* frac, const int32_t* perm,
                                                         const int32_t* jobs, T* subgrid) {
    constexpr int TS = spread_tile_edge(D, W);
    constexpr int PE = TS + W - 1;
    constexpr int PSUB = D == 1 ? PE : (D == 2 ? PE * PE : PE * PE * PE);
    constexpr bool ACC = D == 1 || (D == 2 && W * W * (int)sizeof(T) <= 256);
    constexpr int NWAVE = kSpreadBlock / 64;
    constexpr int SB = 2;   // samples loaded per batch
    __shared__ double tile[2 * PSUB];
    const int njobs = jobs[0];
    const int np = src.npairs;
    const T kp = (T)g.kparam;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int segid = lane * NWAVE + wave;
    for (int b = blockIdx.x; b < njobs; b += gridDim.x) {
        const int job = jobs[4 + 4 * b + 3];
        const int32_t* jd = jobs + 4 + 4 * job;
        const int s_beg = jd[1];
        const int n = jd[2] - jd[1];
        const int seg = (n + kSpreadBlock - 1) / kSpreadBlock;
        const int q0 = min(n, segid * seg), q1 = min(n, q0 + seg);
        for (int p = 0; p < np; ++p) {
            for (int q = threadIdx.x; q < 2 * PSUB; q += blockDim.x) tile[q] = 0.0;
            __syncthreads();
            if (ACC) {
                T ar[D == 1 ? W : W * W], ai[D == 1 ? W : W * W];
#pragma unroll
                for (int k = 0; k < (D == 1 ? W : W * W); ++k) ar[k] = ai[k] = (T)0;
                int cur_base = -1;
                // Batches of SB samples: all loads of a batch are issued before
                // any of its samples is used (memory-level parallelism).
                for (int qb = q0; qb < q1; qb += SB) {
                    int bb[SB];
                    int64_t ip[SB];
                    T f0[SB], f1[SB], wr[SB], wi[SB];
#pragma unroll
                    for (int u = 0; u < SB; ++u) {
                        const int q = qb + u;
                        bb[u] = -1;
                        if (q < q1) {
                            const int64_t s = s_beg + q;
                            const uint32_t l = loc[s];
                            bb[u] = (int)(l & 1023) + (D > 1 ? PE * (int)((l >> 10) & 1023) : 0);
                            f0[u] = frac[s * D];
                            f1[u] = D > 1 ? frac[s * D + 1] : (T)0;
                            ip[u] = perm[s];
                            wr[u] = (T)wval_mem(src.w[2 * p], s, ip[u]);
                            wi[u] = (T)wval_mem(src.w[2 * p + 1], s, ip[u]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < SB; ++u) {
                        if (bb[u] < 0) break;
                        if (bb[u] != cur_base && cur_base >= 0) {   // flush the running cell
                            double* re = tile + cur_base;
                            double* im = re + PSUB;
                            if (D == 1) {
#pragma unroll
                                for (int k0 = 0; k0 < W; ++k0) {
                                    atomicAdd(re + k0, (double)ar[k0]);
                                    atomicAdd(im + k0, (double)ai[k0]);
                                    ar[k0] = ai[k0] = (T)0;
                                }
                            } else {
#pragma unroll
                                for (int k1 = 0; k1 < W; ++k1)
#pragma unroll
                                    for (int k0 = 0; k0 < W; ++k0) {
                                        atomicAdd(re + k1 * PE + k0, (double)ar[k1 * W + k0]);
                                        atomicAdd(im + k1 * PE + k0, (double)ai[k1 * W + k0]);
                                        ar[k1 * W + k0] = ai[k1 * W + k0] = (T)0;
                                    }
                            }
                        }
                        cur_base = bb[u];
                        T kv0[W];
                        kernel_row<W, T, KER>(f0[u], kp, kv0);
                        if (D == 1) {
#pragma unroll
                            for (int k0 = 0; k0 < W; ++k0) {
                                ar[k0] += kv0[k0] * wr[u];
                                ai[k0] += kv0[k0] * wi[u];
                            }
                        } else {
                            T kv1[W];
                            kernel_row<W, T, KER>(f1[u], kp, kv1);
#pragma unroll
                            for (int k1 = 0; k1 < W; ++k1) {
                                const T a = kv1[k1] * wr[u], b = kv1[k1] * wi[u];
#pragma unroll
                                for (int k0 = 0; k0 < W; ++k0) {
                                    ar[k1 * W + k0] += kv0[k0] * a;
                                    ai[k1 * W + k0] += kv0[k0] * b;
                                }
                            }
                        }
                    }
                }
                if (cur_base >= 0) {   // flush the last cell
                    double* re = tile + cur_base;
                    double* im = re + PSUB;
                    if (D == 1) {
#pragma unroll
                        for (int k0 = 0; k0 < W; ++k0) {
                            atomicAdd(re + k0, (double)ar[k0]);
                            atomicAdd(im + k0, (double)ai[k0]);
                        }
                    } else {
#pragma unroll
                        for (int k1 = 0; k1 < W; ++k1)
#pragma unroll
                            for (int k0 = 0; k0 < W; ++k0) {
                                atomicAdd(re + k1 * PE + k0, (double)ar[k1 * W + k0]);
                                atomicAdd(im + k1 * PE + k0, (double)ai[k1 * W + k0]);
                            }
                    }
                }
            } else {
                for (int qb = q0; qb < q1; qb += SB) {
                    int bb[SB];
                    int64_t ip[SB];
                    T f0[SB], f1[SB], f2[SB], wr[SB], wi[SB];
#pragma unroll
                    for (int u = 0; u < SB; ++u) {
                        const int q = qb + u;
                        bb[u] = -1;
                        if (q < q1) {
                            const int64_t s = s_beg + q;
                            const uint32_t l = loc[s];
                            bb[u] = (int)(l & 1023) + (D > 1 ? PE * (int)((l >> 10) & 1023) : 0) +
                                    (D > 2 ? PE * PE * (int)((l >> 20) & 1023) : 0);
                            f0[u] = frac[s * D];
                            f1[u] = D > 1 ? frac[s * D + 1] : (T)0;
                            f2[u] = D > 2 ? frac[s * D + 2] : (T)0;
                            ip[u] = perm[s];
                            wr[u] = (T)wval_mem(src.w[2 * p], s, ip[u]);
                            wi[u] = (T)wval_mem(src.w[2 * p + 1], s, ip[u]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < SB; ++u) {
                        if (bb[u] < 0) break;
                        T kv0[W], kv1[W];
                        kernel_row<W, T, KER>(f0[u], kp, kv0);
                        if (D > 1) kernel_row<W, T, KER>(f1[u], kp, kv1);
                        double* re = tile + bb[u];
                        double* im = re + PSUB;
                        if (D == 1) {
#pragma unroll
                            for (int k0 = 0; k0 < W; ++k0) {
                                atomicAdd(re + k0, (double)(kv0[k0] * wr[u]));
                                atomicAdd(im + k0, (double)(kv0[k0] * wi[u]));
                            }
                        } else if (D == 2) {
#pragma unroll
                            for (int k1 = 0; k1 < W; ++k1) {
                                const double a = (double)(kv1[k1] * wr[u]), b = (double)(kv1[k1] * wi[u]);
#pragma unroll
                                for (int k0 = 0; k0 < W; ++k0) {
                                    atomicAdd(re + k1 * PE + k0, (double)kv0[k0] * a);
                                    atomicAdd(im + k1 * PE + k0, (double)kv0[k0] * b);
                                }
                            }
                        } else {
                            for (int k2 = 0; k2 < W; ++k2) {
                                const T v2 = kernel_value<T, KER>((T)k2 - f2[u], W, kp);
                                const double a2 = (double)(v2 * wr[u]), b2 = (double)(v2 * wi[u]);
                                double* re2 = re + k2 * PE * PE;
                                double* im2 = im + k2 * PE * PE;
#pragma unroll
                                for (int k1 = 0; k1 < W; ++k1) {
                                    const double a = (double)kv1[k1] * a2, b = (double)kv1[k1] * b2;
#pragma unroll
                                    for (int k0 = 0; k0 < W; ++k0) {
                                        atomicAdd(re2 + k1 * PE + k0, (double)kv0[k0] * a);
                                        atomicAdd(im2 + k1 * PE + k0, (double)kv0[k0] * b);
                                    }
                                }
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // subgrid layout [job][pair][cell][re, im]
            T* dst = subgrid + ((int64_t)job * np + p) * PSUB * 2;
            for (int c = threadIdx.x; c < PSUB; c += blockDim.x) {
                dst[2 * c] = (T)tile[c];
                dst[2 * c + 1] = (T)tile[PSUB + c];
            }
            __syncthreads();
        }
    }
}

// Lane layout of the group spread: a group of G lanes covers the W^D
// footprint cells of one sample, R cells per lane, and 64 / G groups share a
// wave.  In 2-D a lane owns column dx = gl % W and rows gl / W + GY r; in 3-D
// it owns the column (gl % W, gl / W) and every plane dz = r.
template <int D, int W> struct Foot {
    static constexpr int R = D == 1 ? 1 : (D == 2 ? (W <= 8 ? 2 : (W <= 16 ? 4 : 12)) : W);
    static constexpr int GY = D == 1 ? 1 : (D == 2 ? (W + R - 1) / R : W);
    static constexpr int G = D == 1 ? W : W * GY;
    static constexpr int NG = G <= 64 ? 64 / G : 1;
    static constexpr bool ok = G <= 64 && G >= D * W && spread_tile_edge(D, W) > 0;
};

template <typename T, int NW>
__device__ __forceinline__ void load_weight_row(const T* row, int nw, T (&wv)[NW]) {
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int c = 0; c < NW / 4; ++c) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (4 * c < nw) v = *reinterpret_cast<const float4*>(row + 4 * c);
            wv[4 * c] = v.x; wv[4 * c + 1] = v.y; wv[4 * c + 2] = v.z; wv[4 * c + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int c = 0; c < NW / 2; ++c) {
            double2 v = make_double2(0.0, 0.0);
            if (2 * c < nw) v = *reinterpret_cast<const double2*>(row + 2 * c);
            wv[2 * c] = v.x; wv[2 * c + 1] = v.y;
        }
    }
}

// Group spread of one launch (np <= 8 weight pairs, 2 np real weight columns
// starting at col0 of the sorted weight rows).  One block per job; the job's
// samples (sorted by first footprint cell) are cut into NGB = 4 NG segments,
// one per lane group, interleaved so that the groups of a wave work far
// apart.  The block walks all segments in lockstep chunks of CS samples per
// group: the records (first cell, fractions) and weight rows of the next
// chunk are loaded into registers while the current one, staged in LDS, is
// being spread (double buffer, one barrier per chunk).  For every sample the
// group's lanes evaluate the D kernel rows once (one value per lane),
// exchange them with cross-lane permutes, and add psi * w_k for all weight
// columns to registers that belong to the lane's footprint cells.  Registers
// are added into the FP64 LDS tile only when the group's first footprint cell
// changes, so consecutive samples of one cell cost no LDS atomics.  The tile
// (pitch PE = TS + W - 1) is written out in the element type T exactly as
// the per-pair subgrids of k_spread.
template <int D, int W, typename T, int NWMAX_>
struct GroupStage {
    static constexpr int NGB = (kSpreadBlock / 64) * Foot<D, W>::NG;
    static constexpr int STAGE = sizeof(T) == 4 ? 256 : 128;    // staged samples per chunk
    static constexpr int CS = STAGE / NGB > 0 ? STAGE / NGB : 1;
    static constexpr int NS = NGB * CS;
    static constexpr int NWMAX = NWMAX_;
    static constexpr int RECW = 4;                               // loc bits + up to 3 fractions
    // doubles in LDS: tile [NWMAX][PSUB], then two buffers of NS records and NS rows
    static constexpr size_t stage_bytes = 2 * (size_t)NS * (RECW + NWMAX) * sizeof(T);
};

template <int D, int W, typename T, int KER, int NWMAX>
__global__ __launch_bounds__(kSpreadBlock) void k_spread_group(Geo g, int np, const T* wrow, int wstride,
                                                               int col0, const uint32_t* loc, const T* frac,
                                                               const int32_t* jobs, T* subgrid) {
    using F = Foot<D, W>;
    using GS = GroupStage<D, W, T, NWMAX>;
    constexpr int TS = spread_tile_edge(D, W);
    constexpr int PE = TS + W - 1;
    constexpr int PSUB = D == 1 ? PE : (D == 2 ? PE * PE : PE * PE * PE);
    constexpr int NWAVE = kSpreadBlock / 64;
    constexpr int NGB = GS::NGB, CS = GS::CS, NS = GS::NS, RECW = GS::RECW;
    constexpr int PPP = NWMAX / 2;
    constexpr int R = F::R;
    constexpr int U = 4;   // samples per group per step (CS is a multiple of U)
    extern __shared__ double tile[];   // [NWMAX][PSUB] doubles, then the staging buffers
    // staging in LDS (integer offsets keep the accesses in the LDS address space):
    // records [2][NS][RECW], then weight rows [2][NS][NWMAX]
    T* const stg = reinterpret_cast<T*>(tile + NWMAX * PSUB);
    constexpr int WOFF = 2 * NS * RECW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = min(lane / F::G, F::NG - 1);
    const int gl = lane - grp * F::G;
    const bool member = lane < F::NG * F::G;
    const int gbase = grp * F::G;
    const int segid = grp * NWAVE + wave;
    const int dx = gl % W;
    const int dyb = D == 1 ? 0 : gl / W;
    const int pj = min(gl / W, D - 1), pk = gl % W;
    const bool psi_lane = gl < D * W;
    const T kp = (T)g.kparam;
    // loader role: thread -> (segment, sample within the chunk)
    const int lseg = threadIdx.x / CS, lk = threadIdx.x - lseg * CS;
    const bool loader = threadIdx.x < NS;
    const int njobs = jobs[0];
    for (int b = blockIdx.x; b < njobs; b += gridDim.x) {
        const int job = jobs[4 + 4 * b + 3];
        const int32_t* jd = jobs + 4 + 4 * job;
        const int s_beg = jd[1];
        const int n = jd[2] - jd[1];
        const int seg = (n + NGB - 1) / NGB;
        const int nchunk = (seg + CS - 1) / CS;
        const int q0 = min(n, segid * seg);
        const int len = member ? min(n, q0 + seg) - q0 : 0;
        // the loader's segment (segments are numbered like segid)
        const int lq0 = min(n, lseg * seg), lq1 = min(n, lq0 + seg);
        for (int p0 = 0; p0 < np; p0 += PPP) {
            const int nw = 2 * min(PPP, np - p0);
            for (int c = threadIdx.x; c < nw * PSUB; c += blockDim.x) tile[c] = 0.0;
            // register copy of the next chunk
            T rrec[RECW], rw[NWMAX];
            auto fetch = [&](int ch) {
                const int q = lq0 + ch * CS + lk;
                const bool ok = loader && q < lq1;
                const int64_t sidx = s_beg + (ok ? q : 0);
                rrec[0] = ok ? __builtin_bit_cast(T, (typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type)loc[sidx]) : (T)0;
#pragma unroll
                for (int j = 0; j < 3; ++j) rrec[1 + j] = (ok && j < D) ? frac[sidx * D + j] : (T)0;
                if (ok) load_weight_row<T, NWMAX>(wrow + sidx * wstride + col0 + 2 * p0, nw, rw);
            };
            auto stash = [&](int buf) {
                if (!loader) return;
                const int slot = lseg * CS + lk;
#pragma unroll
                for (int j = 0; j < RECW; ++j) stg[(buf * NS + slot) * RECW + j] = rrec[j];
#pragma unroll
                for (int k = 0; k < NWMAX; k += 2) {
                    if (k >= nw) break;
                    stg[WOFF + (buf * NS + slot) * NWMAX + k] = rw[k];
                    stg[WOFF + (buf * NS + slot) * NWMAX + k + 1] = rw[k + 1];
                }
            };
            T acc[R][NWMAX];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < NWMAX; ++k) acc[r][k] = (T)0;
            int cur = -1;
            if (nchunk > 0) fetch(0);
            for (int ch = 0; ch < nchunk; ++ch) {
                const int buf = ch & 1;
                stash(buf);
                __syncthreads();
                if (ch + 1 < nchunk) fetch(ch + 1);
                const int rec0 = (buf * NS + segid * CS) * RECW;
                const int wts0 = WOFF + (buf * NS + segid * CS) * NWMAX;
                const int tmax = min(CS, len - ch * CS);   // may be <= 0 for this group
                const int wmax = min(CS, max(0, min(seg, n - wave * seg)) - ch * CS);   // first group of the wave
                // U samples per group per step: their LDS reads, kernel rows
                // and permutes are independent, so their latencies overlap
                for (int t = 0; t < wmax; t += U) {
                    T psi[U][R];
                    int cbu[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int tt = min(t + u, max(tmax - 1, 0));
                        T rv[RECW];
#pragma unroll
                        for (int j = 0; j < RECW; ++j) rv[j] = stg[rec0 + tt * RECW + j];
                        const uint32_t l = (uint32_t)__builtin_bit_cast(
                            typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type, rv[0]);
                        cbu[u] = (int)(l & 1023) + (D > 1 ? PE * (int)((l >> 10) & 1023) : 0) +
                                 (D > 2 ? PE * PE * (int)((l >> 20) & 1023) : 0);
                        T fj = rv[1];
                        if (D > 1 && pj == 1) fj = rv[2];
                        if (D > 2 && pj == 2) fj = rv[3];
                        const T v = psi_lane ? kernel_value<T, KER>((T)pk - fj, W, kp) : (T)0;
                        if (D == 1) {
                            psi[u][0] = v;
                        } else if (D == 2) {
                            const T a = __shfl(v, gbase + dx);
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                const int dy = dyb + F::GY * r;
                                const T b = __shfl(v, gbase + W + min(dy, W - 1));
                                psi[u][r] = dy < W ? a * b : (T)0;
                            }
                        } else {
                            const T ab = __shfl(v, gbase + dx) * __shfl(v, gbase + W + dyb);
#pragma unroll
                            for (int r = 0; r < R; ++r) psi[u][r] = ab * __shfl(v, gbase + 2 * W + r);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (t + u >= tmax) break;
                        const int tt = t + u;
                        if (cbu[u] != cur) {
                            if (cur >= 0) {
#pragma unroll
                                for (int r = 0; r < R; ++r) {
                                    const int dy = dyb + F::GY * r;
                                    if (D == 2 && dy >= W) continue;
                                    const int cell = cur + dx + (D == 2 ? PE * dy : (D == 3 ? PE * dyb + PE * PE * r : 0));
#pragma unroll
                                    for (int k = 0; k < NWMAX; k += 2) {
                                        if (k >= nw) break;
                                        atomicAdd(&tile[k * PSUB + cell], (double)acc[r][k]);
                                        atomicAdd(&tile[(k + 1) * PSUB + cell], (double)acc[r][k + 1]);
                                        acc[r][k] = acc[r][k + 1] = (T)0;
                                    }
                                }
                            }
                            cur = cbu[u];
                        }
#pragma unroll
                        for (int k = 0; k < NWMAX; k += 2) {
                            if (k >= nw) break;
                            const T w0 = stg[wts0 + tt * NWMAX + k], w1 = stg[wts0 + tt * NWMAX + k + 1];
#pragma unroll
                            for (int r = 0; r < R; ++r) {
                                acc[r][k] += psi[u][r] * w0;
                                acc[r][k + 1] += psi[u][r] * w1;
                            }
                        }
                    }
                }
            }
            if (cur >= 0) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int dy = dyb + F::GY * r;
                    if (D == 2 && dy >= W) continue;
                    const int cell = cur + dx + (D == 2 ? PE * dy : (D == 3 ? PE * dyb + PE * PE * r : 0));
#pragma unroll
                    for (int k = 0; k < NWMAX; k += 2) {
                        if (k >= nw) break;
                        atomicAdd(&tile[k * PSUB + cell], (double)acc[r][k]);
                        atomicAdd(&tile[(k + 1) * PSUB + cell], (double)acc[r][k + 1]);
                    }
                }
            }
            __syncthreads();
            // subgrid layout [job][pair][cell][re, im]
            for (int q = 0; 2 * q < nw; ++q) {
                T* dst = subgrid + ((int64_t)job * np + p0 + q) * PSUB * 2;
                for (int c = threadIdx.x; c < PSUB; c += blockDim.x) {
                    dst[2 * c] = (T)tile[2 * q * PSUB + c];
                    dst[2 * c + 1] = (T)tile[(2 * q + 1) * PSUB + c];
                }
            }
            __syncthreads();
        }
    }
}

// Fine cell (c_0, .., c_{d-1}) of pair p = sum over the padded tiles that
// cover it and over the jobs of each such tile, in a fixed order
// (deterministic).  One thread per (cell, pair) item; consecutive threads take
// consecutive cells of one pair, so the subgrid reads of a wave fall on rows
// of the same tiles.  With a0_step = 2 only the covering tiles a0 = a0_first,
// a0_first + 2, .. of dimension 0 are summed (two threads share a cell).
template <int D, typename T>
__device__ __forceinline__ double2 fold_at(const FoldArgs& fa, int p, unsigned cell, int a0_first = 0,
                                           int a0_step = 1) {
    const T* subgrid = static_cast<const T*>(fa.subgrid);
    const int cs = 1 + 2 * kCoverSlots;
    const int32_t* cv[3];
    unsigned rem = cell;
    int64_t cov_base = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j < D) {
            const unsigned mr = (unsigned)fa.Mr[j];
            const unsigned qj = rem / mr;
            const unsigned c = rem - qj * mr;
            rem = qj;
            cv[j] = fa.cover + cov_base + (int64_t)c * cs;
            cov_base += (int64_t)mr * cs;
        }
    }
    const int64_t lsize = fa.Psub * fa.np * 2;
    const int n0 = cv[0][0];
    const int n1 = D > 1 ? cv[1][0] : 1;
    const int n2 = D > 2 ? cv[2][0] : 1;
    double re = 0.0, im = 0.0;
    if (n0 <= 2 && n1 <= 2 && n2 <= 2) {
        // Common case, at most two covering tiles per dimension: every job
        // offset, then every first-job subgrid value, is loaded before any is
        // used, so the chain is cover -> job offsets -> subgrids (a dense
        // tile's further jobs follow).  Same summation order as below.
        constexpr int NT = 1 << D;
        int64_t tl[NT], of[NT];
        bool ok[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const int a0 = k & 1, a1 = (k >> 1) & 1, a2 = (k >> 2) & 1;
            ok[k] = a0 < n0 && (D < 2 || a1 < n1) && (D < 3 || a2 < n2) &&
                    (a0_step == 1 || a0 == a0_first);
            int64_t tile = 0, off = 0;
            if (ok[k]) {
                tile = cv[0][1 + 2 * a0];
                off = cv[0][2 + 2 * a0];
                if (D > 1) {
                    tile += fa.nt0 * cv[1][1 + 2 * a1];
                    off += fa.pe0 * cv[1][2 + 2 * a1];
                }
                if (D > 2) {
                    tile += fa.nt0 * fa.nt1 * cv[2][1 + 2 * a2];
                    off += fa.pe0 * fa.pe1 * cv[2][2 + 2 * a2];
                }
            }
            tl[k] = tile;
            of[k] = off;
        }
        int j0[NT], j1[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            j0[k] = ok[k] ? fa.job_off[tl[k]] : 0;
            j1[k] = ok[k] ? fa.job_off[tl[k] + 1] : 0;
        }
        T fr[NT], fi[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            fr[k] = fi[k] = (T)0;
            if (j0[k] < j1[k]) {
                const T* sg = subgrid + (int64_t)j0[k] * lsize + (p * fa.Psub + of[k]) * 2;
                fr[k] = sg[0];
                fi[k] = sg[1];
            }
        }
        // loop order a2 > a1 > a0, as below
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            if (j0[k] >= j1[k]) continue;
            re += (double)fr[k];
            im += (double)fi[k];
            const T* sg = subgrid + (int64_t)(j0[k] + 1) * lsize + (p * fa.Psub + of[k]) * 2;
            for (int jj = j0[k] + 1; jj < j1[k]; ++jj, sg += lsize) {
                re += (double)sg[0];
                im += (double)sg[1];
            }
        }
        return make_double2(re, im);
    }
    for (int a2 = 0; a2 < n2; ++a2)
        for (int a1 = 0; a1 < n1; ++a1)
            for (int a0 = a0_first; a0 < n0; a0 += a0_step) {
                int64_t tile = cv[0][1 + 2 * a0];
                int64_t off = cv[0][2 + 2 * a0];
                if (D > 1) {
                    tile += fa.nt0 * cv[1][1 + 2 * a1];
                    off += fa.pe0 * cv[1][2 + 2 * a1];
                }
                if (D > 2) {
                    tile += fa.nt0 * fa.nt1 * cv[2][1 + 2 * a2];
                    off += fa.pe0 * fa.pe1 * cv[2][2 + 2 * a2];
                }
                const int j0 = fa.job_off[tile], j1 = fa.job_off[tile + 1];
                const T* sg = subgrid + (int64_t)j0 * lsize + (p * fa.Psub + off) * 2;
                for (int jj = j0; jj < j1; ++jj, sg += lsize) {
                    re += (double)sg[0];
                    im += (double)sg[1];
                }
            }
    return make_double2(re, im);
}

// The fine grid [pair][Mr^d] of the launch's pairs, one workgroup per
// (spreading tile, pair): thread = fine cell of the tile's interior (x
// fastest), its value the fold of the covering padded tiles' subgrids (the
// same sum as fold_at, in the same order).  The workgroup's cells share
// their covering tiles, so the cover and job lookups hit the caches and the
// subgrid reads of a wave are runs of consecutive cells.
template <int D, typename TS, typename T>
__global__ __launch_bounds__(512) void k_fold_grid(FoldArgs fa, int64_t nt0, int64_t nt1, int64_t ts0, int64_t ts1,
                                                   int64_t ts2, int64_t Mrtot, typename V2<T>::t* grid) {
    const int64_t b = blockIdx.x;
    const int p = blockIdx.y;
    const int64_t b0 = b % nt0, b1 = (b / nt0) % nt1, b2 = b / (nt0 * nt1);
    const int tid = threadIdx.x;
    const int lx = (int)(tid % ts0), ly = (int)((tid / ts0) % ts1), lz = (int)(tid / (ts0 * ts1));
    if (lz >= ts2) return;
    const int64_t c0 = b0 * ts0 + lx, c1 = b1 * ts1 + ly, c2 = b2 * ts2 + lz;
    if (c0 >= fa.Mr[0] || c1 >= fa.Mr[1] || c2 >= fa.Mr[2]) return;
    const int64_t cell = c0 + fa.Mr[0] * (c1 + fa.Mr[1] * c2);
    const double2 v = fold_at<D, TS>(fa, p, (unsigned)cell);
    typename V2<T>::t o;
    o.x = (T)v.x;
    o.y = (T)v.y;
    grid[(int64_t)p * Mrtot + cell] = o;
}

// The same when no fine cell is covered by more than two padded tiles in any
// dimension and no padded tile is wider than the period: the cell's covering
// tiles are its own tile and, per dimension, the previous one (periodically)
// where the cell lies in that tile's halo.
// The eight (neighbour, job range) pairs are the workgroup's, so the loop
// over them is uniform and each step is one coalesced subgrid load per lane.
// (Summation order: own tile first, then the neighbours, jobs ascending.)
template <typename TS, typename T>
__global__ __launch_bounds__(512) void k_fold_tiles(FoldArgs fa, int w, int64_t nt0, int64_t nt1, int64_t nt2,
                                                    int64_t ts0, int64_t ts1, int64_t ts2, int64_t Mrtot,
                                                    typename V2<T>::t* grid) {
    const int64_t b = blockIdx.x;
    const int p = blockIdx.y;
    const int64_t bt[3] = {b % nt0, (b / nt0) % nt1, b / (nt0 * nt1)};
    const int64_t nt[3] = {nt0, nt1, nt2}, ts[3] = {ts0, ts1, ts2};
    const int tid = threadIdx.x;
    const int64_t l[3] = {tid % ts0, (tid / ts0) % ts1, tid / (ts0 * ts1)};
    if (l[2] >= ts2) return;
    int64_t c[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) c[j] = bt[j] * ts[j] + l[j];
    if (c[0] >= fa.Mr[0] || c[1] >= fa.Mr[1] || c[2] >= fa.Mr[2]) return;
    const TS* sub = static_cast<const TS*>(fa.subgrid);
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        int64_t t[3], off[3];
        bool ok = true;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int oj = (o >> j) & 1;
            if (oj && nt[j] == 1) ok = false;   // the only tile: no other cover
            t[j] = bt[j] - oj;
            if (t[j] < 0) t[j] += nt[j];
            off[j] = c[j] - t[j] * ts[j];
            if (off[j] < 0) off[j] += fa.Mr[j];
            const int64_t interior = min(ts[j], fa.Mr[j] - t[j] * ts[j]);
            ok = ok && off[j] < interior + w - 1;
        }
        const int64_t tile = t[0] + nt0 * (t[1] + nt1 * t[2]);
        const int j0 = fa.job_off[tile], j1 = fa.job_off[tile + 1];
        if (!ok) continue;
        const int64_t cell = off[0] + fa.pe0 * (off[1] + fa.pe1 * off[2]);
        for (int job = j0; job < j1; ++job) {
            const TS* v = sub + (((int64_t)job * fa.np + p) * fa.Psub + cell) * 2;
            re += (double)v[0];
            im += (double)v[1];
        }
    }
    typename V2<T>::t out;
    out.x = (T)re;
    out.y = (T)im;
    grid[(int64_t)p * Mrtot + c[0] + fa.Mr[0] * (c[1] + fa.Mr[1] * c[2])] = out;
}

void launch_fold_grid(int prec, int tprec, const Geo& g, const FoldArgs& fa, int npairs, bool two_covers,
                      void* grid, hipStream_t s) {
    const dim3 nb((unsigned)g.n_tiles, (unsigned)npairs);
    const unsigned nt = (unsigned)(g.ts[0] * g.ts[1] * g.ts[2]);
    if (two_covers) {
#define FKR_FOLDT(TS, T) k_fold_tiles<TS, T><<<nb, nt, 0, s>>>(fa, g.w, g.nt[0], g.nt[1], g.nt[2], g.ts[0], g.ts[1], \
                                                               g.ts[2], g.Mrtot, static_cast<typename V2<T>::t*>(grid))
        if (tprec == FKR_F64) {
            if (prec == FKR_F64) FKR_FOLDT(double, double); else FKR_FOLDT(float, double);
        } else {
            FKR_FOLDT(float, float);
        }
#undef FKR_FOLDT
        return;
    }
#define FKR_FOLDG(TS, T) k_fold_grid<3, TS, T><<<nb, nt, 0, s>>>(fa, g.nt[0], g.nt[1], g.ts[0], g.ts[1], g.ts[2], \
                                                                 g.Mrtot, static_cast<typename V2<T>::t*>(grid))
    if (tprec == FKR_F64) {
        if (prec == FKR_F64) FKR_FOLDG(double, double); else FKR_FOLDG(float, double);
    } else {
        FKR_FOLDG(float, float);
    }
#undef FKR_FOLDG
}

// One radix-RAD Stockham stage (Govindaraju et al., SC'08 formulation):
// butterfly j reads a[j + q F/RAD], twiddles by W_F^(q k F/(Ns RAD)) with
// k = j mod Ns, and writes b[(j/Ns) Ns RAD + k + q Ns].
template <typename T, bool INV, int RAD>
__device__ __forceinline__ void stockham_stage(const typename V2<T>::t* a, typename V2<T>::t* b,
                                               int F, int Ns, int t, int tpr, const double2* tw) {
    using C = typename V2<T>::t;
    const int sgn = INV ? 1 : -1;
    const int nb = F / RAD;
    const int tws = F / (Ns * RAD);
    // j / Ns through a float reciprocal (exact after one correction: j < 2^24)
    const float rns = 1.0f / (float)Ns;
    for (int j = t; j < nb; j += tpr) {
        int jq = (int)((float)j * rns);
        jq -= jq * Ns > j ? 1 : 0;
        jq += (jq + 1) * Ns <= j ? 1 : 0;
        const int k = j - jq * Ns;
        C v[RAD];
#pragma unroll
        for (int q = 0; q < RAD; ++q) v[q] = a[j + q * nb];
        if (Ns > 1) {
#pragma unroll
            for (int q = 1; q < RAD; ++q) {
                const double2 w = tw[q * k * tws];
                C c;
                c.x = (T)w.x;
                c.y = (T)(INV ? -w.y : w.y);
                v[q] = cmul(v[q], c);
            }
        }
        C y[RAD];
        if (RAD == 2) {
            y[0] = cadd(v[0], v[1]);
            y[1] = csub(v[0], v[1]);
        } else if (RAD == 4) {
            const C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
            const C t2 = cadd(v[1], v[3]), t3 = cmuli(csub(v[1], v[3]), sgn);
            y[0] = cadd(t0, t2);
            y[2] = csub(t0, t2);
            y[1] = cadd(t1, t3);
            y[3] = csub(t1, t3);
        } else if (RAD == 3) {
            const T c3 = (T)0.86602540378443864676;
            const C tt = cadd(v[1], v[2]);
            const C u = cmuli(cscale(csub(v[1], v[2]), c3), sgn);
            const C m = csub(v[0], cscale(tt, (T)0.5));
            y[0] = cadd(v[0], tt);
            y[1] = cadd(m, u);
            y[2] = csub(m, u);
        } else {
            const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
            const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
            const C a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[3]);
            const C b1 = csub(v[1], v[4]), b2 = csub(v[2], v[3]);
            y[0] = cadd(v[0], cadd(a1, a2));
            const C r1 = cadd(v[0], cadd(cscale(a1, c1), cscale(a2, c2)));
            const C r2 = cadd(v[0], cadd(cscale(a1, c2), cscale(a2, c1)));
            const C i1 = cmuli(cadd(cscale(b1, s1), cscale(b2, s2)), sgn);
            const C i2 = cmuli(csub(cscale(b1, s2), cscale(b2, s1)), sgn);
            y[1] = cadd(r1, i1);
            y[4] = csub(r1, i1);
            y[2] = cadd(r2, i2);
            y[3] = csub(r2, i2);
        }
        const int base = jq * Ns * RAD + k;
#pragma unroll
        for (int q = 0; q < RAD; ++q) b[base + q * Ns] = y[q];
    }
}

// The Stockham stages of a workgroup's nr rows (R rows of F elements in
// buf0, the other buffer as scratch); returns the buffer holding the result.
template <typename T, bool INV>
__device__ __forceinline__ const typename V2<T>::t* fft_stages(typename V2<T>::t* buf0, typename V2<T>::t* buf1,
                                                               const FftPass& f, int nr, int tpr, int rl, int t,
                                                               const double2* twl) {
    using C = typename V2<T>::t;
    const int F = (int)f.F;
    C* src = buf0;
    C* dst = buf1;
    int Ns = 1;
    for (int s = 0; s < f.nfac; ++s) {
        const int rad = f.fac[s];
        if (rl < nr) {
            const C* a = src + (int64_t)rl * F;
            C* b = dst + (int64_t)rl * F;
            switch (rad) {
                case 4: stockham_stage<T, INV, 4>(a, b, F, Ns, t, tpr, twl); break;
                case 2: stockham_stage<T, INV, 2>(a, b, F, Ns, t, tpr, twl); break;
                case 3: stockham_stage<T, INV, 3>(a, b, F, Ns, t, tpr, twl); break;
                default: stockham_stage<T, INV, 5>(a, b, F, Ns, t, tpr, twl); break;
            }
        }
        __syncthreads();
        C* tmp = src; src = dst; dst = tmp;
        Ns *= rad;
    }
    return src;
}

// Store the transformed rows row0 .. row0 + nr - 1 (outputs 0 .. n_out - 1,
// or the band modes) through the output row map; rows below `skip` are kept.
template <typename T>
__device__ __forceinline__ void fft_store(const typename V2<T>::t* src, typename V2<T>::t* out, const FftPass& f,
                                          int64_t row0, int nr, int64_t skip) {
    using C = typename V2<T>::t;
    const int F = (int)f.F;
    const int nout = (int)f.n_out;
    const int kout = (int)(f.K % F);
    const unsigned rdiv = (unsigned)f.out_rdiv;
    // contiguous output rows: consecutive threads take consecutive elements
    // of a row; strided rows: consecutive rows of one element
    const bool efast = f.out_estride == 1;
    for (int q = threadIdx.x; q < nout * nr; q += blockDim.x) {
        int e, r;
        if (efast) {
            r = (int)((unsigned)q / (unsigned)nout);
            e = q - r * nout;
        } else {
            e = (int)((unsigned)q / (unsigned)nr);
            r = q - e * nr;
        }
        int pos = e;
        if (f.out_band) {   // mode e - K at (e - K) mod F (a band wider than F wraps)
            pos = e - kout;
            pos = pos < 0 ? pos + F : (pos >= F ? pos % F : pos);
        }
        if (row0 + r < skip) continue;
        C v = src[r * F + pos];
        if (f.fac_out) v = cscale(v, (T)f.fac_out[e]);
        const unsigned row = (unsigned)(row0 + r);
        const unsigned rq = row / rdiv;
        out[(int64_t)e * f.out_estride + f.out_roff + (int64_t)rq * f.out_rmul + (row - rq * rdiv)] = v;
    }
}

// LDS of a transform workgroup: two buffers of R rows of F elements, then
// the F twiddles (FP64 pairs, 16-byte aligned).
__host__ __device__ constexpr size_t fft_twiddle_offset(int R, int F, size_t csz) {
    return ((size_t)2 * R * F * csz + 15) & ~(size_t)15;
}
__host__ __device__ constexpr size_t fft_lds_bytes(int R, int F, size_t csz) {
    return fft_twiddle_offset(R, F, csz) + (size_t)F * 16;
}

// ---------------------------------------------------------------------------
// Stockham FFT along the contiguous axis of `rows` rows, in LDS.
// ---------------------------------------------------------------------------
template <typename T, bool INV, int FD = 0, typename TS = float>
__global__ __launch_bounds__(1024) void k_fft(const typename V2<T>::t* __restrict__ in,
                                              typename V2<T>::t* __restrict__ out, FftPass f) {
    using C = typename V2<T>::t;
    extern __shared__ unsigned char smem_raw[];
    const int R = f.rows_per_block;
    const int64_t row0 = (int64_t)blockIdx.x * R;
    const int nr = (int)min<int64_t>(R, f.rows - row0);
    // rows kept from an earlier call: a block that holds only such rows
    // returns, one that straddles the boundary neither loads nor stores them
    const int64_t skip = (f.skip_flag && *f.skip_flag) ? f.skip_rows : 0;
    if (row0 + nr <= skip) return;
    const int F = (int)f.F;
    C* buf0 = reinterpret_cast<C*>(smem_raw);
    C* buf1 = buf0 + (int64_t)R * F;
    // the F twiddles after the two row buffers (read by every stage)
    double2* twl = reinterpret_cast<double2*>(smem_raw + fft_twiddle_offset(R, F, sizeof(C)));
    for (int q = threadIdx.x; q < F; q += blockDim.x) twl[q] = reinterpret_cast<const double2*>(f.tw)[q];
    const int tpr = blockDim.x / R;
    const int rl = threadIdx.x / tpr, t = threadIdx.x % tpr;
    const int64_t n_in = f.n_in;
    if (f.in_band) {
        // Modes n = e - K, e < n_in, placed at n mod F; modes that coincide
        // modulo F (band wider than the transform) are summed, which is exact
        // for the values at the F output points.  The positions no mode
        // reaches are zero.
        // (32-bit index arithmetic: a block's rows hold well under 2^31 elements)
        const int kin = (int)(f.K % F), nin = (int)n_in;
        const int ns = min(nin, F);   // band slots; slot s takes modes s, s + F, ..
        if (ns < F) {
            for (int q = threadIdx.x; q < nr * F; q += blockDim.x) {
                buf0[q].x = 0;
                buf0[q].y = 0;
            }
            __syncthreads();
        }
        // strided rows: consecutive threads take consecutive rows (the
        // loads of one element of neighbouring rows are adjacent)
        const bool rfast = f.in_rdiv > 0 && f.in_estride != 1;
        for (int q = threadIdx.x; q < nr * ns; q += blockDim.x) {
            int r, sl;
            if (rfast) {
                sl = (int)((unsigned)q / (unsigned)nr);
                r = q - sl * nr;
            } else {
                r = (int)((unsigned)q / (unsigned)ns);
                sl = q - r * ns;
            }
            int pos = sl - kin;
            pos = pos < 0 ? pos + F : pos;
            C acc;
            acc.x = 0;
            acc.y = 0;
            if (row0 + r >= skip) {
                const int64_t row = row0 + r;
                const int64_t rq = row / f.in_rdiv;
                const C* rowp = in + rq * f.in_rmul + (row - rq * f.in_rdiv);
                for (int e = sl; e < nin; e += F) acc = cadd(acc, rowp[(int64_t)e * f.in_estride]);
            }
            buf0[r * F + pos] = acc;
        }
    } else if constexpr (FD > 0) {
        // fold the row from the subgrids (forward first pass, nin = F = Mr_0);
        // split: two threads per element, one per parity of the covering
        // tile index of dimension 0, the odd half added through buf1
        const int nin = (int)n_in;
        const unsigned rest = (unsigned)f.fold_rest;
        const int halves = f.fold_split ? 2 : 1;
        for (int q = threadIdx.x; q < halves * nr * nin; q += blockDim.x) {
            const int h = q >= nr * nin ? 1 : 0;
            const int qq = q - h * nr * nin;
            const int r = (int)((unsigned)qq / (unsigned)nin), e = qq - r * nin;
            const unsigned row = (unsigned)(row0 + r);
            const int p = (int)(row / rest);
            const unsigned cell = (row - (unsigned)p * rest) * (unsigned)nin + (unsigned)e;
            const double2 v = fold_at<FD, TS>(f.fold, p, cell, h, halves);
            C c;
            c.x = (T)v.x;
            c.y = (T)v.y;
            (h ? buf1 : buf0)[r * F + e] = c;
        }
        if (halves == 2) {
            __syncthreads();
            for (int q = threadIdx.x; q < nr * nin; q += blockDim.x) {
                const int r = (int)((unsigned)q / (unsigned)nin), e = q - r * nin;
                buf0[r * F + e] = cadd(buf0[r * F + e], buf1[r * F + e]);
            }
        }
    } else {
        const int nin = (int)n_in;
        const bool rfast = f.in_estride != 1;
        for (int q = threadIdx.x; q < nr * nin; q += blockDim.x) {
            int r, e;
            if (rfast) {
                e = (int)((unsigned)q / (unsigned)nr);
                r = q - e * nr;
            } else {
                r = (int)((unsigned)q / (unsigned)nin);
                e = q - r * nin;
            }
            const int64_t row = row0 + r;
            const int64_t rq = row / f.in_rdiv;
            buf0[r * F + e] = in[rq * f.in_rmul + (row - rq * f.in_rdiv) + (int64_t)e * f.in_estride];
        }
        // rows shorter than the transform are zero-padded
        for (int q = threadIdx.x; q < nr * (F - nin); q += blockDim.x) {
            const int r = (int)((unsigned)q / (unsigned)(F - nin));
            C z;
            z.x = 0;
            z.y = 0;
            buf0[r * F + nin + (q - r * (F - nin))] = z;
        }
    }
    __syncthreads();

    const C* src = fft_stages<T, INV>(buf0, buf1, f, nr, tpr, rl, t, twl);
    fft_store<T>(src, out, f, row0, nr, skip);
}

// ---------------------------------------------------------------------------
// Channel spectra from the pair spectra (Hermite form of the Gaussian's
// moment transforms): channel (r, a) at band index n is
// C_r(n) i^{|a|} prod_j He_{a_j}(u_j) exp(-u_j^2 / 2) / T_j with
// u_j = h_j 2 pi (e_j - K_j) / T_j; the division by h^a (equilibration) is
// implicit in using He_a(u) without the h^a factor.  C_r is unpacked from the
// pair spectra Z_p = C_{2p} + i C_{2p+1}, and channel pair c is
// X_{2c} + i X_{2c+1}.
// ---------------------------------------------------------------------------
// One thread per band index n: workgroup row blockIdx.y forms the channel
// pairs [y cpr, (y + 1) cpr) in weight order, reading each weight pair's
// spectra at n and at its mirror once (the pairs of one band index are
// adjacent); its moment multipliers (one exponential per dimension, the
// degrees by the Hermite recurrence) are kept in LDS.
constexpr int kExpandThreads = 128;
constexpr int kExpandDeg = 5;   // moment degrees per dimension (<= 2 l = 4)
template <typename T>
__global__ __launch_bounds__(kExpandThreads) void k_expand_n(ExpandArgs a, const int* es, const int* et,
                                                             const typename V2<T>::t* spec,
                                                             typename V2<T>::t* out, const long long* skip_flag,
                                                             int64_t c_keep) {
    __shared__ double mloc[3][kExpandDeg][kExpandThreads];
    const int tid = threadIdx.x;
    const int64_t n = (int64_t)blockIdx.x * kExpandThreads + tid;
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0 && a.ill_clear) *a.ill_clear = 0ull;
    if (n >= a.Btot) return;
    unsigned nn = 0, rem = (unsigned)n, stride = 1;
    for (int j = 0; j < a.d; ++j) {
        const unsigned bj = (unsigned)a.B[j];
        const unsigned qj = rem / bj;
        const int ej = (int)(rem - qj * bj);
        rem = qj;
        nn += (bj - 1 - (unsigned)ej) * stride;
        stride *= bj;
        // multiplier of degree k: He_k(u) exp(-u^2 / 2) / T_j, u = h_j 2 pi (e_j - K_j) / T_j;
        // its derivative in log h_j is u d/du of it, -u He_{k+1}(u) exp(-u^2 / 2) / T_j
        const double u = a.h[j] * (2.0 * M_PI * (double)(ej - a.K[j]) / a.T[j]);
        const double gj = exp(-0.5 * u * u) / a.T[j];
        double he[kExpandDeg + 1];
        he[0] = 1.0;
        he[1] = u;
#pragma unroll
        for (int k = 1; k < kExpandDeg; ++k) he[k + 1] = u * he[k] - k * he[k - 1];
        const bool dj = j == a.deriv_dim;
        if (a.ktab) {   // a compact kernel: the multipliers of its sampled moments
            int64_t off = 0;   // dimension j's table, or the derivative block after all d
            for (int i = 0; i < (dj ? a.d : j); ++i) off += a.kdeg * a.B[i];
#pragma unroll
            for (int k = 0; k < kExpandDeg; ++k) mloc[j][k][tid] = k < a.kdeg ? a.ktab[off + k * a.B[j] + ej] : 0.0;
            continue;
        }
#pragma unroll
        for (int k = 0; k < kExpandDeg; ++k) mloc[j][k][tid] = (dj ? -u * he[k + 1] : he[k]) * gj;
    }
    // the row's channel pairs [c_lo, c_hi) and the real weights they use,
    // r of channel ch: 0 for the s-channels, then n_t channels per weight
    const int c_lo = (int)blockIdx.y * a.cpr, c_hi = min(a.ncp, c_lo + a.cpr);
    auto weight_of = [&](int ch) { return ch < a.n_s ? 0 : 1 + (ch - a.n_s) / a.n_t; };
    // the channels run in weight order, so the thread keeps one pair's
    // spectra Z_p(n), Z_p(-n) in registers and reads each pair once
    int cur_p = -1;
    double2 zn = make_double2(0.0, 0.0), zm = make_double2(0.0, 0.0);
    const int c_first = (skip_flag && *skip_flag) ? (int)c_keep : 0;
    for (int c = max(c_lo, c_first); c < c_hi; ++c) {
        double acc_re = 0.0, acc_im = 0.0;
        for (int half = 0; half < 2; ++half) {
            const int ch = 2 * c + half;
            if (ch >= a.nreal) break;
            const int r = weight_of(ch);
            const int* ex = ch < a.n_s ? es + 3 * ch : et + 3 * ((ch - a.n_s) % a.n_t);
            double m = 1.0;
            int deg = 0;
            for (int j = 0; j < a.d; ++j) {
                m *= mloc[j][ex[j]][tid];
                deg += ex[j];
            }
            if ((r >> 1) != cur_p) {
                cur_p = r >> 1;
                const typename V2<T>::t a0 = spec[n * a.npairs + cur_p];
                const typename V2<T>::t a1 = spec[(int64_t)nn * a.npairs + cur_p];
                zn = make_double2((double)a0.x, (double)a0.y);
                zm = make_double2((double)a1.x, (double)a1.y);
            }
            // real weight spectrum C_r(n), r = 2 p + half, from Z_p(n) and Z_p(-n)
            const double2 cr = (r & 1) == 0 ? make_double2(0.5 * (zn.x + zm.x), 0.5 * (zn.y - zm.y))
                                            : make_double2(0.5 * (zn.y + zm.y), -0.5 * (zn.x - zm.x));
            double xr = cr.x * m, xi = cr.y * m;
            switch (deg & 3) {   // multiply by i^deg
                case 1: { const double t0 = xr; xr = -xi; xi = t0; break; }
                case 2: xr = -xr; xi = -xi; break;
                case 3: { const double t0 = xr; xr = xi; xi = -t0; break; }
                default: break;
            }
            if (half == 0) { acc_re += xr; acc_im += xi; }
            else { acc_re -= xi; acc_im += xr; }   // + i * X
        }
        typename V2<T>::t o;
        o.x = (T)acc_re;
        o.y = (T)acc_im;
        out[(int64_t)c * a.Btot + n] = o;
    }
}

// Channel spectra for a full bandwidth matrix: one thread per band index n;
// the multipliers of all s-channels by the multivariate Hermite recurrence
// into LDS, then every channel pair of the launch (t-channel b uses the
// s-channel of b; the weight spectra are unpacked from the pair spectra).
// DER: the derivative along fh.dH of every multiplier M_c = m_c G / sc_c
// (m_c the Hermite recurrence, G = exp(-w^T H w / 2) / prod T, sc_c the
// equilibration prod_k s_k^{a_k}, s_k = sqrt(H_kk)), by forward
// differentiation of the recurrence: dM_c = (G / sc_c) (dm_c - m_c
// (w^T dH w / 2 + sum_k a_k dH_kk / (2 H_kk))).
// The multipliers M_c of every s-channel at band index n into mf[c][tid]
// (DER: their derivatives along fh.dH); returns the band index of -n.
template <bool DER>
__device__ __forceinline__ unsigned full_multipliers(const ExpandArgs& a, const FullH& fh, const int* es, int64_t n,
                                                     int tid, double (*mf)[kExpandThreads],
                                                     double (*dmf)[kExpandThreads]) {
    unsigned nn = 0, rem = (unsigned)n, stride = 1;
    double w[3] = {0.0, 0.0, 0.0};
    double tprod = 1.0;
    for (int j = 0; j < a.d; ++j) {
        const unsigned bj = (unsigned)a.B[j];
        const unsigned qj = rem / bj;
        const int ej = (int)(rem - qj * bj);
        rem = qj;
        nn += (bj - 1 - (unsigned)ej) * stride;
        stride *= bj;
        w[j] = 2.0 * M_PI * (double)(ej - a.K[j]) / a.T[j];
        tprod *= a.T[j];
    }
    double z[3] = {0.0, 0.0, 0.0}, q = 0.0;
    for (int j = 0; j < a.d; ++j) {
        for (int k = 0; k < a.d; ++k) z[j] += fh.H[3 * j + k] * w[k];
        q += w[j] * z[j];
    }
    const double G = exp(-0.5 * q) / tprod;
    double dz[3] = {0.0, 0.0, 0.0}, dq = 0.0;
    if constexpr (DER) {
        for (int j = 0; j < a.d; ++j) {
            for (int k = 0; k < a.d; ++k) dz[j] += fh.dH[3 * j + k] * w[k];
            dq += w[j] * dz[j];
        }
        dmf[0][tid] = 0.0;
    }
    mf[0][tid] = 1.0;
    for (int c = 1; c < a.n_s; ++c) {
        const int j = fh.rj[c];
        double v = z[j] * mf[fh.rb[c]][tid];
        double dv = 0.0;
        if constexpr (DER) dv = dz[j] * mf[fh.rb[c]][tid] + z[j] * dmf[fh.rb[c]][tid];
        for (int k = 0; k < a.d; ++k) {
            const int bk = fh.rbk[c][k];
            if (bk >= 0) {
                const double bkk = (double)es[3 * fh.rb[c] + k];
                v -= bkk * fh.H[3 * j + k] * mf[bk][tid];
                if constexpr (DER) dv -= bkk * (fh.dH[3 * j + k] * mf[bk][tid] + fh.H[3 * j + k] * dmf[bk][tid]);
            }
        }
        mf[c][tid] = v;
        if constexpr (DER) dmf[c][tid] = dv;
    }
    for (int c = 0; c < a.n_s; ++c) {
        double sc = 1.0, dls = 0.0;   // dls: d log(sc) along dH
        for (int k = 0; k < a.d; ++k)
            for (int e = 0; e < es[3 * c + k]; ++e) {
                sc *= fh.s[k];
                if constexpr (DER) dls += 0.5 * fh.dH[4 * k] / fh.H[4 * k];
            }
        if constexpr (DER)
            mf[c][tid] = G / sc * (dmf[c][tid] - mf[c][tid] * (0.5 * dq + dls));
        else
            mf[c][tid] *= G / sc;
    }
    return nn;
}

template <typename T, bool DER>
__global__ __launch_bounds__(kExpandThreads) void k_expand_full(ExpandArgs a, FullH fh, const int* es,
                                                                const int* pidx, const typename V2<T>::t* spec,
                                                                typename V2<T>::t* out) {
    __shared__ double mf[kMaxChannels][kExpandThreads];
    __shared__ double dmf[DER ? kMaxChannels : 1][kExpandThreads];
    const int tid = threadIdx.x;
    const int64_t n = (int64_t)blockIdx.x * kExpandThreads + tid;
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0 && a.ill_clear) *a.ill_clear = 0ull;
    if (n >= a.Btot) return;
    const unsigned nn = full_multipliers<DER>(a, fh, es, n, tid, mf, dmf);
    for (int c = (int)blockIdx.y; c < a.ncp; c += (int)gridDim.y) {
        double acc_re = 0.0, acc_im = 0.0;
        for (int half = 0; half < 2; ++half) {
            const int ch = 2 * c + half;
            if (ch >= a.nreal) break;
            int r, si;
            if (ch < a.n_s) { r = 0; si = ch; }
            else { r = 1 + (ch - a.n_s) / a.n_t; si = pidx[((ch - a.n_s) % a.n_t) * kMaxP]; }
            int deg = 0;
            for (int k = 0; k < a.d; ++k) deg += es[3 * si + k];
            const typename V2<T>::t zn = spec[n * a.npairs + (r >> 1)];
            const typename V2<T>::t zm = spec[(int64_t)nn * a.npairs + (r >> 1)];
            double cr, ci;
            if ((r & 1) == 0) { cr = 0.5 * ((double)zn.x + (double)zm.x); ci = 0.5 * ((double)zn.y - (double)zm.y); }
            else { cr = 0.5 * ((double)zn.y + (double)zm.y); ci = -0.5 * ((double)zn.x - (double)zm.x); }
            const double m = mf[si][tid];
            double xr = cr * m, xi = ci * m;
            switch (deg & 3) {   // multiply by i^deg
                case 1: { const double t0 = xr; xr = -xi; xi = t0; break; }
                case 2: xr = -xr; xi = -xi; break;
                case 3: { const double t0 = xr; xr = xi; xi = -t0; break; }
                default: break;
            }
            if (half == 0) { acc_re += xr; acc_im += xi; }
            else { acc_re -= xi; acc_im += xr; }
        }
        typename V2<T>::t o;
        o.x = (T)acc_re;
        o.y = (T)acc_im;
        out[(int64_t)c * a.Btot + n] = o;
    }
}

// Moment multipliers of a compact kernel sampled at the grid offsets (the
// discrete convolution of eq. 12-13 in the frequency domain): per dimension
// j, degree a and band index e, with w = 2 pi (e - K_j) / T_j,
// Re(i^a D(w)) / T_j, D(w) = delta sum_m (m delta / h)^a K(m delta / h) / h
// exp(-i w m delta) over the offsets inside the support (the same phase
// convention as the Gaussian's He_a(u) exp(-u^2/2) / T_j).  With every mode
// |n| <= L/2 kept, each sample contributes the trigonometric interpolant of
// the sampled moment kernel, exact at the grid offsets.  square: K^2 in
// place of K (the squared kernel of the variance of the fit, eq. 27, up to
// prod_j 1 / h_j).
__device__ __forceinline__ double compact_kernel(int kind, double u) {
    const double a = fabs(u);
    if (a > 1.0) return 0.0;
    const double q = 1.0 - u * u;
    switch (kind) {
        case FKR_REG_BOX: return 0.5;
        case FKR_REG_TRIANGLE: return 1.0 - a;
        case FKR_REG_EPANECHNIKOV: return 0.75 * q;
        case FKR_REG_BIWEIGHT: return 0.9375 * q * q;
        default: return 1.09375 * q * q * q;
    }
}

// u K'(u) of the compact kernels (the box's is zero inside the support; the
// sampled box kernel changes only by steps, where a grid offset crosses
// |u| = 1, which a derivative in h does not see)
__device__ __forceinline__ double compact_kernel_udu(int kind, double u) {
    if (fabs(u) > 1.0) return 0.0;
    const double q = 1.0 - u * u;
    switch (kind) {
        case FKR_REG_BOX: return 0.0;
        case FKR_REG_TRIANGLE: return -fabs(u);
        case FKR_REG_EPANECHNIKOV: return -1.5 * u * u;
        case FKR_REG_BIWEIGHT: return -3.75 * u * u * q;
        default: return -6.5625 * u * u * q * q;
    }
}

// Tables per dimension [d][kdeg][B_j]; with a.deriv_dim >= 0 one more block
// [kdeg][B_j] for that dimension holds the derivative in log h_j of the
// sampled moment kernel, d/dlog h (K(u/h) / h (u/h)^a) =
// -((1 + a) K(v) + v K'(v)) v^a / h with v = u / h.
__global__ __launch_bounds__(256) void k_ktab(ExpandArgs a, double d0, double d1, double d2, int kind, int square,
                                              double* tab) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t off = 0, rem = id;
    int j = 0;
    for (; j < a.d; ++j) {
        const int64_t nj = (int64_t)a.kdeg * a.B[j];
        if (rem < nj) break;
        rem -= nj;
        off += nj;
    }
    bool deriv = false;
    if (j >= a.d) {   // the derivative block
        if (a.deriv_dim < 0 || rem >= (int64_t)a.kdeg * a.B[a.deriv_dim]) return;
        j = a.deriv_dim;
        deriv = true;
    }
    const int deg = (int)(rem / a.B[j]);
    const int64_t e = rem - (int64_t)deg * a.B[j];
    const double delta = j == 0 ? d0 : (j == 1 ? d1 : d2);
    const double h = a.h[j];
    const double w = 2.0 * M_PI * (double)(e - a.K[j]) / a.T[j];
    const int64_t mmax = (int64_t)floor(h / delta);
    double re = 0.0, im = 0.0;
    for (int64_t m = -mmax; m <= mmax; ++m) {
        const double u = (double)m * delta / h;
        const double kv = compact_kernel(kind, u);
        double v = (square ? kv * kv : kv) / h * delta;
        if (deriv) v = -((1.0 + deg) * kv + compact_kernel_udu(kind, u)) / h * delta;
        for (int k = 0; k < deg; ++k) v *= u;
        double sn, cs;
        sincos(w * (double)m * delta, &sn, &cs);
        re += v * cs;
        im -= v * sn;
    }
    // i^deg (re + i im), real part
    double r;
    switch (deg & 3) {
        case 0: r = re; break;
        case 1: r = -im; break;
        case 2: r = -re; break;
        default: r = im; break;
    }
    // even L: the modes +-L/2 alias to one Nyquist term, each carries half
    const int64_t Lj = llround(a.T[j] / delta);
    if (2 * llabs(e - a.K[j]) == Lj) r *= 0.5;
    tab[off + rem] = r / a.T[j];
}

void launch_ktab(const ExpandArgs& a, const double* delta, int reg_kernel, int square, double* ktab, hipStream_t s) {
    int64_t n = 0;
    for (int j = 0; j < a.d; ++j) n += (int64_t)a.kdeg * a.B[j];
    if (a.deriv_dim >= 0) n += (int64_t)a.kdeg * a.B[a.deriv_dim];
    k_ktab<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, delta[0], a.d > 1 ? delta[1] : 1.0, a.d > 2 ? delta[2] : 1.0,
                                                      reg_kernel, square, ktab);
}

void launch_expand_full(int prec, const ExpandArgs& a, const FullH& fh, const int* es, const int* pidx,
                        const void* spec, void* out, hipStream_t s) {
    const dim3 nbn((unsigned)((a.Btot + kExpandThreads - 1) / kExpandThreads),
                   (unsigned)std::min(4, std::max(1, a.ncp)));
#define FKR_EXF(T, D) k_expand_full<T, D><<<nbn, kExpandThreads, 0, s>>>(a, fh, es, pidx, \
        static_cast<const typename V2<T>::t*>(spec), static_cast<typename V2<T>::t*>(out))
    if (prec == FKR_F64) {
        if (fh.deriv) FKR_EXF(double, true); else FKR_EXF(double, false);
    } else {
        if (fh.deriv) FKR_EXF(float, true); else FKR_EXF(float, false);
    }
#undef FKR_EXF
}

void launch_expand(int prec, const ExpandArgs& a, const int* es, const int* et, const void* spec, void* out,
                   const long long* skip_flag, int64_t c_keep, hipStream_t s) {
    // workgroup rows of contiguous channel pairs: at least four (more waves
    // for few band indices), at most eight pairs each
    ExpandArgs b = a;
    const int ncp = std::max(1, a.ncp);
    int rows = std::max(std::min(4, ncp), (ncp + 7) / 8);
    b.cpr = (ncp + rows - 1) / rows;
    rows = (ncp + b.cpr - 1) / b.cpr;
    const dim3 nbn((unsigned)((a.Btot + kExpandThreads - 1) / kExpandThreads), (unsigned)std::max(1, rows));
    if (prec == FKR_F64)
        k_expand_n<double><<<nbn, kExpandThreads, 0, s>>>(b, es, et, static_cast<const double2*>(spec),
                                                          static_cast<double2*>(out), skip_flag, c_keep);
    else
        k_expand_n<float><<<nbn, kExpandThreads, 0, s>>>(b, es, et, static_cast<const float2*>(spec),
                                                         static_cast<float2*>(out), skip_flag, c_keep);
}


// ---------------------------------------------------------------------------
// Per-grid-point solve (eq. 3 / 11) in FP64.
// ---------------------------------------------------------------------------
// Workgroup row blockIdx.y takes the weights 1 + y wpg .. of every point
// (each row factors the point's matrix itself), so a call with many weight
// vectors runs several threads per grid point.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_solve(SolveArgs a, const int* pidx, const T* chan) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.Mtot) return;
    const int grp = blockIdx.y;
    const int r_beg = 1 + grp * a.wpg, r_end = min(a.nr, r_beg + a.wpg);
    // channels are stored pair-major, [pair][M][re, im]: real channel r of
    // point k is chan[((r / 2) M + k) 2 + r % 2] (coalesced over k)
    auto ch = [&](int r) { return chan[(((int64_t)(r >> 1)) * a.Mtot + k) * 2 + (r & 1)]; };
    double A[P][P];
#pragma unroll
    for (int b = 0; b < P; ++b)
#pragma unroll
        for (int c = 0; c <= b; ++c) A[b][c] = (double)ch(pidx[b * kMaxP + c]);
    const double s0 = (double)ch(0);
    // s_0 is the first pivot; every pivot must clear the floors (ill-posed
    // otherwise) and, for the point to be resolved, resolve A_cc.
    bool ill = !isfinite(s0);
    bool unres = false;
    // Cholesky A = L L^T (lower triangle in place).
    double diag0[P];
#pragma unroll
    for (int b = 0; b < P; ++b) diag0[b] = A[b][b];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        double v = A[c][c];
#pragma unroll
        for (int q = 0; q < c; ++q) v -= A[c][q] * A[c][q];
        if (!(v > fmax(a.rel_floor * diag0[c], a.abs_floor))) ill = true;
        if (!(v > a.resolve * diag0[c])) unres = true;
        const double l = sqrt(fmax(v, 1e-300));
        A[c][c] = l;
        const double il = 1.0 / l;
#pragma unroll
        for (int b = c + 1; b < P; ++b) {
            double u = A[b][c];
#pragma unroll
            for (int q = 0; q < c; ++q) u -= A[b][q] * A[c][q];
            A[b][c] = u * il;
        }
    }
    // r0 = A^{-1} e_0 (row 0 of the symmetric inverse).
    double y[P], r0[P];
#pragma unroll
    for (int b = 0; b < P; ++b) {
        double v = b == 0 ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < b; ++q) v -= A[b][q] * y[q];
        y[b] = v / A[b][b];
    }
#pragma unroll
    for (int b = P - 1; b >= 0; --b) {
        double v = y[b];
#pragma unroll
        for (int q = b + 1; q < P; ++q) v -= A[q][b] * r0[q];
        r0[b] = v / A[b][b];
    }
    const double nan = __builtin_nan("");
    unres = unres || ill;
    if (grp == 0) {
        if (a.s0_out) a.s0_out[k] = s0;
        if (a.r0_out) {
#pragma unroll
            for (int b = 0; b < P; ++b) a.r0_out[b * a.Mtot + k] = ill ? nan : r0[b];
        }
        if (a.sup_out) a.sup_out[k] = unres ? __builtin_nanf("") : 0.f;
        if (ill && a.ill_count) atomicAdd(a.ill_count, 1ull);
    }
    // the caller's fits are NaN where ill-posed; the internal rows that feed
    // the DF / RSS sums are NaN wherever the point is not resolved
    for (int r = r_beg; r < r_end; ++r) {
        const int t0 = a.n_s + (r - 1) * a.n_t;
        double m = 0.0;
#pragma unroll
        for (int b = 0; b < P; ++b) m += r0[b] * (double)ch(t0 + b);
        if (ill) m = nan;
        const double mr = unres ? nan : m;
        if (r <= a.ny) {
            if (a.y_out) {
                const int cpl = a.y_cplx ? 2 : 1;
                const int col = (r - 1) / cpl, part = (r - 1) % cpl;
                a.y_out[(col * a.Mtot + k) * cpl + part] = m;
            }
            if (a.rows_with_y && a.probe_out) static_cast<float*>(a.probe_out)[k * a.probe_stride + (r - 1)] = (float)mr;
        } else if (a.probe_out) {
            const int64_t o = k * a.probe_stride + (r - 1 - (a.rows_with_y ? 0 : a.ny));
            if (a.probe_f32) static_cast<float*>(a.probe_out)[o] = (float)mr;
            else static_cast<double*>(a.probe_out)[o] = mr;
        }
    }
}

// Derivatives of the fits in log h_j, one grid point per thread (resolved
// points only): the Cholesky factor of the equilibrated matrix A at h, then
// for every weight m = A^{-1} t and d m_hat = e_0^T A^{-1} (dt - dA m), the
// channels dA, dt being those of the derivative multipliers.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_dsolve(DSolveArgs a, const int* pidx, const T* cb, const T* cd) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.Mtot) return;
    const double nan = __builtin_nan("");
    if (!(a.sup[k] == 0.f)) {
        for (int r = 1; r < a.nr; ++r) a.out[(r - 1) * a.Mtot + k] = nan;
        return;
    }
    auto chb = [&](int r) { return (double)cb[(((int64_t)(r >> 1)) * a.Mtot + k) * 2 + (r & 1)]; };
    auto chd = [&](int r) { return (double)cd[(((int64_t)(r >> 1)) * a.Mtot + k) * 2 + (r & 1)]; };
    double L[P][P], dA[P][P];
#pragma unroll
    for (int b = 0; b < P; ++b)
#pragma unroll
        for (int c = 0; c <= b; ++c) {
            const int sidx = pidx[b * kMaxP + c];
            L[b][c] = chb(sidx);
            dA[b][c] = chd(sidx);
            dA[c][b] = dA[b][c];
        }
#pragma unroll
    for (int c = 0; c < P; ++c) {
        double v = L[c][c];
#pragma unroll
        for (int q = 0; q < c; ++q) v -= L[c][q] * L[c][q];
        L[c][c] = sqrt(fmax(v, 1e-300));
#pragma unroll
        for (int b = c + 1; b < P; ++b) {
            double u = L[b][c];
#pragma unroll
            for (int q = 0; q < c; ++q) u -= L[b][q] * L[c][q];
            L[b][c] = u / L[c][c];
        }
    }
    // x = A^{-1} v by the two triangular solves
    auto solve = [&](double (&v)[P]) {
#pragma unroll
        for (int b = 0; b < P; ++b) {
#pragma unroll
            for (int q = 0; q < b; ++q) v[b] -= L[b][q] * v[q];
            v[b] /= L[b][b];
        }
#pragma unroll
        for (int b = P - 1; b >= 0; --b) {
#pragma unroll
            for (int q = b + 1; q < P; ++q) v[b] -= L[q][b] * v[q];
            v[b] /= L[b][b];
        }
    };
    double c0[P];
#pragma unroll
    for (int b = 0; b < P; ++b) c0[b] = b == 0 ? 1.0 : 0.0;
    solve(c0);
    for (int r = 1; r < a.nr; ++r) {
        const int t0 = a.n_s + (r - 1) * a.n_t;
        double m[P];
#pragma unroll
        for (int b = 0; b < P; ++b) m[b] = chb(t0 + b);
        solve(m);
        double dm = 0.0;
#pragma unroll
        for (int b = 0; b < P; ++b) {
            double v = chd(t0 + b);
#pragma unroll
            for (int c = 0; c < P; ++c) v -= dA[b][c] * m[c];
            dm += c0[b] * v;
        }
        a.out[(r - 1) * a.Mtot + k] = dm;
    }
}

// Variance of the fit and its confidence band (eq. 27-28), one grid point per
// thread: Sigma = scale r0^T Q r0 with Q_bc the s-channel of b + c of the
// sigma^2-weighted samples under the squared kernel, brought to the
// equilibration of r0; the band is m_hat -/+ z sqrt(max(Sigma, 0)).
template <int P, typename T>
__global__ __launch_bounds__(256) void k_interval(IntervalArgs a, const T* chan) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.Mtot) return;
    auto ch = [&](int r) { return (double)chan[(((int64_t)(r >> 1)) * a.Mtot + k) * 2 + (r & 1)]; };
    double r0[P];
#pragma unroll
    for (int b = 0; b < P; ++b) r0[b] = a.r0[b * a.Mtot + k];
    double v = 0.0;
#pragma unroll
    for (int b = 0; b < P; ++b) {
        double row = 0.0;
#pragma unroll
        for (int c = 0; c < P; ++c) row += a.fac[b * kMaxP + c] * ch(a.sidx[b * kMaxP + c]) * r0[c];
        v += r0[b] * row;
    }
    const double sig = a.scale * v;
    a.sigma[k] = sig;
    if (a.lower || a.upper) {
        const double m = a.mhat[k];
        const double half = a.z * sqrt(fmax(sig, 0.0));
        if (a.lower) a.lower[k] = m - half;
        if (a.upper) a.upper[k] = m + half;
    }
}

// ---------------------------------------------------------------------------
// Multilinear interpolation helpers
// ---------------------------------------------------------------------------
template <int D>
struct Corners {
    int64_t idx[1 << D];
    double w[1 << D];
};

template <int D>
__device__ __forceinline__ Corners<D> corners(const Geo& g, int x_type, const void* X, int64_t i) {
    int64_t cell[3];
    double fr[3];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double x = load_as_double(X, x_type, i * D + j);
        const double t = (x - g.lo[j]) * g.inv_delta[j];
        double fl = floor(t);
        fl = fmin(fmax(fl, 0.0), (double)(g.M[j] - 2));
        cell[j] = (int64_t)fl;
        fr[j] = t - fl;
    }
    Corners<D> c;
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) {
        double w = 1.0;
        int64_t id = 0, stride = 1;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int bit = (q >> j) & 1;
            w *= bit ? fr[j] : 1.0 - fr[j];
            id += (cell[j] + bit) * stride;
            stride *= g.M[j];
        }
        c.idx[q] = id;
        c.w[q] = w;
    }
    return c;
}

template <int D>
__global__ __launch_bounds__(256) void k_interp(Geo g, int nv, const double* G, int64_t Nq,
                                                const void* X, int x_type, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nq) return;
    const Corners<D> c = corners<D>(g, x_type, X, i);
    for (int v = 0; v < nv; ++v) {
        const double* gv = G + (int64_t)v * g.Mtot;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) s += c.w[q] * gv[c.idx[q]];
        out[(int64_t)v * Nq + i] = s;
    }
}

// ---------------------------------------------------------------------------
// Prediction by tensor-product cubic spline (the 'spline' interpolation with
// 'linear' extrapolation of Table 1's y_grid_opt).  Along one dimension the
// not-a-knot spline through f_0 .. f_{n-1} (unit node spacing) is fixed by
// its second derivatives m_k: C^2 continuity gives
// m_{k-1} + 4 m_k + m_{k+1} = r_k = 6 (f_{k-1} - 2 f_k + f_{k+1}), and the
// not-a-knot ends (third derivative continuous at nodes 1 and n-2) turn the
// equations at k = 1 and k = n-2 into 6 m_1 = r_1 and 6 m_{n-2} = r_{n-2};
// the rest is a (1, 4, 1) tridiagonal system for m_2 .. m_{n-3}, and
// m_0 = 2 m_1 - m_2, m_{n-1} = 2 m_{n-2} - m_{n-3}.  Three nodes give the
// parabola (m constant), two the line (m = 0).  In d dimensions the spline
// value on a cell needs, at its 2^d corners, every mixed derivative
// d^2|S| / prod_{j in S} dx_j^2 for S a subset of the dimensions: array S of
// the coefficient block is array S minus dimension j differentiated along j.
// ---------------------------------------------------------------------------
constexpr int kSplineCp = 32;   // forward-sweep factors kept; later ones equal the limit 2 - sqrt 3 in FP64

__global__ __launch_bounds__(256) void k_copy_f64(const double* in, double* out, int64_t n, int64_t in_stride,
                                                  int64_t out_stride, int nv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nv) return;
    const int64_t v = i / n, k = i - v * n;
    out[v * out_stride + k] = in[v * in_stride + k];
}

// One thread per grid line along dimension j: lines of array S (S without
// bit j) of every grid function go to array S | (1 << j).
__global__ __launch_bounds__(256) void k_spline_line(double* coef, int64_t Mtot, int d, int j, int64_t n,
                                                     int64_t st, int64_t nlines, int nv) {
    __shared__ double cp[kSplineCp];
    if (threadIdx.x < kSplineCp) {
        // Thomas factors of the (1, 4, 1) system: c_0 = 1/4, c_u = 1 / (4 - c_{u-1})
        double c = 0.25;
        for (int u = 1; u <= (int)threadIdx.x; ++u) c = 1.0 / (4.0 - c);
        cp[threadIdx.x] = c;
    }
    __syncthreads();
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nsub = (int64_t)1 << j;
    if (id >= nlines * nsub * nv) return;
    const int64_t a = id / nlines, l = id - a * nlines;
    const int64_t v = a >> j, S = a & (nsub - 1);
    const int64_t o = l / st, r = l - o * st;
    const int64_t base = o * n * st + r;
    const double* f = coef + ((v << d) + S) * Mtot + base;
    double* m = coef + ((v << d) + (S | nsub)) * Mtot + base;
    if (n <= 2) {
        for (int64_t k = 0; k < n; ++k) m[k * st] = 0.0;
        return;
    }
    if (n == 3) {
        const double c = f[0] - 2.0 * f[st] + f[2 * st];
        m[0] = c; m[st] = c; m[2 * st] = c;
        return;
    }
    const double m1 = f[0] - 2.0 * f[st] + f[2 * st];
    const double mL = f[(n - 3) * st] - 2.0 * f[(n - 2) * st] + f[(n - 1) * st];
    const int64_t nu = n - 4;   // unknowns m_2 .. m_{n-3}
    double fa = f[st], fb = f[2 * st], dp = 0.0;
    for (int64_t u = 0; u < nu; ++u) {
        const int64_t k = u + 2;
        const double fc = f[(k + 1) * st];
        double rhs = 6.0 * (fa - 2.0 * fb + fc);
        if (k == 2) rhs -= m1;
        if (k == n - 3) rhs -= mL;
        dp = (rhs - dp) * cp[u < kSplineCp ? u : kSplineCp - 1];
        m[k * st] = dp;
        fa = fb; fb = fc;
    }
    double nx = 0.0;
    for (int64_t u = nu - 1; u >= 0; --u) {
        const int64_t k = u + 2;
        const double x = m[k * st] - (u == nu - 1 ? 0.0 : cp[u < kSplineCp ? u : kSplineCp - 1] * nx);
        m[k * st] = x;
        nx = x;
    }
    const double m2 = n >= 5 ? m[2 * st] : mL;
    const double mN3 = n >= 5 ? m[(n - 3) * st] : m1;
    m[st] = m1;
    m[(n - 2) * st] = mL;
    m[0] = 2.0 * m1 - m2;
    m[(n - 1) * st] = 2.0 * mL - mN3;
}

// Spline value at each query point: per dimension the cell k (clamped to
// [0, M - 2]) and offset u; weights (1 - u, u) on the corner values and, on
// the second derivatives, ((1-u)^3 - (1-u)) / 6, (u^3 - u) / 6 inside the box,
// or the end tangent's (-u/3, -u/6) below it and (v/6, v/3), v = u - 1, above.
template <int D>
__global__ __launch_bounds__(256) void k_spline_eval(Geo g, int nv, const double* coef, int64_t Nq, const void* X,
                                                     int x_type, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nq) return;
    double aw[D][2], cw[D][2];
    int64_t base = 0, off[D], stride = 1;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double t = (load_as_double(X, x_type, i * D + j) - g.lo[j]) * g.inv_delta[j];
        bad |= !isfinite(t);
        const double top = (double)(g.M[j] - 2);
        const double kf = isfinite(t) ? fmin(fmax(floor(t), 0.0), top) : 0.0;
        const double u = isfinite(t) ? t - kf : 0.0;
        aw[j][0] = 1.0 - u;
        aw[j][1] = u;
        if (t < 0.0) {
            cw[j][0] = -u / 3.0; cw[j][1] = -u / 6.0;
        } else if (t > top + 1.0) {
            const double w = u - 1.0;
            cw[j][0] = w / 6.0; cw[j][1] = w / 3.0;
        } else {
            const double b = 1.0 - u;
            cw[j][0] = (b * b * b - b) / 6.0; cw[j][1] = (u * u * u - u) / 6.0;
        }
        base += (int64_t)kf * stride;
        off[j] = stride;
        stride *= g.M[j];
    }
    for (int v = 0; v < nv; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int S = 0; S < (1 << D); ++S) {
            const double* c = coef + (((int64_t)v << D) + S) * g.Mtot + base;
#pragma unroll
            for (int q = 0; q < (1 << D); ++q) {
                double w = 1.0;
                int64_t o = 0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int e = (q >> j) & 1;
                    w *= ((S >> j) & 1) ? cw[j][e] : aw[j][e];
                    o += e ? off[j] : 0;
                }
                acc += w * c[o];
            }
        }
        out[(int64_t)v * Nq + i] = bad ? __builtin_nan("") : acc;
    }
}

// Per-block sums of a fixed-size accumulator vector; thread 0 of the block
// holds the result afterwards (LDS tree, fixed order).
template <int NA>
__device__ __forceinline__ void block_sum(double (&acc)[NA], double* sh) {
#pragma unroll
    for (int q = 0; q < NA; ++q) sh[q * 256 + threadIdx.x] = acc[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
#pragma unroll
            for (int q = 0; q < NA; ++q) sh[q * 256 + threadIdx.x] += sh[q * 256 + threadIdx.x + off];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = sh[q * 256];
}


// Fused interpolation and cv sums over the samples in sorted order: for the
// response columns of the launch sum |y - yhat|^2 (eq. 22), for its probes
// sum w^2 and sum w w_hat (Girard ratios, Sec. 2.1).  The probe fits are
// interleaved per grid point, so the 2^D corners of a sample bring all probes
// in contiguous loads; indexes past the launch's count are clamped (loaded,
// never summed).  Wave sums by cross-lane reduction, block sums in LDS.
template <int D, typename TW, int PC, bool YR>
__global__ __launch_bounds__(256) void k_reduce_cv(Geo g, ReduceCvArgs a) {
    constexpr int YC = kRedYCols, NA = YC + 2 * PC + 1;
    __shared__ double sh[NA][4];
    double ay[YC], aw[PC], ah[PC], an = 0.0;
#pragma unroll
    for (int j = 0; j < YC; ++j) ay[j] = 0.0;
#pragma unroll
    for (int j = 0; j < PC; ++j) aw[j] = ah[j] = 0.0;
    const TW* wrow = static_cast<const TW*>(a.wsorted);
    const int cpl = a.y_cplx ? 2 : 1;
    const int pcol = 1 + a.ny_cols * cpl + a.p0;
    // FP32 rows [1, y, probes of this launch ..] that 16-byte loads can take whole
    constexpr int NQ = (2 + PC + 3) / 4;
    const bool vec_row = YR && sizeof(TW) == 4 && pcol == 2 &&
                         (a.wgstride ? true : ((a.wstride % 4) == 0 && a.wstride >= 4 * NQ));
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.N;
         s += (int64_t)gridDim.x * blockDim.x) {
        const Corners<D> c = corners<D>(g, a.x_type, a.X, s);
        const TW* row = wrow + s * a.wstride;
        // column k of the sample's staged weights (rows or column groups)
        auto wcol = [&](int k) -> double {
            return (double)(a.wgstride ? wrow[(k >> 2) * a.wgstride + s * 4 + (k & 3)] : row[k]);
        };
        if constexpr (YR) {
            // FP32 rows [y | probes | pad] of 16-byte loads: the fit of the one
            // real response comes with the probe fits (all probes in this launch)
            constexpr int NV = 1 + PC, NC = (NV + 3) / 4;
            double fa[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) fa[j] = 0.0;
            const float* pf = static_cast<const float*>(a.pfit);
            const int last = (1 + a.np_launch + 3) / 4 - 1;
#pragma unroll
            for (int q = 0; q < (1 << D); ++q) {
                const float4* gv = reinterpret_cast<const float4*>(pf + c.idx[q] * a.pstride);
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const float4 v4 = gv[min(j, last)];
                    const float vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (4 * j + e < NV) fa[4 * j + e] += c.w[q] * (double)vv[e];
                }
            }
            // a sample whose cell touches an unresolved corner (NaN rows,
            // whatever the corner's weight) is left out of every sum
            if (isnan(fa[0])) continue;
            an += 1.0;
            if (vec_row) {
                // the staged row [1, y, probes ..] in 16-byte loads (probe
                // slots past the launch's count feed sums never written out)
                float rv[4 * NQ];
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    const float4 v4 = *reinterpret_cast<const float4*>(a.wgstride ? wrow + k * a.wgstride + s * 4
                                                                                  : row + 4 * k);
                    rv[4 * k] = v4.x; rv[4 * k + 1] = v4.y; rv[4 * k + 2] = v4.z; rv[4 * k + 3] = v4.w;
                }
                const double e0 = (double)rv[1] - fa[0];
                ay[0] += e0 * e0;
#pragma unroll
                for (int j = 0; j < PC; ++j) {
                    const double wv = (double)rv[2 + j];
                    aw[j] += wv * wv;
                    ah[j] += wv * fa[1 + j];
                }
                continue;
            }
            const double e0 = wcol(1) - fa[0];
            ay[0] += e0 * e0;
#pragma unroll
            for (int j = 0; j < PC; ++j) {
                const double wv = wcol(pcol + min(j, a.np_launch - 1));
                aw[j] += wv * wv;
                ah[j] += wv * fa[1 + j];
            }
            continue;
        }
        {
            float su = 0.f;
#pragma unroll
            for (int q = 0; q < (1 << D); ++q) su += a.sup[c.idx[q]];
            if (isnan(su)) continue;
            an += 1.0;
        }
#pragma unroll
        for (int j = 0; j < YC; ++j) {
            if (j >= a.ny_launch) break;
            const int col = a.y0 + j;
            if (a.y_cplx) {
                const double* gv = a.yfit + (int64_t)col * g.Mtot * 2;
                double fr = 0.0, fi = 0.0;
#pragma unroll
                for (int q = 0; q < (1 << D); ++q) {
                    fr += c.w[q] * gv[2 * c.idx[q]];
                    fi += c.w[q] * gv[2 * c.idx[q] + 1];
                }
                const double er = wcol(1 + 2 * col) - fr, ei = wcol(2 + 2 * col) - fi;
                ay[j] += er * er + ei * ei;
            } else {
                const double* gv = a.yfit + (int64_t)col * g.Mtot;
                double f = 0.0;
#pragma unroll
                for (int q = 0; q < (1 << D); ++q) f += c.w[q] * gv[c.idx[q]];
                const double e = wcol(1 + col) - f;
                ay[j] += e * e;
            }
        }
        if (a.np_launch > 0) {
            double fh[PC];
#pragma unroll
            for (int j = 0; j < PC; ++j) fh[j] = 0.0;
            const TW* pf = static_cast<const TW*>(a.pfit);
            // fits of the probes beyond np_launch (row padding included) land
            // in fh[j >= np_launch], which is never written out
            if (sizeof(TW) == 4 && (a.pstride % 4) == 0 && (a.p0 % 4) == 0) {
                // FP32 rows padded to 16 bytes: float4 loads
                const int last = (a.np_launch + 3) / 4 - 1;
#pragma unroll
                for (int q = 0; q < (1 << D); ++q) {
                    const float4* gv = reinterpret_cast<const float4*>(pf + c.idx[q] * a.pstride + a.p0);
#pragma unroll
                    for (int j = 0; j < (PC + 3) / 4; ++j) {
                        const float4 v4 = gv[min(j, last)];
                        const float vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (4 * j + e < PC) fh[4 * j + e] += c.w[q] * (double)vv[e];
                    }
                }
            } else if (sizeof(TW) == 8 && PC % 2 == 0 && (a.np_launch % 2) == 0 && (a.pstride % 2) == 0 &&
                       (a.p0 % 2) == 0) {
                // FP64 rows: 16-byte loads
                const int last = a.np_launch / 2 - 1;
#pragma unroll
                for (int q = 0; q < (1 << D); ++q) {
                    const double2* gv = reinterpret_cast<const double2*>(pf + c.idx[q] * a.pstride + a.p0);
#pragma unroll
                    for (int j = 0; j < PC / 2; ++j) {
                        const double2 v2 = gv[min(j, last)];
                        fh[2 * j] += c.w[q] * v2.x;
                        fh[2 * j + 1] += c.w[q] * v2.y;
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < (1 << D); ++q) {
                    const TW* gv = pf + c.idx[q] * a.pstride + a.p0;
#pragma unroll
                    for (int j = 0; j < PC; ++j) fh[j] += c.w[q] * (double)gv[min(j, a.np_launch - 1)];
                }
            }
#pragma unroll
            for (int j = 0; j < PC; ++j) {
                const double wv = wcol(pcol + min(j, a.np_launch - 1));
                aw[j] += wv * wv;
                ah[j] += wv * fh[j];
            }
        }
    }
    double acc[NA];
#pragma unroll
    for (int j = 0; j < YC; ++j) acc[j] = ay[j];
#pragma unroll
    for (int j = 0; j < PC; ++j) { acc[YC + 2 * j] = aw[j]; acc[YC + 2 * j + 1] = ah[j]; }
    acc[NA - 1] = an;
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NA; ++q) sh[q][wave] = acc[q];
    __syncthreads();
    if (threadIdx.x < NA) {
        const int q = threadIdx.x;
        const double v = sh[q][0] + sh[q][1] + sh[q][2] + sh[q][3];
        int slot = -1;
        if (q == NA - 1) {
            slot = a.count_slot;
        } else if (q < YC) {
            if (q < a.ny_launch) slot = 2 * (a.y0 + q);
        } else {
            const int j = (q - YC) >> 1;
            if (j < a.np_launch) slot = 2 * (a.ny_cols + a.p0 + j) + ((q - YC) & 1);
        }
        if (slot >= 0) {
            a.partial[(int64_t)slot * kRedBlocks + blockIdx.x] = v;
            // a launch of fewer than kRedBlocks workgroups: the slots no
            // workgroup owns hold zeros
            for (int b = blockIdx.x + gridDim.x; b < kRedBlocks; b += gridDim.x)
                a.partial[(int64_t)slot * kRedBlocks + b] = 0.0;
        }
    }
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* partial, double* out) {
    __shared__ double sh[256];
    const int slot = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += 256) v += partial[(int64_t)slot * kRedBlocks + b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[slot] = sh[0];
}

// True (and the stale flag set) when the points on the device are not the
// ones this launch was made for.  Uniform over the grid.
__device__ __forceinline__ bool points_stale(const PointsCheck& pc) {
    const bool bad = pc.diag[kDiagN] != (long long)pc.n || pc.diag[kDiagEpoch] != pc.epoch;
    if (bad && blockIdx.x == 0 && threadIdx.x == 0) pc.diag[kDiagStale] = 1;
    return bad;
}

__global__ void k_chan_tag(long long* diag, double h0, double h1, double h2) {
    if (threadIdx.x != 0) return;
    diag[kDiagChanEpoch] = diag[kDiagEpoch];
    diag[kDiagChanH] = __double_as_longlong(h0);
    diag[kDiagChanH + 1] = __double_as_longlong(h1);
    diag[kDiagChanH + 2] = __double_as_longlong(h2);
}

__global__ void k_chan_reuse(long long* diag, double h0, double h1, double h2) {
    if (threadIdx.x != 0) return;
    diag[kDiagReuse] = diag[kDiagChanEpoch] == diag[kDiagEpoch] && diag[kDiagChanH] == __double_as_longlong(h0) &&
                       diag[kDiagChanH + 1] == __double_as_longlong(h1) &&
                       diag[kDiagChanH + 2] == __double_as_longlong(h2) && diag[kDiagResidExcl] == 0;
}

// Girard ratios, RSS and GCV of one bandwidth over the N_I supported
// samples (red[2 n_items] holds N_I).  With rho_in the Girard mean is that
// of the given ratios (a DF computed by an earlier call).
__global__ void k_finalize_cv(int hidx, int Np, int q, const double* red, int n_items, int ny_cols,
                              const double* rho_in, double* rho_out, double* rss_out, double* gcv_out,
                              double* nused_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double n_used = red[2 * n_items];
    double mean = 0.0;
    for (int p = 0; p < Np; ++p) {
        double rho;
        if (rho_in) {
            rho = rho_in[(int64_t)hidx * Np + p];
        } else {
            const int item = ny_cols + p;
            const double ww = red[2 * item], wh = red[2 * item + 1];
            rho = (ww - wh) / ww;
        }
        if (rho_out) rho_out[(int64_t)hidx * Np + p] = rho;
        mean += rho;
    }
    mean = Np > 0 ? mean / Np : __builtin_nan("");
    if (nused_out) nused_out[hidx] = n_used;
    for (int c = 0; c < q; ++c) {
        const double rss = red[2 * c];
        if (rss_out) rss_out[(int64_t)hidx * q + c] = rss;
        if (gcv_out) gcv_out[(int64_t)hidx * q + c] = (rss / n_used) / (mean * mean);
    }
}

// Gradient sums over the supported samples (all 2^d corners of the cell
// resolved), in sorted order, for up to 32 columns of the derivative grids
// (all dimensions in one pass: column c of dimension j is grid j ncol + c):
// c < ny sums r_c d yhat_c with r = y - yhat, c = ny + p sums w_p d w_hat_p.
// Wave sums by cross-lane reduction, block sums in LDS.
template <int D, typename TW>
__global__ __launch_bounds__(256) void k_grad_sums(Geo g, GradSumArgs a) {
    constexpr int NA = 32;
    __shared__ double sh[NA][4];
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    const TW* W = static_cast<const TW*>(a.wsorted);
    auto wcol = [&](int64_t s, int col) {
        return (double)(a.wgstride ? W[(col >> 2) * a.wgstride + s * 4 + (col & 3)] : W[s * a.wstride + col]);
    };
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.N; s += (int64_t)gridDim.x * blockDim.x) {
        const Corners<D> c = corners<D>(g, a.x_type, a.X, s);
        bool ok = true;
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) ok &= a.sup[c.idx[q]] == 0.f;
        if (!ok) continue;
        // residuals of the (at most two) response parts
        double r0 = 0.0, r1 = 0.0;
        {
            double y0 = 0.0, y1 = 0.0;
#pragma unroll
            for (int e = 0; e < (1 << D); ++e) {
                y0 += c.w[e] * a.yfit[c.idx[e] * a.ny];
                if (a.ny > 1) y1 += c.w[e] * a.yfit[c.idx[e] * a.ny + 1];
            }
            r0 = wcol(s, 1) - y0;
            if (a.ny > 1) r1 = wcol(s, 2) - y1;
        }
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            if (q >= a.nall) break;
            const int gc = a.col0 + q;
            const int col = gc % a.ncol;
            const double coef = col < a.ny ? (col == 0 ? r0 : r1) : wcol(s, 1 + col);
            const double* gd = a.dfit + (int64_t)gc * g.Mtot;
            double dv = 0.0;
#pragma unroll
            for (int e = 0; e < (1 << D); ++e) dv += c.w[e] * gd[c.idx[e]];
            acc[q] += coef * dv;
        }
    }
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NA; ++q) sh[q][wave] = acc[q];
    __syncthreads();
    if ((int)threadIdx.x < a.nall)
        a.partial[(int64_t)(a.col0 + threadIdx.x) * kRedBlocks + blockIdx.x] =
            sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
}

// d GCV / d log h_j = GCV (dRSS / RSS - 2 d rho_bar / rho_bar), dRSS = -2 sum
// Re(conj(r) d yhat), d rho_p = -sum w_p d w_hat_p / sum w_p^2 (the supported
// set fixed).  red: the base sums (RSS of the response, then per probe sum
// w^2 and sum w w_hat, then N_I); gred: ny + Np gradient sums per dimension.
__global__ void k_finalize_grad(int d, int ny, int Np, const double* red, const double* gred, double* gcv_out,
                                double* dlogh) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int n_items = 1 + Np;
    const double n_used = red[2 * n_items];
    const double rss = red[0];
    double mean = 0.0;
    for (int p = 0; p < Np; ++p) {
        const double ww = red[2 * (1 + p)], wh = red[2 * (1 + p) + 1];
        mean += (ww - wh) / ww;
    }
    mean /= Np;
    const double gcv = (rss / n_used) / (mean * mean);
    if (gcv_out) *gcv_out = gcv;
    for (int j = 0; j < d; ++j) {
        const double* gj = gred + (int64_t)j * (ny + Np);
        double drss = 0.0;
        for (int c = 0; c < ny; ++c) drss += -2.0 * gj[c];
        double dmean = 0.0;
        for (int p = 0; p < Np; ++p) dmean += -gj[ny + p] / red[2 * (1 + p)];
        dmean /= Np;
        dlogh[j] = gcv * (drss / rss - 2.0 * dmean / mean);
    }
}

// ---------------------------------------------------------------------------
// Gradient of GCV in y: d GCV / dy = 2 / (N_I rho_bar^2) (r - S^T r), with r
// the residuals on the supported samples and S^T the adjoint of the smoother
// (interpolation, solve, moments): (S^T r)_l = sum_g sum_b v_b(g) k_b(x_l - g)
// with u = P^T r (the interpolation weights of the supported samples scattered
// to the grid), v_b = u c_b and c = A^{-1} e_0.  The sum over g is a type-2
// transform: the v_b on the zero-padded grid to the band (forward FFT), times
// the conjugate moment multipliers and the deconvolution, summed over b, back
// to the fine grid (inverse FFT), then the spreading kernel at each sample.
// ---------------------------------------------------------------------------
template <int D>
struct AdjWindow {   // grid cells per dimension of a workgroup's LDS accumulation window
    static constexpr int E = D == 1 ? 1024 : (D == 2 ? 32 : 12);
    static constexpr int SIZE = D == 1 ? E : (D == 2 ? E * E : E * E * E);
};

// u_c = P^T r_c for the ny parts of the residual, one sample per thread:
// the workgroup's samples (consecutive in sorted order, so near each other)
// add into an LDS window of grid cells anchored at their lowest cell, and
// the window goes to the grid with one atomic add per touched cell; corners
// outside the window are added to the grid directly.
template <int D, typename TW>
__global__ __launch_bounds__(256) void k_adj_scatter(Geo g, int64_t N, int x_type, const void* X, const TW* W,
                                                     int wstride, int64_t wgstride, int ny, const double* yfit,
                                                     const float* sup, double* u) {
    using AW = AdjWindow<D>;
    __shared__ double win[2][AW::SIZE];
    __shared__ int lo_s[3];
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x < 3) lo_s[threadIdx.x] = INT32_MAX;
    for (int q = threadIdx.x; q < 2 * AW::SIZE; q += blockDim.x) (&win[0][0])[q] = 0.0;
    __syncthreads();
    bool ok = s < N;
    Corners<D> c{};
    int cell[3] = {0, 0, 0};
    double r[2] = {0.0, 0.0};
    if (ok) {
        c = corners<D>(g, x_type, X, s);
        double yh[2] = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) {
            ok &= sup[c.idx[q]] == 0.f;
            for (int p = 0; p < ny; ++p) yh[p] += c.w[q] * yfit[c.idx[q] * ny + p];
        }
        for (int p = 0; p < ny; ++p)
            r[p] = (double)(wgstride ? W[s * 4 + 1 + p] : W[s * wstride + 1 + p]) - yh[p];
        int64_t rem = c.idx[0];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            cell[j] = (int)(rem % g.M[j]);
            rem /= g.M[j];
        }
        if (ok)
#pragma unroll
            for (int j = 0; j < D; ++j) atomicMin(&lo_s[j], cell[j]);
    }
    __syncthreads();
    if (ok) {
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) {
            int wi = 0, wstr = 1;
            bool inside = true;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int rj = cell[j] + ((q >> j) & 1) - lo_s[j];
                inside &= rj < AW::E;
                wi += rj * wstr;
                wstr *= AW::E;
            }
            for (int p = 0; p < ny; ++p) {
                const double v = c.w[q] * r[p];
                if (inside) atomicAdd(&win[p][wi], v);
                else atomicAdd(&u[p * g.Mtot + c.idx[q]], v);
            }
        }
    }
    __syncthreads();
    if (lo_s[0] == INT32_MAX) return;   // no supported sample in the workgroup
    for (int q = threadIdx.x; q < AW::SIZE; q += blockDim.x) {
        int rem = q;
        int64_t gi = 0, gstr = 1;
        bool valid = true;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int cj = lo_s[j] + rem % AW::E;
            rem /= AW::E;
            valid &= cj < g.M[j];
            gi += (int64_t)cj * gstr;
            gstr *= g.M[j];
        }
        if (!valid) continue;
        for (int p = 0; p < ny; ++p) {
            const double v = win[p][q];
            if (v != 0.0) atomicAdd(&u[p * g.Mtot + gi], v);
        }
    }
}

// v_b = u c_b packed two per complex grid function, [ceil(P/2)][M]; for
// the two parts of a complex response (cplx) one complex function per b,
// v_b = (u_re + i u_im) c_b, [P][M].  Zero where no supported sample reaches
// the grid point (c may be NaN there).
template <typename T>
__global__ __launch_bounds__(256) void k_adj_pack(int P, int64_t Mtot, const double* u, const double* c, int cplx,
                                                  typename V2<T>::t* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mtot) return;
    if (cplx) {
        const double ur = u[k], ui = u[Mtot + k];
        const bool zero = ur == 0.0 && ui == 0.0;
        for (int b = 0; b < P; ++b) {
            const double cb = zero ? 0.0 : c[b * Mtot + k];
            typename V2<T>::t v;
            v.x = (T)(ur * cb);
            v.y = (T)(ui * cb);
            out[b * Mtot + k] = v;
        }
        return;
    }
    const double uk = u[k];
    for (int q = 0; q < (P + 1) / 2; ++q) {
        const int b0 = 2 * q, b1 = 2 * q + 1;
        typename V2<T>::t v;
        v.x = (T)(uk == 0.0 ? 0.0 : uk * c[b0 * Mtot + k]);
        v.y = (T)(b1 < P && uk != 0.0 ? uk * c[b1 * Mtot + k] : 0.0);
        out[q * Mtot + k] = v;
    }
}

// Band spectrum of the adjoint: G(n) = prod_j fac_j(e_j) sum_b (-i)^{|b|}
// prod_j He_{b_j}(u_j) exp(-u_j^2/2) / T_j V_b(n), V_b unpacked from the pair
// spectra Z_q = V_{2q} + i V_{2q+1} ([band index][pairs]).
template <typename T>
__global__ __launch_bounds__(256) void k_adj_combine(ExpandArgs a, int P, int cplx, const int* et, const double* fac,
                                                     const typename V2<T>::t* spec, typename V2<T>::t* out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.Btot) return;
    const int npv = cplx ? P : (P + 1) / 2;
    double mloc[3][kExpandDeg];
    unsigned nn = 0, rem = (unsigned)n, stride = 1;
    double dec = 1.0;
    int64_t foff = 0;
    for (int j = 0; j < a.d; ++j) {
        const unsigned bj = (unsigned)a.B[j];
        const unsigned qj = rem / bj;
        const int ej = (int)(rem - qj * bj);
        rem = qj;
        nn += (bj - 1 - (unsigned)ej) * stride;
        stride *= bj;
        dec *= fac[foff + ej];
        foff += a.B[j];
        const double u = a.h[j] * (2.0 * M_PI * (double)(ej - a.K[j]) / a.T[j]);
        const double gj = exp(-0.5 * u * u) / a.T[j];
        if (a.ktab) {   // a compact kernel: the multipliers of its sampled moments
            int64_t off = 0;
            for (int i = 0; i < j; ++i) off += a.kdeg * a.B[i];
            for (int k = 0; k < kExpandDeg; ++k) mloc[j][k] = k < a.kdeg ? a.ktab[off + k * a.B[j] + ej] : 0.0;
            continue;
        }
        double hm = 1.0, he = u;
        mloc[j][0] = gj;
        mloc[j][1] = u * gj;
        for (int k = 1; k + 1 < kExpandDeg; ++k) {
            const double hn = u * he - k * hm;
            hm = he;
            he = hn;
            mloc[j][k + 1] = he * gj;
        }
    }
    double gr = 0.0, gi = 0.0;
    for (int b = 0; b < P; ++b) {
        double vr, vi;
        if (cplx) {   // the complex function of b itself (the map is linear over the complex numbers)
            const typename V2<T>::t zb = spec[n * npv + b];
            vr = (double)zb.x;
            vi = (double)zb.y;
        } else {
            const typename V2<T>::t zn = spec[n * npv + (b >> 1)];
            const typename V2<T>::t zm = spec[(int64_t)nn * npv + (b >> 1)];
            if ((b & 1) == 0) { vr = 0.5 * ((double)zn.x + (double)zm.x); vi = 0.5 * ((double)zn.y - (double)zm.y); }
            else { vr = 0.5 * ((double)zn.y + (double)zm.y); vi = -0.5 * ((double)zn.x - (double)zm.x); }
        }
        double m = 1.0;
        int deg = 0;
        for (int j = 0; j < a.d; ++j) {
            m *= mloc[j][et[3 * b + j]];
            deg += et[3 * b + j];
        }
        double xr = vr * m, xi = vi * m;
        switch (deg & 3) {   // multiply by (-i)^deg
            case 1: { const double t0 = xr; xr = xi; xi = -t0; break; }
            case 2: xr = -xr; xi = -xi; break;
            case 3: { const double t0 = xr; xr = -xi; xi = t0; break; }
            default: break;
        }
        gr += xr;
        gi += xi;
    }
    typename V2<T>::t o;
    o.x = (T)(gr * dec);
    o.y = (T)(gi * dec);
    out[n] = o;
}

// The same band spectrum for a full bandwidth matrix: G(n) = prod_j
// fac_j(e_j) sum_b (-i)^{|b|} M_{s(b)}(w_n) V_b(n) with M the forward
// channels' multipliers (the multivariate Hermite recurrence, the Gaussian
// factor and the equilibration) of the s-channel of multi-index b.
template <typename T>
__global__ __launch_bounds__(kExpandThreads) void k_adj_combine_full(ExpandArgs a, FullH fh, int P, int cplx,
                                                                     const int* es, const int* pidx,
                                                                     const double* fac,
                                                                     const typename V2<T>::t* spec,
                                                                     typename V2<T>::t* out) {
    __shared__ double mf[kMaxChannels][kExpandThreads];
    __shared__ double dmf[1][kExpandThreads];
    const int tid = threadIdx.x;
    const int64_t n = (int64_t)blockIdx.x * kExpandThreads + tid;
    if (n >= a.Btot) return;
    const int npv = cplx ? P : (P + 1) / 2;
    const unsigned nn = full_multipliers<false>(a, fh, es, n, tid, mf, dmf);
    double dec = 1.0;
    unsigned rem = (unsigned)n;
    int64_t foff = 0;
    for (int j = 0; j < a.d; ++j) {
        const unsigned bj = (unsigned)a.B[j];
        const unsigned qj = rem / bj;
        dec *= fac[foff + (int64_t)(rem - qj * bj)];
        rem = qj;
        foff += a.B[j];
    }
    double gr = 0.0, gi = 0.0;
    for (int b = 0; b < P; ++b) {
        double vr, vi;
        if (cplx) {
            const typename V2<T>::t zb = spec[n * npv + b];
            vr = (double)zb.x;
            vi = (double)zb.y;
        } else {
            const typename V2<T>::t zn = spec[n * npv + (b >> 1)];
            const typename V2<T>::t zm = spec[(int64_t)nn * npv + (b >> 1)];
            if ((b & 1) == 0) { vr = 0.5 * ((double)zn.x + (double)zm.x); vi = 0.5 * ((double)zn.y - (double)zm.y); }
            else { vr = 0.5 * ((double)zn.y + (double)zm.y); vi = -0.5 * ((double)zn.x - (double)zm.x); }
        }
        const int si = pidx[b * kMaxP];
        int deg = 0;
        for (int k = 0; k < a.d; ++k) deg += es[3 * si + k];
        const double m = mf[si][tid];
        double xr = vr * m, xi = vi * m;
        switch (deg & 3) {   // multiply by (-i)^deg
            case 1: { const double t0 = xr; xr = xi; xi = -t0; break; }
            case 2: xr = -xr; xi = -xi; break;
            case 3: { const double t0 = xr; xr = -xi; xi = t0; break; }
            default: break;
        }
        gr += xr;
        gi += xi;
    }
    typename V2<T>::t o;
    o.x = (T)(gr * dec);
    o.y = (T)(gi * dec);
    out[n] = o;
}

// (S^T r) at each sample from the fine grid f (the spreading kernel over the
// sample's footprint, the real part), and the gradient in original order.
// The transpose of the tiled spread: one workgroup per spreading job stages
// the job's padded tile of f in LDS, then its samples (first cell relative
// to the tile and fractions from the sort) read their footprints there; the
// kernel values are those of the spread (its precision KT).
template <int D, typename T, int KER, typename KT>
__global__ __launch_bounds__(256) void k_adj_gather(Geo g, int Np, const int32_t* jobs, const uint32_t* loc,
                                                    const KT* frac, int x_type, const void* X,
                                                    const int32_t* perm, const typename V2<T>::t* fgrid,
                                                    int ny, int part, const double* yfit, const float* sup,
                                                    const void* Wv, int w_type, int wstride, int64_t wgstride,
                                                    const double* red, double* grad) {
    // part < 0: both parts of a complex response, from the real and the
    // imaginary part of f (tile [2][PE^D] in LDS)
    extern __shared__ double tl[];
    const int pe0 = (int)g.pe[0], pe1 = D > 1 ? (int)g.pe[1] : 1, pe2 = D > 2 ? (int)g.pe[2] : 1;
    const int ps = pe0 * pe1 * pe2;
    const int w = g.w;
    const KT kp = (KT)g.kparam;
    const int n_items = 1 + Np;
    double mean = 0.0;
    for (int p = 0; p < Np; ++p) mean += (red[2 * (1 + p)] - red[2 * (1 + p) + 1]) / red[2 * (1 + p)];
    mean /= Np;
    const double scale = 2.0 / (red[2 * n_items] * mean * mean);
    const int njobs = jobs[0];
    for (int b = blockIdx.x; b < njobs; b += gridDim.x) {
        const int job = jobs[4 + 4 * b + 3];
        int tile = jobs[4 + 4 * job];
        const int s_beg = jobs[4 + 4 * job + 1], s_end = jobs[4 + 4 * job + 2];
        int org[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int ntj = (int)g.nt[j];
            org[j] = (tile % ntj) * (int)g.ts[j];
            tile /= ntj;
        }
        for (int c = threadIdx.x; c < ps; c += blockDim.x) {
            int rem = c;
            int64_t fi = 0, fs = 1;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int pj = j == 0 ? pe0 : (j == 1 ? pe1 : pe2);
                const int m = (org[j] + rem % pj) % (int)g.Mr[j];   // periodic fine grid
                rem /= pj;
                fi += (int64_t)m * fs;
                fs *= g.Mr[j];
            }
            const typename V2<T>::t fv = fgrid[fi];
            tl[c] = (double)fv.x;
            if (part < 0) tl[ps + c] = (double)fv.y;
        }
        __syncthreads();
        for (int64_t s = s_beg + threadIdx.x; s < s_end; s += blockDim.x) {
            const uint32_t l = loc[s];
            int bc[3] = {0, 0, 0};
            double kv[D][kMaxW];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                bc[j] = (int)((l >> (10 * j)) & 1023);
                const KT fr = frac[s * D + j];
                for (int k = 0; k < w; ++k) kv[j][k] = (double)kernel_value<KT, KER>((KT)k - fr, w, kp);
            }
            const int nparts = part < 0 ? 2 : 1;
            double accp[2] = {0.0, 0.0};
            for (int pp = 0; pp < nparts; ++pp) {
                const double* tp = tl + pp * ps;
                double acc = 0.0;
                if (D == 1) {
                    for (int k0 = 0; k0 < w; ++k0) acc += kv[0][k0] * tp[bc[0] + k0];
                } else if (D == 2) {
                    for (int k1 = 0; k1 < w; ++k1) {
                        const double* row = tp + (bc[D > 1 ? 1 : 0] + k1) * pe0 + bc[0];
                        double a1 = 0.0;
                        for (int k0 = 0; k0 < w; ++k0) a1 += kv[0][k0] * row[k0];
                        acc += kv[D > 1 ? 1 : 0][k1] * a1;
                    }
                } else {
                    for (int k2 = 0; k2 < w; ++k2) {
                        double a2 = 0.0;
                        for (int k1 = 0; k1 < w; ++k1) {
                            const double* row =
                                tp + ((bc[D > 2 ? 2 : 0] + k2) * pe1 + bc[D > 1 ? 1 : 0] + k1) * pe0 + bc[0];
                            double a1 = 0.0;
                            for (int k0 = 0; k0 < w; ++k0) a1 += kv[0][k0] * row[k0];
                            a2 += kv[D > 1 ? 1 : 0][k1] * a1;
                        }
                        acc += kv[D > 2 ? 2 : 0][k2] * a2;
                    }
                }
                accp[pp] = acc;
            }
            // the sample's own residual when it is supported
            const Corners<D> c = corners<D>(g, x_type, X, s);
            bool ok = true;
#pragma unroll
            for (int q = 0; q < (1 << D); ++q) ok &= sup[c.idx[q]] == 0.f;
            for (int pp = 0; pp < nparts; ++pp) {
                const int pt = part < 0 ? pp : part;
                double yh = 0.0;
#pragma unroll
                for (int q = 0; q < (1 << D); ++q) yh += c.w[q] * yfit[c.idx[q] * ny + pt];
                double y;
                if (w_type == FKR_F64) {
                    const double* W = static_cast<const double*>(Wv);
                    y = wgstride ? W[s * 4 + 1 + pt] : W[s * wstride + 1 + pt];
                } else {
                    const float* W = static_cast<const float*>(Wv);
                    y = (double)(wgstride ? W[s * 4 + 1 + pt] : W[s * wstride + 1 + pt]);
                }
                const double r = ok ? y - yh : 0.0;
                accp[pp] = scale * (r - accp[pp]);
            }
            if (part < 0)
                reinterpret_cast<double2*>(grad)[perm[s]] = make_double2(accp[0], accp[1]);
            else
                grad[(int64_t)perm[s] * ny + part] = accp[0];
        }
        __syncthreads();
    }
}

// Residuals of the mean fit for the variance pass (Sec. 3), in sorted sample
// order s: rows[s] = (1, z, 0, 0), the staged weight row of the second fit's
// spread (z = log(r + 1/N) or r, in the spreading precision TW), and
// r_out[s] = r.
template <int D, typename TW>
__global__ __launch_bounds__(256) void k_resid(Geo g, int mode, PointsCheck pc, int x_type, const void* xs,
                                               const int32_t* perm, int y_type, const void* Y,
                                               int y_cplx, const double* mhat, double* r_out, TW* rows,
                                               int rstride) {
    if (points_stale(pc)) return;
    const int64_t N = pc.n;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const Corners<D> c = corners<D>(g, x_type, xs, s);
    const int64_t i = perm[s];
    double r;
    if (y_cplx) {
        double fr = 0.0, fi = 0.0;
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) { fr += c.w[q] * mhat[2 * c.idx[q]]; fi += c.w[q] * mhat[2 * c.idx[q] + 1]; }
        const double yr = load_as_double(Y, y_type, 2 * i) - fr;
        const double yi = load_as_double(Y, y_type, 2 * i + 1) - fi;
        r = yr * yr + yi * yi;
    } else {
        double f = 0.0;
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) f += c.w[q] * mhat[c.idx[q]];
        const double e = load_as_double(Y, y_type, i) - f;
        r = e * e;
    }
    // a sample whose residual is undefined (NaN mean fit at a corner) is
    // left out of the second fit: density and response weights 0
    const bool ok = isfinite(r);
    const TW one = ok ? (TW)1 : (TW)0;
    const TW z = ok ? (TW)(mode == FKR_VAR_LOG ? log(r + 1.0 / (double)N) : r) : (TW)0;
    if constexpr (sizeof(TW) == 4) {
        if (rstride == 2) reinterpret_cast<float2*>(rows)[s] = make_float2(one, z);
        else reinterpret_cast<float4*>(rows)[s] = make_float4(one, z, 0.f, 0.f);
    } else {
        reinterpret_cast<double2*>(rows)[2 * s] = make_double2(one, z);
        reinterpret_cast<double2*>(rows)[2 * s + 1] = make_double2(0.0, 0.0);
    }
    r_out[s] = ok ? r : __builtin_nan("");
    if (!ok) pc.diag[kDiagResidExcl] = 1;
}

// A grid function (a variance estimate) at every sorted sample by multilinear
// interpolation, staged as the two-column rows (G(x_s), 0) of a spread;
// samples where it is undefined get weight 0 (they are left out).
template <int D, typename TW>
__global__ __launch_bounds__(256) void k_stage_grid(Geo g, PointsCheck pc, int x_type, const void* xs,
                                                    const double* G, TW* rows, int rstride) {
    if (points_stale(pc)) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= pc.n) return;
    const Corners<D> c = corners<D>(g, x_type, xs, s);
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < (1 << D); ++q) v += c.w[q] * G[c.idx[q]];
    const TW w = isfinite(v) ? (TW)v : (TW)0;
    if constexpr (sizeof(TW) == 4) {
        if (rstride == 2) reinterpret_cast<float2*>(rows)[s] = make_float2(w, 0.f);
        else reinterpret_cast<float4*>(rows)[s] = make_float4(w, 0.f, 0.f, 0.f);
    } else {
        reinterpret_cast<double2*>(rows)[2 * s] = make_double2(w, 0.0);
        reinterpret_cast<double2*>(rows)[2 * s + 1] = make_double2(0.0, 0.0);
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_kappa_partial(Geo g, int64_t N, int x_type, const void* xs,
                                                       const int32_t* perm, const double* vhat,
                                                       const double* r, double* partial) {
    __shared__ double sh[2 * 256];
    double acc[2] = {0.0, 0.0};
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
         s += (int64_t)gridDim.x * blockDim.x) {
        const Corners<D> c = corners<D>(g, x_type, xs, s);
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < (1 << D); ++q) v += c.w[q] * vhat[c.idx[q]];
        const double term = r[s] * exp(-v);
        if (isfinite(term)) {
            acc[0] += term;
            acc[1] += 1.0;
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = acc[0];
        partial[kRedBlocks + blockIdx.x] = acc[1];
    }
}

__global__ __launch_bounds__(256) void k_sigma2(int64_t Mtot, const double* vhat, const double* ksum,
                                                double* sigma2, double* kappa_out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double kappa = ksum[1] / ksum[0];   // count / sum of r exp(-v)
    if (k == 0 && kappa_out) kappa_out[0] = kappa;
    if (k >= Mtot) return;
    sigma2[k] = exp(vhat[k]) / kappa;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Weight vectors in sorted order: out[s * nr + r0 + q] = source q at sample
// perm[s].  Probes of one Philox block (indices 4g .. 4g+3) share the block and
// its two Box-Muller transforms.
template <typename T>
__global__ __launch_bounds__(256) void k_stage_weights(SpreadSrc src, int nsrc, int r0, int nr, int64_t gstride,
                                                       PointsCheck pc, const int32_t* perm, T* out) {
    // one sample per thread; when the launch writes whole rows (nsrc == nr)
    // the rows of each wave go out through LDS as one contiguous block
    __shared__ __align__(16) T stg[256 * 2 * kMaxPairsPerSpread];
    if (points_stale(pc)) return;
    const int64_t N = pc.n;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool whole = nsrc == nr && gstride == 0;
    if (s >= N && !whole) return;
    const int64_t i = s < N ? perm[s] : 0;
    uint64_t cached_seed = 0, cached_g = ~0ull;
    T z[4] = {0, 0, 0, 0};
    T vals[2 * kMaxPairsPerSpread];
#pragma unroll
    for (int q = 0; q < 2 * kMaxPairsPerSpread; ++q) {
        vals[q] = (T)0;
        if (q >= nsrc || s >= N) continue;
        const WSrc& w = src.w[q];
        double v;
        if (w.kind == W_PHILOX) {
            const uint64_t gq = (uint64_t)(w.probe >> 2);
            if (gq != cached_g || w.seed != cached_seed) {
                uint32_t x[4];
                philox_block(w.seed, (uint64_t)i, (uint32_t)gq, x);
                box_muller4(x, z);
                cached_g = gq;
                cached_seed = w.seed;
            }
            const int pr = w.probe & 3;   // selects instead of a dynamic register index
            v = (double)(pr == 0 ? z[0] : pr == 1 ? z[1] : pr == 2 ? z[2] : z[3]);
        } else {
            v = wval_mem(w, s, i);
        }
        vals[q] = (T)v;
    }
    // 16-byte stores (nsrc, r0 and nr are multiples of 4 for T = float, of 2
    // for T = double)
    constexpr int VW = 16 / sizeof(T);
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    if (whole) {
        // the wave's rows [s0, s0 + 64) are contiguous in `out`: stage them in
        // LDS and store 16-byte chunks with consecutive lanes on consecutive
        // chunks
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        T* w = stg + wv * 64 * 2 * kMaxPairsPerSpread;
#pragma unroll
        for (int q = 0; q < 2 * kMaxPairsPerSpread; ++q)
            if (q < nsrc) w[lane * nsrc + q] = vals[q];
        __syncthreads();
        const int64_t s0 = s - lane;
        const int64_t nrows = min<int64_t>(64, N - s0);
        if (nrows > 0) {
            const int nv = (int)(nrows * nr / VW);
            V* dst = reinterpret_cast<V*>(out + s0 * nr);
            const V* src4 = reinterpret_cast<const V*>(w);
            for (int k = lane; k < nv; k += 64) dst[k] = src4[k];
        }
        return;
    }
    if (gstride) {
        // column groups of four: consecutive samples' 16-byte chunks are
        // adjacent (r0 and nsrc are multiples of 4)
#pragma unroll
        for (int q = 0; q < 2 * kMaxPairsPerSpread; q += 4) {
            if (q >= nsrc) break;
            T* dg = out + ((r0 + q) >> 2) * gstride + s * 4;
            if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<float4*>(dg) = make_float4(vals[q], vals[q + 1], vals[q + 2], vals[q + 3]);
            } else {
                *reinterpret_cast<double2*>(dg) = make_double2(vals[q], vals[q + 1]);
                *reinterpret_cast<double2*>(dg + 2) = make_double2(vals[q + 2], vals[q + 3]);
            }
        }
        return;
    }
    T* dst = out + s * nr + r0;
#pragma unroll
    for (int q = 0; q < 2 * kMaxPairsPerSpread; q += VW) {
        if (q >= nsrc) break;
        if constexpr (sizeof(T) == 4)
            *reinterpret_cast<float4*>(dst + q) = make_float4(vals[q], vals[q + 1], vals[q + 2], vals[q + 3]);
        else
            *reinterpret_cast<double2*>(dst + q) = make_double2(vals[q], vals[q + 1]);
    }
}

// Per-weight spectra C_r(n) (complex128, [r][n]) from the pair spectra.
template <typename T>
__global__ void k_unpack_spec(int64_t Btot, int d, int64_t B0, int64_t B1, int64_t B2, int npairs,
                              int nw, const typename V2<T>::t* spec, double* out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Btot * nw) return;
    const int r = (int)(idx / Btot);
    const int64_t n = idx - (int64_t)r * Btot;
    const int64_t B[3] = {B0, B1, B2};
    int64_t rem = n, nn = 0, stride = 1;
    for (int j = 0; j < d; ++j) {
        const int64_t e = rem % B[j];
        rem /= B[j];
        nn += (B[j] - 1 - e) * stride;
        stride *= B[j];
    }
    const int p = r >> 1;
    const auto zn = spec[n * npairs + p];
    const auto zm = spec[nn * npairs + p];
    double cr, ci;
    if ((r & 1) == 0) { cr = 0.5 * ((double)zn.x + (double)zm.x); ci = 0.5 * ((double)zn.y - (double)zm.y); }
    else { cr = 0.5 * ((double)zn.y + (double)zm.y); ci = -0.5 * ((double)zn.x - (double)zm.x); }
    out[2 * idx] = cr;
    out[2 * idx + 1] = ci;
}

// Channel grids [k][ncp] complex -> S [n_s][M] and T [nw][n_t][M] (FP64).
template <typename T>
__global__ void k_chan_out(int64_t Mtot, int ncp, int n_s, int n_t, int nw, const T* chan,
                           double* S, double* Tt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nreal = n_s + n_t * nw;
    if (idx >= Mtot * nreal) return;
    const int ch = (int)(idx / Mtot);
    const int64_t k = idx - (int64_t)ch * Mtot;
    const double v = (double)chan[((int64_t)(ch >> 1) * Mtot + k) * 2 + (ch & 1)];   // [pair][M][re, im]
    if (ch < n_s) { if (S) S[(int64_t)ch * Mtot + k] = v; }
    else if (Tt) Tt[(int64_t)(ch - n_s) * Mtot + k] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

void launch_stage_weights(int prec, const SpreadSrc& src, int nsrc, int r0, int nr, int64_t gstride,
                          const PointsCheck& pc, const int32_t* perm, void* out, hipStream_t s) {
    if (pc.n == 0) return;
    if (prec == FKR_F64)
        k_stage_weights<double><<<nblk(pc.n), 256, 0, s>>>(src, nsrc, r0, nr, gstride, pc, perm,
                                                           static_cast<double*>(out));
    else
        k_stage_weights<float><<<nblk(pc.n), 256, 0, s>>>(src, nsrc, r0, nr, gstride, pc, perm,
                                                          static_cast<float*>(out));
}

// ---------------------------------------------------------------------------
// Workspace held by the library for the entry point that allocates nothing
// (fkr_fit_noalloc): one array per device, for the life of the process.  In
// host code the array's name only stands in for it; its device address comes
// from hipGetSymbolAddress, taken once per device and cached.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n > 0) k_zero<<<nblk(n), 256, 0, s>>>(static_cast<uint32_t*>(p), n);
}

void launch_bin_count(const Geo& g, int x_type, const void* X, int64_t N, int32_t* counts, int32_t* bhist,
                      int32_t* obuf, hipStream_t s) {
    if (N == 0) return;
    const unsigned nb = (unsigned)((N + kSortChunk - 1) / kSortChunk);
    const bool use_lds = g.n_tiles <= kLdsHistMax;
    const size_t lds = use_lds ? (size_t)g.n_tiles * 4 : 0;
    switch (g.d) {
        case 1: k_bin_count<1><<<nb, kSortThreads, lds, s>>>(g, x_type, X, N, counts, bhist, obuf); break;
        case 2: k_bin_count<2><<<nb, kSortThreads, lds, s>>>(g, x_type, X, N, counts, bhist, obuf); break;
        default: k_bin_count<3><<<nb, kSortThreads, lds, s>>>(g, x_type, X, N, counts, bhist, obuf); break;
    }
    if (use_lds) k_tile_prefix<<<(unsigned)((g.n_tiles + 63) / 64), 1024, 0, s>>>(g.n_tiles, (int)nb, bhist, counts);
}

void launch_scan(const Geo& g, int64_t N, long long epoch, int32_t* counts, int32_t* tile_off, int32_t* job_off,
                 int32_t* jobs, int32_t* cursor, long long* diag, const int32_t* obuf, hipStream_t s) {
    const int nbins = (int)((N + kSortChunk - 1) / kSortChunk);
    k_scan<<<1, 1024, 0, s>>>(g.n_tiles, g.chunk, N, epoch, counts, tile_off, job_off, jobs, cursor, diag, obuf,
                              nbins);
}

void launch_chan_tag(long long* diag, const double* h, int d, hipStream_t s) {
    k_chan_tag<<<1, 64, 0, s>>>(diag, h[0], d > 1 ? h[1] : 0.0, d > 2 ? h[2] : 0.0);
}

__global__ void k_chan_untag(long long* diag) {
    if (threadIdx.x == 0) diag[kDiagChanEpoch] = -1;
}

void launch_chan_untag(long long* diag, hipStream_t s) { k_chan_untag<<<1, 64, 0, s>>>(diag); }

void launch_chan_reuse(long long* diag, const double* h, int d, hipStream_t s) {
    k_chan_reuse<<<1, 64, 0, s>>>(diag, h[0], d > 1 ? h[1] : 0.0, d > 2 ? h[2] : 0.0);
}

template <int D, typename T>
static void sort_cells_dt(const Geo& g, int x_type, const void* X, int64_t N, int64_t n_jobs_max,
                          const int32_t* tile_off, int32_t* cursor, const int32_t* jobs, const int32_t* bhist,
                          void* trec_v, uint32_t* loc, void* frac, int32_t* perm, void* xs, hipStream_t s) {
    using R = TileRec<D, T>;
    R* trec = static_cast<R*>(trec_v);
    const unsigned nb = (unsigned)((N + kSortChunk - 1) / kSortChunk);
    const size_t lds = g.n_tiles <= kLdsHistMax ? (size_t)g.n_tiles * 4 : 0;
    k_scatter_tiles<D, T><<<nb, kSortThreads, lds, s>>>(g, x_type, X, N, tile_off, cursor, bhist, trec);
    // records staged in LDS when they fit the budget (up to the 160 KB a
    // gfx950 workgroup may hold; 3-D jobs are sized for it); 3-D jobs are
    // large and sorted by 1024 threads
    constexpr int NT = D == 3 ? 1024 : 256;
    const size_t base_bytes = (size_t)g.ncell * 4 + NT * 4;
    const size_t stage_bytes = base_bytes + (size_t)g.chunk * (8 + 2 * D * sizeof(T));
    const int stage = stage_bytes <= 160 * 1024 ? 1 : 0;
    const size_t sort_lds = stage ? stage_bytes : base_bytes;
    if (sort_lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cell_sort<D, T, NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sort_lds);
    k_cell_sort<D, T, NT><<<(unsigned)n_jobs_max, NT, sort_lds, s>>>(g, jobs, trec, stage, loc, static_cast<T*>(frac),
                                                                perm, static_cast<T*>(xs));
}

size_t tile_record_bytes(int d, int prec) {
    if (prec == FKR_F64) return d == 1 ? sizeof(TileRec<1, double>) : d == 2 ? sizeof(TileRec<2, double>) : sizeof(TileRec<3, double>);
    return d == 1 ? sizeof(TileRec<1, float>) : d == 2 ? sizeof(TileRec<2, float>) : sizeof(TileRec<3, float>);
}

void launch_sort_cells(const Geo& g, int prec, int x_type, const void* X, int64_t N, int64_t n_jobs_max,
                       const int32_t* tile_off, int32_t* cursor, const int32_t* jobs, const int32_t* bhist,
                       void* trec, uint32_t* loc, void* frac, int32_t* perm, void* xs, hipStream_t s) {
    if (N == 0) return;
#define FKR_SC(D, T) sort_cells_dt<D, T>(g, x_type, X, N, n_jobs_max, tile_off, cursor, jobs, bhist, trec, loc, frac, perm, xs, s)
    if (prec == FKR_F64) {
        if (g.d == 1) FKR_SC(1, double); else if (g.d == 2) FKR_SC(2, double); else FKR_SC(3, double);
    } else {
        if (g.d == 1) FKR_SC(1, float); else if (g.d == 2) FKR_SC(2, float); else FKR_SC(3, float);
    }
#undef FKR_SC
}

// 2-D spread with one sample stream per wave (footprints of at most 64
// cells).  Lane l owns footprint cell (l % W, l / W); all lanes of the wave
// work on the same sample, so the first-cell test, the flush and the weight
// loads are wave-uniform (scalar loads, SGPR operands in the FMAs).  The
// kernel rows of U = 64 / (2W) consecutive samples are evaluated in one pass
// (lane = sample, dimension, offset) and fetched with two cross-lane permutes
// per sample.  Each wave takes a contiguous segment of the job; registers are
// added into the FP64 LDS tile when the first footprint cell changes.  The
// launch spreads exactly NW = 2 np weight columns (np <= 8 pairs).
template <int W, int KER, int NW>
__global__ __launch_bounds__(512) void k_spread_wave(Geo g, const float* __restrict__ wrow, int wstride,
                                                     int col0, const uint32_t* __restrict__ loc,
                                                     const float* __restrict__ frac, const int32_t* __restrict__ jobs,
                                                     float* __restrict__ subgrid) {
    constexpr int TS = spread_tile_edge(2, W);
    constexpr int PE = TS + W - 1;
    constexpr int PSUB = PE * PE;
    constexpr int NWAVE = 512 / 64;
    constexpr int U = 64 / (2 * W);
    constexpr int NP = NW / 2;
    static_assert(W * W <= 64 && U >= 1 && NW % 2 == 0, "footprint must fit a wave");
    extern __shared__ double tile[];   // [NW][PSUB]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int dx = lane % W, dy = lane / W;
    const bool fp_lane = lane < W * W;
    const int pu = lane / (2 * W), pj = (lane / W) & 1, pk = lane % W;
    const float kp = (float)g.kparam;
    const int njobs = jobs[0];
    for (int b = blockIdx.x; b < njobs; b += gridDim.x) {
        const int job = jobs[4 + 4 * b + 3];
        const int s_beg = jobs[4 + 4 * job + 1];
        const int n = jobs[4 + 4 * job + 2] - s_beg;
        const int seg = (n + NWAVE - 1) / NWAVE;
        const int q0 = min(n, wave * seg), q1 = min(n, q0 + seg);
        for (int c = threadIdx.x; c < NW * PSUB; c += blockDim.x) tile[c] = 0.0;
        __syncthreads();
        float acc[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) acc[k] = 0.f;
        int cur = -1;
        auto flush_to = [&](int cb) {
            if (cb == cur) return;
            if (cur >= 0 && fp_lane) {
                const int cell = cur + dx + PE * dy;
#pragma unroll
                for (int k = 0; k < NW; ++k) atomicAdd(&tile[k * PSUB + cell], (double)acc[k]);
            }
#pragma unroll
            for (int k = 0; k < NW; ++k) acc[k] = 0.f;
            cur = cb;
        };
        auto cell_of = [&](uint32_t l) { return (int)(l & 1023) + PE * (int)((l >> 10) & 1023); };
        // weight rows and records of the wave's segment, advanced per step
        const float* wp = wrow + col0 + (int64_t)(s_beg + q0) * wstride;
        const uint32_t* lp = loc + s_beg + q0;
        const float* fp = frac + 2 * (int64_t)(s_beg + q0);
        // One step = UU consecutive samples.  Every load of the step (first
        // cells, fractions, weight rows) and every cross-lane permute is
        // issued before the first FMA, so the step waits once: scalar loads
        // return out of order and share the LDS counter, so any wait for a
        // permute would otherwise also wait for loads issued after it.
        auto step = [&](auto UUc) {
            constexpr int UU = decltype(UUc)::value;
            const float f = fp[2 * min(pu, UU - 1) + pj];
            uint32_t lu[UU];
            float wv[UU][NW];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                lu[u] = lp[u];
                const float* wr = wp + u * wstride;
#pragma unroll
                for (int k = 0; k < NW; ++k) wv[u][k] = wr[k];
            }
            const float v = kernel_value<float, KER>((float)pk - f, W, kp);
            float psi[UU];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const float a = __shfl(v, 2 * W * u + dx);
                const float b = __shfl(v, 2 * W * u + W + min(dy, W - 1));
                psi[u] = fp_lane ? a * b : 0.f;
            }
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                flush_to(cell_of(lu[u]));
#pragma unroll
                for (int k = 0; k < NW; ++k) acc[k] += psi[u] * wv[u][k];
            }
            wp += UU * wstride;
            lp += UU;
            fp += 2 * UU;
        };
        // samples per step: as many as the kernel-row pass covers, fewer when
        // the weight rows of a step would not fit the scalar registers
        constexpr int US = NW <= 8 ? U : (NW <= 12 ? (U < 4 ? U : 4) : (U < 3 ? U : 3));
        int t = q0;
        for (; t + US <= q1; t += US) step(std::integral_constant<int, US>{});
        for (; t < q1; ++t) step(std::integral_constant<int, 1>{});
        if (cur >= 0 && fp_lane) {
            const int cell = cur + dx + PE * dy;
#pragma unroll
            for (int k = 0; k < NW; ++k) atomicAdd(&tile[k * PSUB + cell], (double)acc[k]);
        }
        __syncthreads();
        // subgrid layout [job][pair][cell][re, im]
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            float* dst = subgrid + ((int64_t)job * NP + q) * PSUB * 2;
            for (int c = threadIdx.x; c < PSUB; c += blockDim.x) {
                dst[2 * c] = (float)tile[2 * q * PSUB + c];
                dst[2 * c + 1] = (float)tile[(2 * q + 1) * PSUB + c];
            }
        }
        __syncthreads();
    }
}

// 3-D spread on the matrix cores, W = 8.  Within a job the samples are sorted
// by first cell with (x, y) major and z minor, so a wave sees long runs (about
// a hundred samples) of one (x, y) column of first cells, made of runs (about
// sixteen) of one first cell.  For one column the spread is a contraction over
// its samples s:
//
//   S[(dx, dy), (z, c)] += sum_s psi_x(s, dx) psi_y(s, dy) * psi_z(s, z - z0(s)) w(s, c)
//
// a [64 x S] by [S x (15 planes x NC columns)] product with the 64 footprint
// columns as rows.  It runs as FP32 MFMA 16x16x4 blocks: four row blocks of
// 16 (dx, dy) and NC column blocks of 16 (16 / NC planes x NC weight
// columns).  One block step takes up to four samples of one first cell, so
// the plane offset z0 is uniform over the step: with z0 = ZPB a + b the
// window z0 .. z0 + 7 meets column blocks a .. a + 8 / ZPB (the last only
// when b > 0), and the B operand of block a + t is psi_z at offset
// ZPB t + (plane in block) - b, read from psi_z staged with zeros on both
// sides.  The accumulators stay in the matrix unit for the whole column and
// go to the FP64 LDS tile when the (x, y) column changes.
//
// A wave takes its samples in batches of kCol3Batch: one lane pair per sample
// loads the record and weights with vector loads (the next batch is fetched
// while the current one is spread), evaluates the sample's 24 kernel values
// (12 per lane) and writes them with the weights to a per-wave LDS row, from
// which the block operands are read.  A run of one first cell that a batch
// cuts leaves its last (length mod 4) samples to the next batch, so no step
// is cut short.  A launch spreads np pairs in passes of NC / 2 pairs (the LDS
// tile holds NC columns).
constexpr int kCol3Batch = 32;
// Doubles per weight column of the LDS tile: the 15^3 cells and 9 of padding,
// which puts the columns 8 bank pairs apart (3384 = 24 mod 32) so that the
// FP64 atomic adds of a flush spread over the banks (3375: 3.91 ms for the
// step's two 3-D spread launches; 3384: 3.53 ms; 3392: 3.97 ms).
constexpr int kCol3TileStride = 15 * 15 * 15 + 9;
// Staged sample row (floats): psi_x[8], psi_y[8] (permuted), PAD zeros,
// psi_z[8], PAD zeros, w[4]; PAD = 16 / NC covers the plane offsets a step
// reads around psi_z (one column: the window offset is below 8)
template <int NC>
struct Col3Row {
    static constexpr int PAD = NC == 1 ? 8 : 16 / NC;
    static constexpr int Z = 16 + PAD;     // psi_z[0]
    static constexpr int W = Z + 8 + PAD;  // w[0]
    static constexpr int N = W + 4;
};

typedef float col3_v4 __attribute__((ext_vector_type(4)));

// Row offset of kernel value slot s (0..23): psi_x(s) for s < 8; psi_y for
// s < 16, stored as [dy % 2][dy / 2] so that a lane reads its four row
// blocks' values with one 16-byte load; psi_z(s - 16) after the zeros.
__device__ __forceinline__ int col3_slot_offset(int s) {
    if (s < 8) return s;
    if (s < 16) {
        const int t = s - 8;
        return 2 * (t & 3) + (t >> 2);
    }
    return s - 16;
}

__device__ __forceinline__ uint32_t lane_value(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Column blocks a step touches: its window of eight planes starts in block
// a = z0 / ZPB and reaches block a + 8 / ZPB (one column: the 16 planes of
// the one block hold every window, z0 < 8).
template <int NC>
constexpr int col3_blocks() { return 8 / (16 / NC) + 1; }

// Accumulator blocks t = 0 .. NF - 1 of one (x, y) column to the LDS tile:
// block t holds planes ZPB (base + t) .. ZPB (base + t) + ZPB - 1; in it
// row block rb, lane l, register r is footprint row 4 (l / 16) + r of the
// row block, column l % 16 (plane offset (l % 16) / NC, weight (l % 16) % NC).
template <int NC, int NF>
__device__ __forceinline__ void col3_flush(col3_v4 (&acc)[col3_blocks<NC>()][4], double* tile, int cur, int base,
                                           int lane) {
    constexpr int PE = 15, PSUB = kCol3TileStride, ZPB = 16 / NC;
    const int q = lane >> 4, j = lane & 15;
    const int zc = j / NC, c = j % NC;
    double* t = tile + c * PSUB + (cur & 1023) + 4 * (q & 1) + PE * (((cur >> 10) & 1023) + (q >> 1));
#pragma unroll
    for (int tb = 0; tb < NF; ++tb) {
        const int z = ZPB * (base + tb) + zc;   // planes past 14 only ever hold zeros
        if (z < PE) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    // columns past the pass's count hold zeros and land in
                    // tile columns that are never written out
                    atomicAdd(t + r + PE * (2 * rb) + PE * PE * z, (double)acc[tb][rb][r]);
        }
    }
}

// Block base to the tile, the others move down one block (a zero block
// comes in at the top).
template <int NC>
__device__ __forceinline__ void col3_flush_first(col3_v4 (&acc)[col3_blocks<NC>()][4], double* tile, int cur,
                                                 int base, int lane) {
    constexpr int NB = col3_blocks<NC>();
    col3_flush<NC, 1>(acc, tile, cur, base, lane);
#pragma unroll
    for (int tb = 0; tb + 1 < NB; ++tb)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[tb][rb] = acc[tb + 1][rb];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[NB - 1][rb] = col3_v4{0.f, 0.f, 0.f, 0.f};
}

// NC = 1 spreads only the second column of each pair and stores zeros as
// the first (the variance pass when the density moments are kept).  With a
// gate the launch runs only when (*gate != 0) == gate_on (a flag the device
// sets, so a captured graph holds both launches and one of them returns).
template <int KER, int NC, int NT>
__global__ __launch_bounds__(NT) void k_spread_col3(Geo g, int np, const float* __restrict__ wrow, int wstride,
                                                    int64_t gstride, int col0, const uint32_t* __restrict__ loc,
                                                    const float* __restrict__ frac,
                                                    const int32_t* __restrict__ jobs,
                                                    float* __restrict__ subgrid, const long long* gate,
                                                    int gate_on) {
    constexpr int W = 8, PE = 15, PSUB = kCol3TileStride, NCELL = PE * PE * PE;
    constexpr int NWAVE = NT / 64;
    constexpr int PPP = NC == 1 ? 1 : NC / 2;   // pairs per pass
    constexpr int B = kCol3Batch;
    constexpr int ZPB = 16 / NC;   // planes per column block
    constexpr int NB = col3_blocks<NC>();
    static_assert(NC == 1 || NC == 2 || NC == 4, "columns per pass");
    if (gate && ((*gate != 0) != (gate_on != 0))) return;   // uniform over the grid
    // LDS: the tile [NC][PSUB] (cell = x + PE (y + PE z)), then one staging
    // area of B rows per wave
    extern __shared__ double tile[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    using RW = Col3Row<NC>;
    float* const stage = reinterpret_cast<float*>(tile + NC * PSUB) + wave * B * RW::N;
    // block-operand roles: sample k of the step; row i (A) and column j (B)
    const int k = lane >> 4, ij = lane & 15;
    const int ax = ij & 7, ah = ij >> 3;      // A row i = (dx, dy) = (i % 8, 2 rb + i / 8)
    const int bz = ij / NC, bc = ij % NC;     // B column j = (plane ZPB cb + j / NC, weight j % NC)
    // staging role: sample sl of the batch; the low half of the wave takes
    // kernel slots 0..11 of the row, the high half 12..23 and the weights
    const int sl = lane & (B - 1);
    const int hi = lane >> 5;
    const float kp = (float)g.kparam;
    // the zeros around psi_z are never overwritten
    for (int r = lane; r < B; r += 64) {
        float* row = stage + r * RW::N;
#pragma unroll
        for (int u = 0; u < RW::PAD; u += 4) {
            *reinterpret_cast<float4*>(row + RW::Z - RW::PAD + u) = make_float4(0.f, 0.f, 0.f, 0.f);
            *reinterpret_cast<float4*>(row + RW::Z + 8 + u) = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    const int njobs = jobs[0];
    for (int b = blockIdx.x; b < njobs; b += gridDim.x) {
        const int job = jobs[4 + 4 * b + 3];
        const int s_beg = jobs[4 + 4 * job + 1];
        const int n = jobs[4 + 4 * job + 2] - s_beg;
        const int seg = (n + NWAVE - 1) / NWAVE;
        const int q0 = min(n, wave * seg), q1 = min(n, q0 + seg);
        for (int p0 = 0; p0 < np; p0 += PPP) {
            const int nw = NC == 1 ? 1 : 2 * min(PPP, np - p0);   // columns of this pass
            for (int c = threadIdx.x; c < NC * PSUB; c += blockDim.x) tile[c] = 0.0;
            __syncthreads();
            // the column's accumulators, blocks base .. base + NB - 1; planes
            // ascend within a column, so base moves at most once (0 to 1,
            // after block 0 has gone to the tile)
            col3_v4 acc[NB][4];
#pragma unroll
            for (int tb = 0; tb < NB; ++tb)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) acc[tb][rb] = col3_v4{0.f, 0.f, 0.f, 0.f};
            int cur = -1;   // packed (x, y) first cell held in the accumulators
            int base = 0;
            // the pass's four columns: a group of the grouped layout, or
            // four columns of the rows
            const int cb = col0 + 2 * p0 + (NC == 1 ? 1 : 0);
            const float* wp = wrow + (gstride ? (cb >> 2) * gstride + (cb & 3) : (int64_t)cb) + (int64_t)s_beg * wstride;
            // the batch in registers: sample q0 + bt + sl; lane 63 also
            // holds the key of the sample after the batch (or ~0)
            uint32_t rkey = 0, rnext = ~0u;
            float rf[3] = {0.f, 0.f, 0.f}, rw[4] = {0.f, 0.f, 0.f, 0.f};
            auto fetch = [&](int bt) {
                const int q = bt + sl;
                if (q < q1) {
                    const int64_t si = (int64_t)s_beg + q;
                    rkey = loc[si];
#pragma unroll
                    for (int j = 0; j < 3; ++j) rf[j] = frac[3 * si + j];
                    if (hi)
#pragma unroll
                        for (int c = 0; c < 4; ++c) rw[c] = c < nw ? wp[(int64_t)q * wstride + c] : 0.f;
                }
                if (lane == 63) rnext = q + 1 < q1 ? loc[(int64_t)s_beg + q + 1] : ~0u;
            };
            fetch(q0);
            int ne = 0;
            for (int bt = q0; bt < q1; bt += ne) {
                const int nb = min(B, q1 - bt);
                // kernel values of the staged row (slots 12 hi .. 12 hi + 11),
                // then the weights
                {
                    float* row = stage + sl * RW::N;
                    float kv[12];
#pragma unroll
                    for (int u = 0; u < 12; ++u) {
                        const int s = 12 * hi + u;
                        const float f = s < 8 ? rf[0] : (s < 16 ? rf[1] : rf[2]);
                        kv[u] = kernel_value<float, KER>((float)col3_slot_offset(s) - f, W, kp);
                    }
                    if (!hi) {
#pragma unroll
                        for (int u = 0; u < 12; u += 4)
                            *reinterpret_cast<float4*>(row + u) = make_float4(kv[u], kv[u + 1], kv[u + 2], kv[u + 3]);
                    } else {
                        *reinterpret_cast<float4*>(row + 12) = make_float4(kv[0], kv[1], kv[2], kv[3]);
                        *reinterpret_cast<float4*>(row + RW::Z) = make_float4(kv[4], kv[5], kv[6], kv[7]);
                        *reinterpret_cast<float4*>(row + RW::Z + 4) = make_float4(kv[8], kv[9], kv[10], kv[11]);
                        *reinterpret_cast<float4*>(row + RW::W) = make_float4(rw[0], rw[1], rw[2], rw[3]);
                    }
                }
                const uint32_t keys = rkey;
                // runs of one first cell in the batch: bit l set where sample
                // l starts one
                const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute(4 * max(lane - 1, 0), (int)keys);
                const uint64_t starts = __builtin_amdgcn_ballot_w64(lane < nb && (lane == 0 || keys != prev));
                // a run that goes on past the batch leaves its last len % 4
                // samples to the next batch
                int defer = 0;
                if (nb == B && lane_value(rnext, 63) == lane_value(keys, B - 1))
                    defer = (nb - (63 - __builtin_clzll(starts))) & 3;
                ne = nb - defer;
                if (bt + ne < q1) fetch(bt + ne);   // next batch, in flight while this one is spread
                for (int i = 0; i < ne;) {
                    // one block step: up to four samples of one first cell
                    const uint32_t key0 = lane_value(keys, i);
                    const int xy = (int)(key0 & 0xFFFFFu);
                    const int z0 = (int)(key0 >> 20);
                    const int za = z0 / ZPB, zb = z0 % ZPB;
                    if (xy != cur || za != base) {
                        if (xy != cur) {
                            if (cur >= 0) col3_flush<NC, NB>(acc, tile, cur, base, lane);
#pragma unroll
                            for (int tb = 0; tb < NB; ++tb)
#pragma unroll
                                for (int rb = 0; rb < 4; ++rb) acc[tb][rb] = col3_v4{0.f, 0.f, 0.f, 0.f};
                        } else {
                            // the column moves on to planes past block base:
                            // that block is complete
                            col3_flush_first<NC>(acc, tile, cur, base, lane);
                        }
                        cur = xy;
                        base = za;
                    }
                    const uint64_t later = starts >> (i + 1);   // i < 32
                    const int run_end = later ? i + 1 + (int)__builtin_ctzll(later) : ne;
                    const int gsz = min(4, min(ne, run_end) - i);
                    // lanes past the step's samples read sample i's row (finite)
                    // and contribute zero A rows
                    const bool kin = k < gsz;
                    const float* row = stage + (i + (kin ? k : 0)) * RW::N;
                    const float px = row[ax];
                    const float4 py = *reinterpret_cast<const float4*>(row + 8 + 4 * ah);
                    const float wc = row[RW::W + bc];
                    const float* pz = row + RW::Z + bz - zb;
                    const float am = kin ? px : 0.f;
                    const float a[4] = {am * py.x, am * py.y, am * py.z, am * py.w};
                    // block base + t: plane offsets ZPB t + plane - zb (zero
                    // outside the window; zero for the last block when the
                    // window is block aligned)
#pragma unroll
                    for (int tb = 0; tb < NB; ++tb) {
                        // a block-aligned window (zb = 0, uniform over the
                        // wave) leaves the last block zero: its MFMAs are skipped
                        if (NB > 1 && tb == NB - 1 && zb == 0) break;
                        const float bv = pz[ZPB * tb] * wc;
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb)
                            acc[tb][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb], bv, acc[tb][rb], 0, 0, 0);
                    }
                    i += gsz;
                }
            }
            if (cur >= 0) col3_flush<NC, NB>(acc, tile, cur, base, lane);
            __syncthreads();
            // subgrid layout [job][pair][cell][re, im]
            if constexpr (NC == 1) {
                float* dst = subgrid + ((int64_t)job * np + p0) * NCELL * 2;
                for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
                    dst[2 * c] = 0.f;
                    dst[2 * c + 1] = (float)tile[c];
                }
            } else {
                for (int q = 0; 2 * q < nw; ++q) {
                    float* dst = subgrid + ((int64_t)job * np + p0 + q) * NCELL * 2;
                    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
                        dst[2 * c] = (float)tile[2 * q * PSUB + c];
                        dst[2 * c + 1] = (float)tile[(2 * q + 1) * PSUB + c];
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <int KER, int NC>
static void spread_col3(const Geo& g, const SpreadSrc& src, const uint32_t* loc, const void* frac,
                        const int32_t* jobs, unsigned nb, void* subgrid, hipStream_t s,
                        const long long* gate = nullptr, int gate_on = 0) {
    constexpr int PSUB = kCol3TileStride;
    constexpr int NT = NC <= 2 ? 1024 : 768;
    constexpr size_t lds =
        (size_t)NC * PSUB * sizeof(double) + (size_t)(NT / 64) * kCol3Batch * Col3Row<NC>::N * sizeof(float);
    static_assert(lds <= 160 * 1024, "tile and staging rows exceed the LDS of a workgroup");
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spread_col3<KER, NC, NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_spread_col3<KER, NC, NT><<<nb, NT, lds, s>>>(g, src.npairs, static_cast<const float*>(src.w[0].ptr),
                                                   (int)src.w[0].stride, src.w[0].gstride, (int)src.w[0].col, loc,
                                                   static_cast<const float*>(frac), jobs,
                                                   static_cast<float*>(subgrid), gate, gate_on);
}

template <int W, int KER, int NW>
static void spread_wave(const Geo& g, const SpreadSrc& src, const uint32_t* loc, const void* frac,
                        const int32_t* jobs, unsigned nb, void* subgrid, hipStream_t s) {
    constexpr int TS = spread_tile_edge(2, W);
    constexpr int PE = TS + W - 1;
    const size_t lds = (size_t)NW * PE * PE * sizeof(double);
    k_spread_wave<W, KER, NW><<<nb, 512, lds, s>>>(g, static_cast<const float*>(src.w[0].ptr),
                                                   (int)src.w[0].stride, (int)src.w[0].col, loc,
                                                   static_cast<const float*>(frac), jobs,
                                                   static_cast<float*>(subgrid));
}

template <int D, int W, typename T, int KER, int NWMAX>
static void spread_group(const Geo& g, const SpreadSrc& src, const uint32_t* loc, const void* frac,
                         const int32_t* jobs, unsigned nb, void* subgrid, hipStream_t s) {
    if constexpr (Foot<D, W>::ok && sizeof(T) == 4) {
        constexpr int TS = spread_tile_edge(D, W);
        constexpr int PE = TS + W - 1;
        constexpr int PSUB = D == 1 ? PE : (D == 2 ? PE * PE : PE * PE * PE);
        const size_t lds = (size_t)NWMAX * PSUB * sizeof(double) + GroupStage<D, W, T, NWMAX>::stage_bytes;
        if (lds > 65536)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spread_group<D, W, T, KER, NWMAX>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_spread_group<D, W, T, KER, NWMAX><<<nb, kSpreadBlock, lds, s>>>(
            g, src.npairs, static_cast<const T*>(src.w[0].ptr), (int)src.w[0].stride, (int)src.w[0].col, loc,
            static_cast<const T*>(frac), jobs, static_cast<T*>(subgrid));
    }
}

template <int D, int W, typename T, int KER>
static void spread_w(const Geo& g, const SpreadSrc& src, const uint32_t* loc, const void* frac,
                     const int32_t* perm, const int32_t* jobs, int64_t n_jobs_max, void* subgrid,
                     hipStream_t s) {
    if constexpr (spread_tile_edge(D, W) > 0) {
        const unsigned nb = (unsigned)std::min<int64_t>(n_jobs_max, 65535);
        if constexpr (Foot<D, W>::ok && sizeof(T) == 4) {
            // the group spread reads the staged rows directly: every source of
            // the launch is a column of the sorted weight rows, in order
            // (the one-sample-per-wave kernel reads them with scalar loads, so
            // two columns need only 8-byte rows; the lane-group kernels need
            // 16-byte aligned rows)
            const int al = ((D == 2 || D == 3) && W == 8 && src.npairs == 1) || (D == 2 && W < 8 && src.npairs == 1) ? 2 : 4;
            bool rows = src.w[0].kind == W_SORTED && (src.w[0].col % al) == 0 && (src.w[0].stride % al) == 0;
            for (int q = 1; q < 2 * src.npairs; ++q)
                rows = rows && src.w[q].kind == W_SORTED && src.w[q].ptr == src.w[0].ptr &&
                       src.w[q].col == src.w[0].col + q;
            if (rows) {
                const int nw = 2 * src.npairs;
                if constexpr (D == 2 && W <= 8) {
                    // four weight columns: the lane-group kernel (3 samples per
                    // wave step) wins; two or more than four: the
                    // one-sample-per-wave kernel (measured)
                    switch (nw) {
                        case 2: spread_wave<W, KER, 2>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                        case 4: spread_group<D, W, T, KER, 4>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                        case 6: spread_wave<W, KER, 6>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                        case 8: spread_wave<W, KER, 8>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                        case 10: spread_wave<W, KER, 10>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                        case 12: spread_wave<W, KER, 12>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                        case 14: spread_wave<W, KER, 14>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                        default: spread_wave<W, KER, 16>(g, src, loc, frac, jobs, nb, subgrid, s); break;
                    }
                    return;
                }
                if constexpr (D == 3 && W == 8) {
                    // columns per pass: four (a 108 KB FP64 tile), or two for
                    // one pair (two workgroups per CU)
                    if (src.npairs == 1 && src.keep_first) {
                        // the first column's moments may be kept (decided on the
                        // device): the pair, or only its second column
                        spread_col3<KER, 2>(g, src, loc, frac, jobs, nb, subgrid, s, src.keep_first, 0);
                        spread_col3<KER, 1>(g, src, loc, frac, jobs, nb, subgrid, s, src.keep_first, 1);
                    } else if (src.npairs == 1) {
                        spread_col3<KER, 2>(g, src, loc, frac, jobs, nb, subgrid, s);
                    } else {
                        spread_col3<KER, 4>(g, src, loc, frac, jobs, nb, subgrid, s);
                    }
                } else if constexpr (D == 3) {
                    spread_group<D, W, T, KER, 4>(g, src, loc, frac, jobs, nb, subgrid, s);
                } else {
                    if (nw <= 4) spread_group<D, W, T, KER, 4>(g, src, loc, frac, jobs, nb, subgrid, s);
                    else if (nw <= 8) spread_group<D, W, T, KER, 8>(g, src, loc, frac, jobs, nb, subgrid, s);
                    else spread_group<D, W, T, KER, 16>(g, src, loc, frac, jobs, nb, subgrid, s);
                }
                return;
            }
        }
        k_spread<D, W, T, KER><<<nb, kSpreadBlock, 0, s>>>(g, src, loc, static_cast<const T*>(frac),
                                                           perm, jobs, static_cast<T*>(subgrid));
    }
}

template <int D, typename T, int KER>
static void spread_d(const Geo& g, const SpreadSrc& src, const uint32_t* loc, const void* frac,
                     const int32_t* perm, const int32_t* jobs, int64_t n_jobs_max, void* subgrid,
                     hipStream_t s) {
    switch (g.w) {
        case 6: spread_w<D, 6, T, KER>(g, src, loc, frac, perm, jobs, n_jobs_max, subgrid, s); break;
        case 8: spread_w<D, 8, T, KER>(g, src, loc, frac, perm, jobs, n_jobs_max, subgrid, s); break;
        case 12: spread_w<D, 12, T, KER>(g, src, loc, frac, perm, jobs, n_jobs_max, subgrid, s); break;
        case 16: spread_w<D, 16, T, KER>(g, src, loc, frac, perm, jobs, n_jobs_max, subgrid, s); break;
        default: spread_w<D, 24, T, KER>(g, src, loc, frac, perm, jobs, n_jobs_max, subgrid, s); break;
    }
}

void launch_spread(const Geo& g, int prec, int kernel, const SpreadSrc& src, const uint32_t* loc,
                   const void* frac, const int32_t* perm, const int32_t* jobs, int64_t n_jobs_max,
                   void* subgrid, hipStream_t s) {
#define FKR_SPREAD(D, T, KER) spread_d<D, T, KER>(g, src, loc, frac, perm, jobs, n_jobs_max, subgrid, s)
#define FKR_SPREAD_K(D, T) do { if (kernel == FKR_KERNEL_ES) FKR_SPREAD(D, T, FKR_KERNEL_ES); else FKR_SPREAD(D, T, FKR_KERNEL_GAUSS); } while (0)
    if (prec == FKR_F64) {
        if (g.d == 1) FKR_SPREAD_K(1, double); else if (g.d == 2) FKR_SPREAD_K(2, double); else FKR_SPREAD_K(3, double);
    } else {
        if (g.d == 1) FKR_SPREAD_K(1, float); else if (g.d == 2) FKR_SPREAD_K(2, float); else FKR_SPREAD_K(3, float);
    }
#undef FKR_SPREAD_K
#undef FKR_SPREAD
}

FoldArgs fold_args(const Geo& g, int npairs, const int32_t* cover, const int32_t* job_off, const void* subgrid) {
    FoldArgs fa{};
    fa.cover = cover;
    fa.job_off = job_off;
    fa.subgrid = subgrid;
    fa.Psub = g.Psub;
    fa.np = npairs;
    fa.nt0 = g.nt[0]; fa.nt1 = g.nt[1];
    fa.pe0 = g.pe[0]; fa.pe1 = g.pe[1];
    for (int j = 0; j < 3; ++j) fa.Mr[j] = g.Mr[j];
    return fa;
}

void launch_fft(int prec, bool inverse, const FftPass& f0, const void* in, void* out, hipStream_t s) {
    FftPass f = f0;
    if (f.in_rdiv == 0) {   // contiguous input rows
        f.in_rdiv = 1;
        f.in_rmul = f.n_in;
        f.in_estride = 1;
    }
    const size_t csz = prec == FKR_F64 ? 16 : 8;
    // rows per workgroup (256 threads share them).  More rows lengthen the
    // runs of the strided loads but cost occupancy (two LDS buffers per
    // row).  Measured: up to 8192 rows (2-D grids) at most two rows per
    // workgroup, with 512 workgroups first; beyond (3-D grids) as many rows
    // as 32 KB of LDS holds (four FP64 rows of 180: 64-byte load runs), with
    // 1024 workgroups first.
    if (f.fold_d > 0 && !inverse) {
        // rows folded from the subgrids: one element per thread, so each
        // thread runs one fold chain; two rows per workgroup where they fit
        int Rf = 2;
        while (Rf > 1 && (Rf * f.F > 1024 || fft_lds_bytes(Rf, (int)f.F, csz) > 65536 || f.rows < (int64_t)Rf * 512)) Rf >>= 1;
        f.rows_per_block = Rf;
        // few rows (one pair): two threads per element halve each fold chain
        f.fold_split = (Rf == 1 && f.rows < 512 && 2 * f.F <= 1024) ? 1 : 0;
        const unsigned ntf = (unsigned)std::min<int64_t>(1024, ((1 + f.fold_split) * Rf * f.F + 63) / 64 * 64);
        const size_t ldsf = fft_lds_bytes(Rf, (int)f.F, csz);
        const unsigned nbf = (unsigned)((f.rows + Rf - 1) / Rf);
        if (nbf == 0) return;
#define FKR_FFTF(T, D, TS) k_fft<T, false, D, TS><<<nbf, ntf, ldsf, s>>>(nullptr, static_cast<typename V2<T>::t*>(out), f)
#define FKR_FFTF_D(T, TS) do { if (f.fold_d == 1) FKR_FFTF(T, 1, TS); else if (f.fold_d == 2) FKR_FFTF(T, 2, TS); else FKR_FFTF(T, 3, TS); } while (0)
        if (prec == FKR_F64) {
            if (f.fold_f64) FKR_FFTF_D(double, double); else FKR_FFTF_D(double, float);
        } else {
            FKR_FFTF_D(float, float);
        }
#undef FKR_FFTF_D
#undef FKR_FFTF
        return;
    }
    const bool many = f.rows > 8192;
    int R = many ? 64 : 2;
    while (R > 1 && fft_lds_bytes(R, (int)f.F, csz) > 32768) R >>= 1;
    while (R > 1 && f.rows < (int64_t)R * (many ? 1024 : 512)) R >>= 1;
    f.rows_per_block = R;
    const size_t lds = fft_lds_bytes(R, (int)f.F, csz);
    const unsigned nb = (unsigned)((f.rows + R - 1) / R);
    const unsigned nt = 256;
    if (nb == 0) return;
    if (prec == FKR_F64) {
        if (inverse) k_fft<double, true><<<nb, nt, lds, s>>>(static_cast<const double2*>(in), static_cast<double2*>(out), f);
        else k_fft<double, false><<<nb, nt, lds, s>>>(static_cast<const double2*>(in), static_cast<double2*>(out), f);
    } else {
        if (inverse) k_fft<float, true><<<nb, nt, lds, s>>>(static_cast<const float2*>(in), static_cast<float2*>(out), f);
        else k_fft<float, false><<<nb, nt, lds, s>>>(static_cast<const float2*>(in), static_cast<float2*>(out), f);
    }
}

void launch_solve2(int prec, const SolveArgs& a0, const int* pidx, const void* chan, hipStream_t s) {
    // Weight vectors per thread.  Small grids (2-D): three, so a call with
    // many weights runs several threads per grid point (the grid alone gives
    // few waves per CU).  Grids of a million points or more (3-D) have the
    // waves: up to 16 per thread, each factoring its point's matrix and
    // reading the density channels once for all of them (measured at
    // M = 128^3 with 11 weights: 0.51 ms with three, 0.34 ms with all).
    SolveArgs a = a0;
    a.wpg = a.Mtot >= (int64_t)1 << 20 ? std::min(16, std::max(1, a.nr - 1)) : 3;
    const unsigned ng = (unsigned)std::max(1, (a.nr - 1 + a.wpg - 1) / a.wpg);
    const dim3 nb(nblk(a.Mtot), ng);
#define FKR_SOLVE(P, T) k_solve<P, T><<<nb, 256, 0, s>>>(a, pidx, static_cast<const T*>(chan))
#define FKR_SOLVE_P(T) do { switch (a.P) { case 1: FKR_SOLVE(1, T); break; case 2: FKR_SOLVE(2, T); break; \
    case 3: FKR_SOLVE(3, T); break; case 4: FKR_SOLVE(4, T); break; case 6: FKR_SOLVE(6, T); break; \
    default: FKR_SOLVE(10, T); break; } } while (0)
    if (prec == FKR_F64) FKR_SOLVE_P(double); else FKR_SOLVE_P(float);
#undef FKR_SOLVE_P
#undef FKR_SOLVE
}

void launch_unpack_spec(int prec, int64_t Btot, const int64_t* B, int d, int npairs, int nw,
                        const void* spec, double* out, hipStream_t s) {
    const int64_t n = Btot * nw;
    if (n == 0) return;
    const int64_t b1 = d > 1 ? B[1] : 1, b2 = d > 2 ? B[2] : 1;
    if (prec == FKR_F64)
        k_unpack_spec<double><<<nblk(n), 256, 0, s>>>(Btot, d, B[0], b1, b2, npairs, nw, static_cast<const double2*>(spec), out);
    else
        k_unpack_spec<float><<<nblk(n), 256, 0, s>>>(Btot, d, B[0], b1, b2, npairs, nw, static_cast<const float2*>(spec), out);
}

void launch_chan_out(int prec, int64_t Mtot, int ncp, int n_s, int n_t, int nw, const void* chan,
                     double* S, double* T, hipStream_t s) {
    const int64_t n = Mtot * (n_s + n_t * nw);
    if (prec == FKR_F64)
        k_chan_out<double><<<nblk(n), 256, 0, s>>>(Mtot, ncp, n_s, n_t, nw, static_cast<const double*>(chan), S, T);
    else
        k_chan_out<float><<<nblk(n), 256, 0, s>>>(Mtot, ncp, n_s, n_t, nw, static_cast<const float*>(chan), S, T);
}

// Workgroups of a reduction launch: at most kRedBlocks, and no more than the
// device holds at once (a second, partly filled round of a register-heavy
// reduction would leave most CUs idle).
template <typename K>
static unsigned red_blocks(K kernel) {
    static std::mutex mu;
    static std::vector<std::pair<const void*, unsigned>> cache;   // per kernel (devices of one kind)
    std::lock_guard<std::mutex> lock(mu);
    const void* key = reinterpret_cast<const void*>(kernel);
    for (const auto& e : cache)
        if (e.first == key) return e.second;
    int per_cu = 0, dev = 0, ncu = 0;
    unsigned nb = kRedBlocks;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, key, 256, 0) == hipSuccess && per_cu > 0 && ncu > 0)
        nb = (unsigned)std::min<int64_t>(kRedBlocks, (int64_t)per_cu * ncu);
    cache.emplace_back(key, nb);
    return nb;
}

template <int PC>
static void reduce_cv_pc(const Geo& g, const ReduceCvArgs& a, hipStream_t s) {
#define FKR_RCV(D, TW, YR) k_reduce_cv<D, TW, PC, YR><<<red_blocks(&k_reduce_cv<D, TW, PC, YR>), 256, 0, s>>>(g, a)
    if (a.w_type == FKR_F64) {
        if (g.d == 1) FKR_RCV(1, double, false); else if (g.d == 2) FKR_RCV(2, double, false); else FKR_RCV(3, double, false);
    } else if (a.yrow) {
        if (g.d == 1) FKR_RCV(1, float, true); else if (g.d == 2) FKR_RCV(2, float, true); else FKR_RCV(3, float, true);
    } else {
        if (g.d == 1) FKR_RCV(1, float, false); else if (g.d == 2) FKR_RCV(2, float, false); else FKR_RCV(3, float, false);
    }
#undef FKR_RCV
}

void launch_reduce_cv(const Geo& g, const ReduceCvArgs& a, hipStream_t s) {
    // probes per launch rounded up to a compiled count
    if (a.np_launch <= 2) reduce_cv_pc<2>(g, a, s);
    else if (a.np_launch <= 4) reduce_cv_pc<4>(g, a, s);
    else if (a.np_launch <= 6) reduce_cv_pc<6>(g, a, s);
    else if (a.np_launch <= 8) reduce_cv_pc<8>(g, a, s);
    else if (a.np_launch <= 10) reduce_cv_pc<10>(g, a, s);
    else if (a.np_launch <= 12) reduce_cv_pc<12>(g, a, s);
    else reduce_cv_pc<16>(g, a, s);
}

void launch_reduce_final(const double* partial, int nslots, double* out, hipStream_t s) {
    if (nslots > 0) k_reduce_final<<<(unsigned)nslots, 256, 0, s>>>(partial, out);
}

void launch_interp(const Geo& g, int nv, const double* G, int64_t Nq, const void* X, int x_type,
                   double* out, hipStream_t s) {
    if (Nq == 0) return;
    switch (g.d) {
        case 1: k_interp<1><<<nblk(Nq), 256, 0, s>>>(g, nv, G, Nq, X, x_type, out); break;
        case 2: k_interp<2><<<nblk(Nq), 256, 0, s>>>(g, nv, G, Nq, X, x_type, out); break;
        default: k_interp<3><<<nblk(Nq), 256, 0, s>>>(g, nv, G, Nq, X, x_type, out); break;
    }
}

void launch_dsolve(int prec, const DSolveArgs& a, const int* pidx, const void* chan_base, const void* chan_der,
                   hipStream_t s) {
#define FKR_DS(P, T) k_dsolve<P, T><<<nblk(a.Mtot), 256, 0, s>>>(a, pidx, static_cast<const T*>(chan_base), \
                                                                 static_cast<const T*>(chan_der))
#define FKR_DS_P(T) do { switch (a.P) { case 1: FKR_DS(1, T); break; case 2: FKR_DS(2, T); break; \
    case 3: FKR_DS(3, T); break; case 4: FKR_DS(4, T); break; case 6: FKR_DS(6, T); break; \
    default: FKR_DS(10, T); break; } } while (0)
    if (prec == FKR_F64) FKR_DS_P(double); else FKR_DS_P(float);
#undef FKR_DS_P
#undef FKR_DS
}

void launch_grad_sums(const Geo& g, const GradSumArgs& a, hipStream_t s) {
#define FKR_GS(D, TW) k_grad_sums<D, TW><<<kRedBlocks, 256, 0, s>>>(g, a)
    if (a.w_type == FKR_F64) {
        if (g.d == 1) FKR_GS(1, double); else if (g.d == 2) FKR_GS(2, double); else FKR_GS(3, double);
    } else {
        if (g.d == 1) FKR_GS(1, float); else if (g.d == 2) FKR_GS(2, float); else FKR_GS(3, float);
    }
#undef FKR_GS
}

void launch_finalize_grad(int d, int ny, int Np, const double* red, const double* gred, double* gcv, double* dlogh,
                          hipStream_t s) {
    k_finalize_grad<<<1, 64, 0, s>>>(d, ny, Np, red, gred, gcv, dlogh);
}

void launch_adj_scatter(const Geo& g, int64_t N, int prec, const void* X, const void* W, int wstride,
                        int64_t wgstride, int ny, const double* yfit, const float* sup, double* u, hipStream_t s) {
    if (N == 0) return;
    // sorted coordinates and staged weights are both in the spreading precision
#define FKR_AS(D, TW) k_adj_scatter<D, TW><<<nblk(N), 256, 0, s>>>(g, N, prec, X, static_cast<const TW*>(W), \
                                                                  wstride, wgstride, ny, yfit, sup, u)
    if (prec == FKR_F64) {
        if (g.d == 1) FKR_AS(1, double); else if (g.d == 2) FKR_AS(2, double); else FKR_AS(3, double);
    } else {
        if (g.d == 1) FKR_AS(1, float); else if (g.d == 2) FKR_AS(2, float); else FKR_AS(3, float);
    }
#undef FKR_AS
}

void launch_adj_pack(int prec, int P, int64_t Mtot, const double* u, const double* c, int cplx, void* out,
                     hipStream_t s) {
    if (prec == FKR_F64) k_adj_pack<double><<<nblk(Mtot), 256, 0, s>>>(P, Mtot, u, c, cplx, static_cast<double2*>(out));
    else k_adj_pack<float><<<nblk(Mtot), 256, 0, s>>>(P, Mtot, u, c, cplx, static_cast<float2*>(out));
}

void launch_adj_combine(int prec, const ExpandArgs& a, int P, int cplx, const int* et, const double* fac,
                        const void* spec, void* out, hipStream_t s) {
    if (prec == FKR_F64)
        k_adj_combine<double><<<nblk(a.Btot), 256, 0, s>>>(a, P, cplx, et, fac, static_cast<const double2*>(spec),
                                                           static_cast<double2*>(out));
    else
        k_adj_combine<float><<<nblk(a.Btot), 256, 0, s>>>(a, P, cplx, et, fac, static_cast<const float2*>(spec),
                                                          static_cast<float2*>(out));
}

void launch_adj_combine_full(int prec, const ExpandArgs& a, const FullH& fh, int P, int cplx, const int* es,
                             const int* pidx, const double* fac, const void* spec, void* out, hipStream_t s) {
    const unsigned nb = (unsigned)((a.Btot + kExpandThreads - 1) / kExpandThreads);
    if (prec == FKR_F64)
        k_adj_combine_full<double><<<nb, kExpandThreads, 0, s>>>(a, fh, P, cplx, es, pidx, fac,
                                                                  static_cast<const double2*>(spec),
                                                                  static_cast<double2*>(out));
    else
        k_adj_combine_full<float><<<nb, kExpandThreads, 0, s>>>(a, fh, P, cplx, es, pidx, fac,
                                                                 static_cast<const float2*>(spec),
                                                                 static_cast<float2*>(out));
}

void launch_adj_gather(const Geo& g, int prec, int tprec, int kernel, int Np, int64_t n_jobs_max,
                       const int32_t* jobs, const uint32_t* loc, const void* frac, const void* X,
                       const int32_t* perm, const void* fgrid, int ny, int part, const double* yfit, const float* sup,
                       const void* W, int wstride, int64_t wgstride, const double* red, double* grad, hipStream_t s) {
    int64_t ps = 1;
    for (int j = 0; j < g.d; ++j) ps *= g.pe[j];
    const size_t lds = (size_t)ps * 8 * (part < 0 ? 2 : 1);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_jobs_max, 4096));
#define FKR_AG3(D, T, K, KT) do { if (lds > 65536) (void)hipFuncSetAttribute( \
        reinterpret_cast<const void*>(&k_adj_gather<D, T, K, KT>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        k_adj_gather<D, T, K, KT><<<nb, 256, lds, s>>>(g, Np, jobs, loc, \
        static_cast<const KT*>(frac), prec, X, perm, static_cast<const typename V2<T>::t*>(fgrid), ny, part, yfit, \
        sup, W, prec, wstride, wgstride, red, grad); } while (0)
#define FKR_AG(D, T, K) do { if (prec == FKR_F64) FKR_AG3(D, T, K, double); else FKR_AG3(D, T, K, float); } while (0)
#define FKR_AG_K(D, T) do { if (kernel == FKR_KERNEL_ES) FKR_AG(D, T, FKR_KERNEL_ES); else FKR_AG(D, T, FKR_KERNEL_GAUSS); } while (0)
#define FKR_AG_D(T) do { if (g.d == 1) FKR_AG_K(1, T); else if (g.d == 2) FKR_AG_K(2, T); else FKR_AG_K(3, T); } while (0)
    if (tprec == FKR_F64) FKR_AG_D(double); else FKR_AG_D(float);
#undef FKR_AG_D
#undef FKR_AG_K
#undef FKR_AG
#undef FKR_AG3
}

void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
    if (n > 0) k_fill_f64<<<nblk(n), 256, 0, s>>>(p, n, v);
}

void launch_stage_grid(const Geo& g, int prec, const PointsCheck& pc, const void* xs, const double* G, void* rows,
                       hipStream_t s) {
    if (pc.n == 0) return;
    const int rstride = resid_row_stride(g, prec);
#define FKR_SG(D, TW) k_stage_grid<D, TW><<<nblk(pc.n), 256, 0, s>>>(g, pc, prec, xs, G, static_cast<TW*>(rows), rstride)
    if (prec == FKR_F64) {
        if (g.d == 1) FKR_SG(1, double); else if (g.d == 2) FKR_SG(2, double); else FKR_SG(3, double);
    } else {
        if (g.d == 1) FKR_SG(1, float); else if (g.d == 2) FKR_SG(2, float); else FKR_SG(3, float);
    }
#undef FKR_SG
}

void launch_interval(int prec, const IntervalArgs& a, const void* chan, hipStream_t s) {
#define FKR_IV(P, T) k_interval<P, T><<<nblk(a.Mtot), 256, 0, s>>>(a, static_cast<const T*>(chan))
#define FKR_IV_P(T) do { switch (a.P) { case 1: FKR_IV(1, T); break; case 2: FKR_IV(2, T); break; \
    case 3: FKR_IV(3, T); break; case 4: FKR_IV(4, T); break; case 6: FKR_IV(6, T); break; \
    default: FKR_IV(10, T); break; } } while (0)
    if (prec == FKR_F64) FKR_IV_P(double); else FKR_IV_P(float);
#undef FKR_IV_P
#undef FKR_IV
}

void launch_spline(const Geo& g, int nv, const double* G, double* coef, hipStream_t s) {
    const int64_t M = g.Mtot;
    // array 0 of each block is the grid function itself
    k_copy_f64<<<nblk(M * nv), 256, 0, s>>>(G, coef, M, M, M << g.d, nv);
    int64_t st = 1;
    for (int j = 0; j < g.d; ++j) {
        const int64_t n = g.M[j];
        const int64_t nlines = M / n;
        const int64_t nthr = nlines * ((int64_t)1 << j) * nv;
        k_spline_line<<<nblk(nthr), 256, 0, s>>>(coef, M, g.d, j, n, st, nlines, nv);
        st *= n;
    }
}

void launch_spline_eval(const Geo& g, int nv, const double* coef, int64_t Nq, const void* X, int x_type,
                        double* out, hipStream_t s) {
    if (Nq == 0) return;
    switch (g.d) {
        case 1: k_spline_eval<1><<<nblk(Nq), 256, 0, s>>>(g, nv, coef, Nq, X, x_type, out); break;
        case 2: k_spline_eval<2><<<nblk(Nq), 256, 0, s>>>(g, nv, coef, Nq, X, x_type, out); break;
        default: k_spline_eval<3><<<nblk(Nq), 256, 0, s>>>(g, nv, coef, Nq, X, x_type, out); break;
    }
}

void launch_finalize_cv(int hidx, int Np, int q, const double* red, int n_items, int ny_cols,
                        const double* rho_in, double* rho_out, double* rss_out, double* gcv_out,
                        double* nused_out, hipStream_t s) {
    k_finalize_cv<<<1, 64, 0, s>>>(hidx, Np, q, red, n_items, ny_cols, rho_in, rho_out, rss_out, gcv_out,
                                   nused_out);
}

int resid_row_stride(const Geo& g, int prec) {
    // (1, z) rows of 8 bytes where the two-column spread is a
    // one-sample-per-wave kernel (FP32: 2-D with w <= 8, 3-D with w = 8),
    // else 16-byte rows
    return prec == FKR_F32 && ((g.d == 2 && g.w <= 8) || (g.d == 3 && g.w == 8)) ? 2 : 4;
}

void launch_resid(const Geo& g, int prec, int mode, const PointsCheck& pc, int x_type, const void* xs,
                  const int32_t* perm, int y_type, const void* Y, int y_cplx, const double* mhat, double* r_out,
                  void* rows, hipStream_t s) {
    launch_zero(pc.diag + kDiagResidExcl, 8, s);
    if (pc.n == 0) return;
    const int rstride = resid_row_stride(g, prec);
#define FKR_RES(D, TW) k_resid<D, TW><<<nblk(pc.n), 256, 0, s>>>(g, mode, pc, x_type, xs, perm, y_type, Y, y_cplx, \
                                                                 mhat, r_out, static_cast<TW*>(rows), rstride)
    if (prec == FKR_F64) {
        if (g.d == 1) FKR_RES(1, double); else if (g.d == 2) FKR_RES(2, double); else FKR_RES(3, double);
    } else {
        if (g.d == 1) FKR_RES(1, float); else if (g.d == 2) FKR_RES(2, float); else FKR_RES(3, float);
    }
#undef FKR_RES
}

void launch_kappa_partial(const Geo& g, int64_t N, int x_type, const void* xs, const int32_t* perm,
                          const double* vhat, const double* r, double* partial, hipStream_t s) {
    switch (g.d) {
        case 1: k_kappa_partial<1><<<kRedBlocks, 256, 0, s>>>(g, N, x_type, xs, perm, vhat, r, partial); break;
        case 2: k_kappa_partial<2><<<kRedBlocks, 256, 0, s>>>(g, N, x_type, xs, perm, vhat, r, partial); break;
        default: k_kappa_partial<3><<<kRedBlocks, 256, 0, s>>>(g, N, x_type, xs, perm, vhat, r, partial); break;
    }
}

void launch_sigma2(int64_t Mtot, const double* vhat, const double* kappa_sums, double* sigma2,
                   double* kappa_out, hipStream_t s) {
    k_sigma2<<<nblk(Mtot), 256, 0, s>>>(Mtot, vhat, kappa_sums, sigma2, kappa_out);
}

}  // namespace fkr
