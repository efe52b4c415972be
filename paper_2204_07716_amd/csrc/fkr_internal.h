// Internal definitions shared by the host planner, the launchers and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/fkr.h"

namespace fkr {

constexpr int kMaxD = FKR_MAX_D;
constexpr int kMaxFactors = 20;      // radix stages of one FFT length
constexpr int kMaxChannels = 36;     // s-channels C(d+2l, 2l) <= 35 for d <= 3, l <= 2
constexpr int kMaxP = 10;            // P = C(d+l, l) <= 10
constexpr int kMaxBatchLanes = 16;   // plans (and streams) of one batch
constexpr int kCoverSlots = 5;       // spreading tiles covering one fine cell (per dimension)
constexpr int kMaxW = 24;            // widest spreading kernel (fine cells)

// Spreading kernel widths compiled into the library; the planner rounds the
// width it derives from eps up to the next one.
constexpr int kWidths[] = {6, 8, 12, 16, 24};

// Interior edge of a spreading tile (fine cells) for dimension D and kernel
// width W; 0 when unsupported.  One workgroup spreads all samples of one tile
// into the padded tile (TS + W - 1)^D, accumulated in FP64 in LDS, so tiles
// are small (many workgroups, no partial tiles to add up).
constexpr int spread_tile_edge(int D, int W) {
    return D <= 2 ? 8 : (W <= 8 ? 8 : (W <= 16 ? 4 : 0));
}

constexpr int kMaxPairsInLaunch = 8;   // weight pairs per spreading launch
constexpr int kSpreadThreads = 256;
constexpr int kRedThreads = 256;

// One FFT length: factorisation into radix stages (4, 2, 3, 5).
struct FftLen {
    int64_t n = 0;
    int nfac = 0;
    int fac[kMaxFactors] = {0};
    size_t tw_off = 0;               // byte offset of its twiddle table in the workspace
};

struct Layout {                      // byte offsets into the workspace
    size_t consts = 0;               // periods (3 doubles), then int32 tables es, et, pidx
    size_t deconv = 0;               // per dim: B_j doubles (1 / psi_hat)
    size_t cover = 0;                // per dim: Mr_j * (1 + 2*kCoverSlots) int32
    size_t diag = 0;                 // int64 counters
    size_t trec = 0, bhist = 0, obuf = 0;   // tile-ordered records, block x tile counts, outside counts per binning block
    size_t counts = 0, tile_off = 0, cursor = 0, job_off = 0, jobs = 0;
    size_t loc = 0, frac = 0, perm = 0, xs = 0;
    size_t subgrid = 0, fftA = 0, fftB = 0, spec = 0;
    size_t chan = 0, mhat = 0, partial = 0, wbuf = 0, red = 0, wsort = 0;
    size_t sup = 0;                  // [M] FP32 resolved flags (0 / NaN) of the last solve
    size_t r0 = 0;                   // [P][M] FP64 row 0 of the equilibrated inverse (variance of the fit)
    size_t ktab = 0;                 // compact kernels: per dim [2 l + 1][B_j] FP64 moment multipliers
    size_t total = 0;
    // element capacities (for checks)
    int64_t cap_jobs = 0, cap_fft = 0, cap_spec = 0, cap_chan = 0, cap_mhat = 0;
    int64_t cap_partial = 0, cap_wbuf = 0;
};

}  // namespace fkr

struct fkr_plan {
    fkr_plan_desc desc{};
    int d = 0, order = 0, n_s = 0, n_t = 0;
    int prec = FKR_F64;              // spreading precision (FKR_F32 / FKR_F64)
    int tprec = FKR_F64;             // transform / channel precision
    int kernel = FKR_KERNEL_ES;
    int64_t M[fkr::kMaxD] = {1, 1, 1};
    int64_t L[fkr::kMaxD] = {1, 1, 1};
    int64_t K[fkr::kMaxD] = {0, 0, 0};
    int64_t B[fkr::kMaxD] = {1, 1, 1};     // 2K + 1
    int64_t Mr[fkr::kMaxD] = {1, 1, 1};
    int64_t ts[fkr::kMaxD] = {1, 1, 1};    // tile edge (fine cells)
    int64_t nt[fkr::kMaxD] = {1, 1, 1};    // tiles per dimension
    int64_t pe[fkr::kMaxD] = {1, 1, 1};    // padded tile edge ts + w - 1
    double lo[fkr::kMaxD] = {0, 0, 0}, hi[fkr::kMaxD] = {0, 0, 0};
    double delta[fkr::kMaxD] = {1, 1, 1}, T[fkr::kMaxD] = {1, 1, 1};
    double hf[fkr::kMaxD] = {1, 1, 1}, inv_hf[fkr::kMaxD] = {1, 1, 1};
    double h_min[fkr::kMaxD] = {0, 0, 0}, h_max[fkr::kMaxD] = {0, 0, 0};
    double eps = 0, sigma = 2.0, U_spec = 0, U_space = 0;
    int reg_kernel = 0;              // FKR_REG_*: 0 the Gaussian, else a compact kernel on |u| <= 1
    int w = 0;
    double kparam = 0;               // ES beta or Gaussian a
    int64_t n_tiles = 1, Psub = 1, Mtot = 1, Btot = 1, Mrtot = 1;
    int tsp = 1, ncell = 1;          // tile pitch of cell ids, cells per tile
    int chunk = 4096;
    int pairs_per_spread = 1;
    int64_t n_max = 0;
    int max_weights = 1, max_h = 1, npairs_max = 1, ncp_max = 1;
    int64_t n_jobs_max = 1;
    int64_t chunk_min = 1;   // the chunk the job table was sized for; a batch may lengthen jobs beyond it
    int es[fkr::kMaxChannels][fkr::kMaxD] = {};   // s-channel exponents
    int et[fkr::kMaxChannels][fkr::kMaxD] = {};   // t-channel exponents
    int pair_index[fkr::kMaxP][fkr::kMaxP] = {};  // s-channel of et[b] + et[c]
    fkr::FftLen fMr[fkr::kMaxD], fL[fkr::kMaxD];
    std::vector<double> deconv[fkr::kMaxD];
    std::vector<int32_t> cover[fkr::kMaxD];
    int max_cover = 0;                     // most padded tiles covering one fine cell in one dimension
    fkr::Layout lay;
    // state
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_ready = false;
    bool points_set = false;
    int64_t N = 0;
    // fkr_set_points calls so far; the sort writes it to the device, and the
    // kernels that index a caller's arrays through the sort permutation
    // check it there (a replayed HIP graph may have re-sorted other points)
    long long epoch = 0;
    void* last_stream = nullptr;
    // constant tables as (workspace offset, bytes), kept for the
    // asynchronous uploads of fkr_fit_noalloc (their source must outlive the
    // copies queued on the stream)
    std::vector<std::pair<size_t, std::vector<unsigned char>>> const_blobs;
    // stage timing (fkr_profile_enable / fkr_profile_read)
    bool prof_on = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs[FKR_N_STAGES];
    ~fkr_plan() {
        for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
        for (auto& v : ev_pairs)
            for (auto& e : v) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    }
};

namespace fkr {

size_t elem_size(int type);
int64_t smooth_up(int64_t n);                   // next 2^a 3^b 5^c >= n
bool factorise(int64_t n, FftLen* out);
fkr_status build_plan(const fkr_plan_desc* desc, fkr_plan* p);
void twiddle_table(int64_t n, std::vector<double>* re_im);
double es_kernel_hat(double xi, int w, double beta);

}  // namespace fkr
