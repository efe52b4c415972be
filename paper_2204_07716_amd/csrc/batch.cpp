// Batches of independent regressions (declared in fkr.h): several plans,
// each with its own HIP stream and slice of one workspace, fed from one call.
// The batch forks from the caller's stream with an event and joins back with
// one event per lane, so the whole batch is enqueued (or captured into one
// HIP graph) by one call, and regressions on different lanes run
// concurrently.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <vector>

#include "fkr_internal.h"
#include "kernels.h"

using namespace fkr;

struct fkr_batch {
    fkr_plan_desc desc{};
    int n_lanes = 0;
    int lanes_used = 0;
    std::vector<fkr_plan*> plans;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    hipEvent_t start = nullptr;
    size_t slice = 0;           // workspace bytes per lane (256-aligned)
    bool ws_ready = false;
    ~fkr_batch() {
        for (fkr_plan* p : plans) fkr_plan_destroy(p);
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
        for (hipEvent_t e : done) (void)hipEventDestroy(e);
        if (start) (void)hipEventDestroy(start);
    }
};

namespace {

struct Shape {
    int R, nh, q, cpl, Np, d;
    int64_t Mtot;
    size_t xsz, ysz;
};

// Largest-first assignment of regressions to lanes by an estimated cost of
// N + 4 M samples (the grid-sized work of a regression -- transforms, solves
// -- counted as that many samples), each to the lane with the least work so
// far.  Lane lists keep the assignment order.
std::vector<std::vector<int>> schedule(const int64_t* off, int R, int lanes, int64_t Mtot) {
    std::vector<int> order(R);
    std::iota(order.begin(), order.end(), 0);
    auto n_of = [&](int r) { return off[r + 1] - off[r]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n_of(a) > n_of(b); });
    std::vector<std::vector<int>> out(lanes);
    std::vector<double> load(lanes, 0.0);
    for (int r : order) {
        if (n_of(r) == 0) continue;
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        out[l].push_back(r);
        load[l] += (double)n_of(r) + 4.0 * (double)Mtot;
    }
    return out;
}

fkr_status enqueue(fkr_batch* b, const int64_t* off, const void* X, int x_type, const double* h,
                   const void* Y, int y_type, int y_complex, uint64_t seed, const Shape& sh, double* mhat,
                   double* rho, double* rss, double* gcv, double* nused, hipStream_t s) {
    // regressions without samples: NaN fits, ratios and GCV, zero RSS and N_I
    for (int r = 0; r < sh.R; ++r) {
        if (off[r + 1] > off[r]) continue;
        const int64_t nm = (int64_t)sh.nh * sh.q * sh.cpl * sh.Mtot;
        if (mhat) launch_fill_f64(mhat + r * nm, nm, NAN, s);
        if (rho) launch_fill_f64(rho + (int64_t)r * sh.nh * sh.Np, (int64_t)sh.nh * sh.Np, NAN, s);
        if (rss) launch_fill_f64(rss + (int64_t)r * sh.nh * sh.q, (int64_t)sh.nh * sh.q, 0.0, s);
        if (gcv) launch_fill_f64(gcv + (int64_t)r * sh.nh * sh.q, (int64_t)sh.nh * sh.q, NAN, s);
        if (nused) launch_fill_f64(nused + (int64_t)r * sh.nh, sh.nh, 0.0, s);
    }
    const int lanes = b->lanes_used;
    const auto plan_lists = schedule(off, sh.R, lanes, sh.Mtot);
    if (hipEventRecord(b->start, s) != hipSuccess) return FKR_E_DEVICE;
    for (int l = 0; l < lanes; ++l) {
        if (plan_lists[l].empty()) continue;
        hipStream_t ls = b->streams[l];
        if (hipStreamWaitEvent(ls, b->start, 0) != hipSuccess) return FKR_E_DEVICE;
        for (int r : plan_lists[l]) {
            const int64_t n = off[r + 1] - off[r];
            const char* xr = static_cast<const char*>(X) + (size_t)off[r] * sh.d * sh.xsz;
            const char* yr = static_cast<const char*>(Y) + (size_t)off[r] * sh.q * sh.cpl * sh.ysz;
            fkr_status st = fkr_set_points(b->plans[l], n, xr, x_type, ls);
            if (st != FKR_OK) return st;
            const int64_t nm = (int64_t)sh.nh * sh.q * sh.cpl * sh.Mtot;
            st = fkr_cv(b->plans[l], sh.nh, h, sh.q, y_complex, yr, y_type, sh.Np, seed + (uint64_t)r, nullptr,
                        mhat ? mhat + r * nm : nullptr, rho ? rho + (int64_t)r * sh.nh * sh.Np : nullptr,
                        rss ? rss + (int64_t)r * sh.nh * sh.q : nullptr,
                        gcv ? gcv + (int64_t)r * sh.nh * sh.q : nullptr, nused ? nused + (int64_t)r * sh.nh : nullptr,
                        ls);
            if (st != FKR_OK) return st;
        }
        if (hipEventRecord(b->done[l], ls) != hipSuccess) return FKR_E_DEVICE;
        if (hipStreamWaitEvent(s, b->done[l], 0) != hipSuccess) return FKR_E_DEVICE;
    }
    return FKR_OK;
}

fkr_status check_call(fkr_batch* b, int R, const int64_t* off, const void* X, int x_type, int nh,
                      const double* h, int q, int y_complex, const void* Y, int y_type, int Np, Shape* sh) {
    if (!b) return FKR_E_ARG;
    if (!b->ws_ready) return FKR_E_WORKSPACE;
    if (R < 1 || !off || off[0] != 0) return FKR_E_ARG;
    if (x_type != FKR_F32 && x_type != FKR_F64) return FKR_E_ARG;
    if (y_type != FKR_F32 && y_type != FKR_F64) return FKR_E_ARG;
    if (q < 1 || (y_complex != 0 && y_complex != 1) || Np < 1 || nh < 1 || !h) return FKR_E_ARG;
    for (int r = 0; r < R; ++r)
        if (off[r + 1] < off[r] || off[r + 1] - off[r] > b->desc.n_max) return FKR_E_ARG;
    if (off[R] > 0 && (!X || !Y)) return FKR_E_ARG;
    const int cpl = y_complex ? 2 : 1;
    if (1 + q * cpl + Np > b->desc.max_weights || nh > b->desc.max_h) return FKR_E_ARG;
    // the bandwidths are checked here, so that no lane's call can fail after the fork
    for (int k = 0; k < nh * b->desc.d; ++k) {
        const int j = k % b->desc.d;
        if (!(h[k] >= b->desc.h_min[j] * (1 - 1e-12) && h[k] <= b->desc.h_max[j] * (1 + 1e-12))) return FKR_E_ARG;
    }
    sh->R = R; sh->nh = nh; sh->q = q; sh->cpl = cpl; sh->Np = Np; sh->d = b->desc.d;
    sh->Mtot = b->plans[0]->Mtot;
    sh->xsz = x_type == FKR_F64 ? 8 : 4;
    sh->ysz = y_type == FKR_F64 ? 8 : 4;
    return FKR_OK;
}

}  // namespace

extern "C" {

fkr_status fkr_batch_create(const fkr_plan_desc* desc, int n_lanes, fkr_batch** out) {
    if (!desc || !out || n_lanes < 1 || n_lanes > kMaxBatchLanes) return FKR_E_ARG;
    *out = nullptr;
    fkr_batch* b = new (std::nothrow) fkr_batch();
    if (!b) return FKR_E_ARG;
    b->desc = *desc;
    b->n_lanes = b->lanes_used = n_lanes;
    for (int l = 0; l < n_lanes; ++l) {
        fkr_plan* p = nullptr;
        const fkr_status st = fkr_plan_create(desc, &p);
        if (st != FKR_OK) { delete b; return st; }
        b->plans.push_back(p);
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        // default priority, non-blocking with respect to the null stream
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) { delete b; return FKR_E_DEVICE; }
        b->streams.push_back(s);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { delete b; return FKR_E_DEVICE; }
        b->done.push_back(e);
    }
    if (hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess) { delete b; return FKR_E_DEVICE; }
    size_t ws = 0;
    fkr_workspace_size(b->plans[0], &ws);
    b->slice = (ws + 255) & ~(size_t)255;
    *out = b;
    return FKR_OK;
}

void fkr_batch_destroy(fkr_batch* b) { delete b; }

fkr_status fkr_batch_workspace_size(const fkr_batch* b, size_t* bytes) {
    if (!b || !bytes) return FKR_E_ARG;
    *bytes = b->slice * b->n_lanes;
    return FKR_OK;
}

fkr_status fkr_batch_set_workspace(fkr_batch* b, void* ws, size_t bytes) {
    if (!b || !ws) return FKR_E_ARG;
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0 || bytes < b->slice * b->n_lanes) return FKR_E_WORKSPACE;
    for (int l = 0; l < b->n_lanes; ++l) {
        const fkr_status st = fkr_set_workspace(b->plans[l], static_cast<char*>(ws) + l * b->slice, b->slice);
        if (st != FKR_OK) return st;
    }
    b->ws_ready = true;
    return FKR_OK;
}

fkr_status fkr_batch_cv(fkr_batch* b, int R, const int64_t* off, const void* X, int x_type, int nh,
                        const double* h, int q, int y_complex, const void* Y, int y_type, int Np, uint64_t seed,
                        double* mhat, double* rho, double* rss, double* gcv, double* nused, void* stream) {
    Shape sh{};
    fkr_status st = check_call(b, R, off, X, x_type, nh, h, q, y_complex, Y, y_type, Np, &sh);
    if (st != FKR_OK) return st;
    return enqueue(b, off, X, x_type, h, Y, y_type, y_complex, seed, sh, mhat, rho, rss, gcv, nused,
                   static_cast<hipStream_t>(stream));
}

fkr_status fkr_batch_tune(fkr_batch* b, int R, const int64_t* off, const void* X, int x_type, int nh,
                          const double* h, int q, int y_complex, const void* Y, int y_type, int Np,
                          uint64_t seed, int reps, int* lanes_out, int64_t* chunk_out, double* ms_out,
                          void* stream) {
    Shape sh{};
    fkr_status st = check_call(b, R, off, X, x_type, nh, h, q, y_complex, Y, y_type, Np, &sh);
    if (st != FKR_OK) return st;
    if (reps < 1) return FKR_E_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return FKR_E_STATE;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return FKR_E_DEVICE;
    // candidates: lanes 1, 2, 4, .. n_lanes; in 1-D and 2-D, job chunks 1, 2
    // and 4 times the plan's own (the job table holds as many jobs as the
    // plan's chunk needs, so longer jobs always fit; 3-D jobs stay sized for
    // the LDS staging of the cell sort)
    const int64_t base_chunk = b->plans[0]->chunk_min;
    const int n_chunk = b->desc.d <= 2 ? 3 : 1;
    std::vector<int> lane_c;
    for (int l = 1; l < b->n_lanes; l *= 2) lane_c.push_back(l);
    lane_c.push_back(b->n_lanes);
    double best = INFINITY;
    int best_l = b->n_lanes;
    int64_t best_c = base_chunk;
    for (int ci = 0; ci < n_chunk; ++ci) {
        const int64_t c = base_chunk << ci;
        for (fkr_plan* p : b->plans) p->chunk = (int)c;
        for (int l : lane_c) {
            b->lanes_used = l;
            st = enqueue(b, off, X, x_type, h, Y, y_type, y_complex, seed, sh, nullptr, nullptr, nullptr,
                         nullptr, nullptr, s);   // warm-up
            if (st != FKR_OK) break;
            (void)hipEventRecord(t0, s);
            for (int k = 0; k < reps && st == FKR_OK; ++k)
                st = enqueue(b, off, X, x_type, h, Y, y_type, y_complex, seed, sh, nullptr, nullptr, nullptr,
                             nullptr, nullptr, s);
            (void)hipEventRecord(t1, s);
            if (st != FKR_OK || hipEventSynchronize(t1) != hipSuccess) break;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, t0, t1);
            const double per = ms / reps;
            if (per < best) { best = per; best_l = l; best_c = c; }
        }
        if (st != FKR_OK) break;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    for (fkr_plan* p : b->plans) p->chunk = (int)best_c;
    b->lanes_used = best_l;
    if (st != FKR_OK) return st;
    if (lanes_out) *lanes_out = best_l;
    if (chunk_out) *chunk_out = best_c;
    if (ms_out) *ms_out = best;
    return FKR_OK;
}

fkr_status fkr_batch_config(fkr_batch* b, int lanes, int64_t chunk) {
    if (!b || lanes < 1 || lanes > b->n_lanes) return FKR_E_ARG;
    if (chunk != 0 && (b->desc.d > 2 || chunk < b->plans[0]->chunk_min || chunk > (int64_t)1 << 20))
        return FKR_E_ARG;
    b->lanes_used = lanes;
    if (chunk != 0)
        for (fkr_plan* p : b->plans) p->chunk = (int)chunk;
    return FKR_OK;
}

}  // extern "C"
