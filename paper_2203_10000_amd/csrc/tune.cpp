// Launch-shape tuner for the pair loop: points per lane x wavefronts per
// workgroup, timed on the device the first time a (device, precision,
// triangle-count bucket, point-count bucket) is seen, then cached for the
// process (and in the file named by SAL_TUNE_CACHE, if set).  Point counts
// at or above the trial size share one bucket.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>

#include "runtime.h"
#include "tune_cache.h"

namespace sal {
namespace {

using Key = TuneKey;

std::mutex g_mu;
TuneMap g_cache;
bool g_loaded = false;

constexpr int64_t kTrialPoints = (int64_t)1 << 19;   // enough workgroups to fill the device

int bucket(int64_t v) {
    int b = 0;
    while (v > 1 && b < 62) {
        v >>= 1;
        ++b;
    }
    return b;
}

std::string arch_name(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    return std::string(p.gcnArchName);
}

void load_file() {
    g_loaded = true;
    const char *path = std::getenv("SAL_TUNE_CACHE");
    if (path) tune_cache_read(path, &g_cache);
}

void save_file() {
    const char *path = std::getenv("SAL_TUNE_CACHE");
    if (path) tune_cache_write(path, g_cache);
}

}  // namespace

// Fills opt->points_per_lane / opt->block_waves when they are 0 (auto).
sal_status tune_launch(sal_context *ctx, const sal_surface_set *set, int64_t n, const float *x,
                       const float *y, const float *z, int32_t *labels, sal_label_options *opt) {
    const bool fp64 = opt->precision == SAL_PREC_FP64;
    if (fp64) opt->points_per_lane = 1;
    if (opt->points_per_lane != 0 && opt->block_waves != 0) return SAL_OK;
    const char *off = std::getenv("SAL_TUNE");
    if ((off && std::strcmp(off, "0") == 0) || n <= 0) {
        if (opt->points_per_lane == 0) opt->points_per_lane = 1;
        if (opt->block_waves == 0) opt->block_waves = 4;
        return SAL_OK;
    }
    // The trials use at most kTrialPoints points, so every larger count runs
    // the same trials: those counts share one entry.
    const Key key(ctx->device, opt->precision, bucket(set->n_tri),
                  bucket(n < kTrialPoints ? n : kTrialPoints), arch_name(ctx->device),
                  opt->points_per_lane, opt->block_waves);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_loaded) load_file();
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            if (opt->points_per_lane == 0) opt->points_per_lane = it->second.first;
            if (opt->block_waves == 0) opt->block_waves = it->second.second;
            return SAL_OK;
        }
    }
    // Trial launches of the pair loop alone on a prefix of the points (enough
    // workgroups to fill the device several times) against the tuner's strip
    // prefix, writing labels that the real launch overwrites.
    const int64_t trial_n = n < kTrialPoints ? n : kTrialPoints;
    PairloopArgs a{};
    a.rec32 = set->rec32;
    a.rec64 = set->rec64;
    a.n_surf = 1;
    a.x = x;
    a.y = y;
    a.z = z;
    a.n = trial_n;
    a.kappa = (float)opt->kappa;
    a.threshold = opt->threshold;
    a.band = opt->recheck_band;
    a.labels = labels;
    a.winding = nullptr;
    a.winding_type = SAL_WINDING_NONE;
    a.flag_list = ctx->flag_list;      // overwritten by the real launch
    a.counters = ctx->tune_counters;   // the call's own counters stay untouched
    // Candidate shapes (those the caller left open).
    struct Shape {
        int p, b;
        float ms;
    };
    Shape cand[12];
    int nc = 0;
    const int ppls[3] = {1, 2, 4};
    const int bws[4] = {1, 2, 4, 8};
    for (int pi = 0; pi < (fp64 ? 1 : 3); ++pi) {
        const int p = fp64 ? 1 : ppls[pi];
        if (opt->points_per_lane != 0 && opt->points_per_lane != p) continue;
        for (int b : bws) {
            if (opt->block_waves != 0 && opt->block_waves != b) continue;
            cand[nc++] = Shape{p, b, 0.0f};
        }
    }
    // Fastest of `reps` launches of one shape against tuner surface `entry`.
    auto time_shape = [&](const Shape &sh, int entry, int reps, float *out) -> sal_status {
        a.surf = set->tune_surf + entry;
        float t_min = 1e30f;
        for (int rep = 0; rep < reps; ++rep) {
            SAL_HIP(launch_fill_u64(ctx->tune_counters, 0ull, kNumCounters, ctx->stream));
            SAL_HIP(hipEventRecord(ctx->ev[5], ctx->stream));
            SAL_HIP(fp64 ? launch_pairloop_f64(a, sh.b, ctx->stream)
                         : launch_pairloop_f32(a, sh.p, sh.b, ctx->stream));
            SAL_HIP(hipEventRecord(ctx->ev[6], ctx->stream));
            SAL_HIP(hipEventSynchronize(ctx->ev[6]));
            float ms = 0.0f;
            SAL_HIP(hipEventElapsedTime(&ms, ctx->ev[5], ctx->ev[6]));
            if (ms < t_min) t_min = ms;
        }
        *out = t_min;
        return SAL_OK;
    };
    sal_status ts;
    // Float32 with more than two shapes open: screen every shape once on the
    // short prefix (a quarter of the pairs), then time the two fastest twice
    // on the full trial prefix.  In the full trials of the c2 and c3 surface
    // sets the one-point shapes with 2-8 wavefronts per workgroup were within
    // 2 % of each other and every other shape 5-35 % slower, so two
    // finalists keep the choice while the tuning costs ~80 ms instead of
    // ~300 ms.
    int n_final = nc;
    if (!fp64 && nc > 2) {
        // one untimed launch first, so that the first screened shape does not
        // also pay for the device warming up
        float warm = 0.0f;
        if ((ts = time_shape(cand[0], 2, 1, &warm)) != SAL_OK) return ts;
        for (int k = 0; k < nc; ++k)
            if ((ts = time_shape(cand[k], 2, 1, &cand[k].ms)) != SAL_OK) return ts;
        for (int k = 0; k < 2; ++k)   // the two fastest to the front, in order
            for (int j = k + 1; j < nc; ++j)
                if (cand[j].ms < cand[k].ms) std::swap(cand[j], cand[k]);
        n_final = 2;
    }
    float best = 1e30f;
    int best_p = 1, best_b = 4;
    for (int k = 0; k < n_final; ++k) {
        float t = 0.0f;
        if ((ts = time_shape(cand[k], fp64 ? 1 : 0, 2, &t)) != SAL_OK) return ts;
        if (t < best) {
            best = t;
            best_p = cand[k].p;
            best_b = cand[k].b;
        }
    }
    if (opt->points_per_lane == 0) opt->points_per_lane = best_p;
    if (opt->block_waves == 0) opt->block_waves = best_b;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = {opt->points_per_lane, opt->block_waves};
    save_file();
    return SAL_OK;
}

}  // namespace sal
