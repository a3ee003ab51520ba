// sal_label_points_noalloc: point labeling for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  The
// same kernels as sal_label_points; their scratch (counters, flag list,
// recheck buffers) lives in one file-scope device array instead of the
// context's growable buffers.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "runtime.h"

namespace sal {
namespace {

constexpr int64_t kNoAllocMaxPoints = (int64_t)1 << 20;
constexpr int64_t kNoAllocPairCap = kNoAllocMaxPoints / 4 + 64 * kMaxSurfaces;

constexpr int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

// Byte offsets of the parts of the scratch array.
constexpr int64_t kOffCounters = 0;
constexpr int64_t kOffFlags = align256(kOffCounters + kNumCounters * 8);
constexpr int64_t kOffRes = align256(kOffFlags + kNoAllocMaxPoints * (int64_t)sizeof(FlagEntry));
constexpr int64_t kOffPairs = align256(kOffRes + kNoAllocMaxPoints * 8);
constexpr int64_t kOffOut = align256(kOffPairs + kNoAllocPairCap * (int64_t)sizeof(RecheckPair));
constexpr int64_t kOffSeg = align256(kOffOut + kNoAllocPairCap * (int64_t)sizeof(RecheckOut));
constexpr int64_t kScratchBytes = align256(kOffSeg + (int64_t)sizeof(RecheckSeg));

// ~38 MB per device, held until the process ends.  Host code must never pass
// this name to a kernel: on the host it is only a stand-in for the symbol;
// the device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
bool g_looked_up[kMaxDevices] = {};

}  // namespace

// Looked up once per device, with that device current (the caller has made
// it current: sal_context_create and the entry point both set it first).
void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_looked_up[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_looked_up[device] = true;
        g_ptr[device] = e == hipSuccess ? p : nullptr;
    }
    return g_ptr[device];
}

}  // namespace sal

using namespace sal;

extern "C" sal_status sal_label_points_noalloc(sal_context *ctx, const sal_surface_set *set,
                                               int64_t n, const float *x, const float *y,
                                               const float *z, const sal_label_options *opt_in,
                                               int32_t *labels, void *winding,
                                               sal_label_stats *stats) {
    try {
        if (!ctx || !set) return set_error(SAL_ERR_INVALID_ARG, "ctx or set is NULL");
        if (n < 0) return set_error(SAL_ERR_INVALID_ARG, "n_points < 0");
        if (n > kNoAllocMaxPoints)
            return set_error(SAL_ERR_CAPACITY,
                             "sal_label_points_noalloc takes at most 1048576 points per call");
        if (set->device != ctx->device)
            return set_error(SAL_ERR_INVALID_ARG, "surface set lives on another device");
        sal_label_options opt;
        sal_status st = resolve_options(opt_in, &opt);
        if (st != SAL_OK) return st;
        if (opt.cull_bounds)
            return set_error(SAL_ERR_INVALID_ARG,
                             "cull_bounds is not available without allocation");
        if (winding && opt.winding_type == SAL_WINDING_NONE)
            return set_error(SAL_ERR_INVALID_ARG, "winding buffer given with SAL_WINDING_NONE");
        if (n > 0 && (!x || !y || !z || !labels))
            return set_error(SAL_ERR_INVALID_ARG, "NULL point or label buffer");
        if (stats) std::memset(stats, 0, sizeof(*stats));
        if (n == 0) return SAL_OK;
        SAL_HIP(hipSetDevice(ctx->device));
        unsigned char *base = (unsigned char *)noalloc_scratch(ctx->device);
        if (!base) return set_error(SAL_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed");
        // no tuning (it times trial launches and synchronises): an unset
        // launch shape takes the tuner's usual choice, 1 point per lane and
        // 4 wavefronts per workgroup
        if (opt.points_per_lane == 0 || opt.precision == SAL_PREC_FP64) opt.points_per_lane = 1;
        if (opt.block_waves == 0) opt.block_waves = 4;
        LabelScratch sc;
        sc.counters = (unsigned long long *)(base + kOffCounters);
        sc.flag_list = (FlagEntry *)(base + kOffFlags);
        sc.rc_res = (unsigned long long *)(base + kOffRes);
        sc.rc_pairs = (RecheckPair *)(base + kOffPairs);
        sc.rc_out = (RecheckOut *)(base + kOffOut);
        sc.rc_seg = (RecheckSeg *)(base + kOffSeg);
        sc.rc_pair_cap = kNoAllocPairCap;
        hipStream_t s = ctx->stream;
        // counters start at zero on every call (a fill kernel, not a memset
        // node, so the call can be captured)
        SAL_HIP(launch_fill_u64(sc.counters, 0ull, kNumCounters, s));
        if (stats) SAL_HIP(hipEventRecord(ctx->ev[0], s));
        st = enqueue_label_with(ctx, set, n, nullptr, x, y, z, opt, labels, winding,
                                stats ? ctx->ev[1] : nullptr, s, nullptr, sc);
        if (st != SAL_OK) return st;
        if (stats) {
            SAL_HIP(hipEventRecord(ctx->ev[2], s));
            SAL_HIP(hipEventSynchronize(ctx->ev[2]));
            unsigned long long c[kNumCounters];
            SAL_HIP(hipMemcpy(c, sc.counters, sizeof(c), hipMemcpyDeviceToHost));
            stats->n_points = n;
            stats->n_pairs = n * set->n_tri;
            stats->n_recheck_points = (int64_t)c[kCntFlagged];
            stats->n_recheck_pairs = (int64_t)c[kCntRecheck];
            stats->n_band_flags = (int64_t)c[kCntBand];
            stats->n_cond_flags = (int64_t)c[kCntCond];
            stats->n_exact_fallbacks = (int64_t)c[kCntExact];
            stats->n_recheck_f64_terms = (int64_t)c[kCntRecheckF64];
            SAL_HIP(hipEventElapsedTime(&stats->ms_pairloop, ctx->ev[0], ctx->ev[1]));
            SAL_HIP(hipEventElapsedTime(&stats->ms_total, ctx->ev[0], ctx->ev[2]));
            stats->ms_recheck = stats->ms_total - stats->ms_pairloop;
            stats->points_per_lane = opt.points_per_lane;
            stats->block_waves = opt.block_waves;
        }
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_label_points_noalloc");
    }
}
