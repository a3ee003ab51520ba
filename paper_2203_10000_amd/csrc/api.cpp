// C-ABI entry points: contexts, surface sets, point labeling.
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "runtime.h"

namespace sal {

static thread_local std::string g_last_error;

sal_status set_error(sal_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

// Allocation fault injection (sal_debug_fail_allocation): the countdown is
// the number of allocations left before the one that fails; 0 = off.
static std::atomic<int64_t> g_fail_countdown{0};

hipError_t dev_malloc(void **ptr, size_t bytes) {
    int64_t c = g_fail_countdown.load();
    while (c > 0 && !g_fail_countdown.compare_exchange_weak(c, c - 1)) {
    }
    if (c == 1) {
        if (ptr) *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(ptr, bytes);
}

sal_status hip_error(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SAL_ERR_OUT_OF_MEMORY : SAL_ERR_DEVICE;
}

// The flag list and the pair-major recheck scratch: a quarter of the flag
// capacity in pairs (a point more often has one flagged surface than two; a
// recheck with more pairs than that takes the per-point form).
sal_status ensure_flag_capacity(sal_context *ctx, int64_t n) {
    if (n <= ctx->flag_cap && ctx->rc_seg) return SAL_OK;
    SAL_HIP(hipStreamSynchronize(ctx->stream));
    auto release = [](void *&p) {
        if (p) (void)hipFree(p);
        p = nullptr;
    };
    release((void *&)ctx->flag_list);
    release((void *&)ctx->rc_pairs);
    release((void *&)ctx->rc_out);
    release((void *&)ctx->rc_res);
    ctx->batch_graph_key = 0;   // a captured batch graph points at the old list
    ctx->flag_cap = 0;
    ctx->rc_pair_cap = 0;
    const int64_t cap = n < 4096 ? 4096 : n;
    const int64_t pcap = cap / 4 + 64 * kMaxSurfaces;
    SAL_HIP(dev_malloc((void **)&ctx->flag_list, (size_t)cap * sizeof(FlagEntry)));
    SAL_HIP(dev_malloc((void **)&ctx->rc_res, (size_t)cap * sizeof(unsigned long long)));
    SAL_HIP(dev_malloc((void **)&ctx->rc_pairs, (size_t)pcap * sizeof(RecheckPair)));
    SAL_HIP(dev_malloc((void **)&ctx->rc_out, (size_t)pcap * sizeof(RecheckOut)));
    if (!ctx->rc_seg) SAL_HIP(dev_malloc((void **)&ctx->rc_seg, sizeof(RecheckSeg)));
    ctx->flag_cap = cap;
    ctx->rc_pair_cap = pcap;
    return SAL_OK;
}

sal_status resolve_options(const sal_label_options *in, sal_label_options *out) {
    sal_label_options_default(out);
    if (in) *out = *in;
    if (out->precision != SAL_PREC_FP64 && out->precision != SAL_PREC_FP32_RECHECK)
        return set_error(SAL_ERR_INVALID_ARG, "precision must be SAL_PREC_FP64 or SAL_PREC_FP32_RECHECK");
    if (out->winding_type < SAL_WINDING_NONE || out->winding_type > SAL_WINDING_F64)
        return set_error(SAL_ERR_INVALID_ARG, "bad winding_type");
    if (!(out->threshold > 0.0 && out->threshold < 1.0))
        return set_error(SAL_ERR_INVALID_ARG, "threshold must be in (0, 1)");
    if (!(out->recheck_band >= 0.0 && out->recheck_band < 1.0))
        return set_error(SAL_ERR_INVALID_ARG, "recheck_band must be in [0, 1)");
    if (out->kappa == 0.0) out->kappa = 0.03125;
    if (!(out->kappa > 0.0 && out->kappa < 1.0))
        return set_error(SAL_ERR_INVALID_ARG, "kappa must be in (0, 1)");
    if (out->points_per_lane != 0 && out->points_per_lane != 1 && out->points_per_lane != 2 &&
        out->points_per_lane != 4)
        return set_error(SAL_ERR_INVALID_ARG, "points_per_lane must be 0, 1, 2 or 4");
    if (out->block_waves != 0 && out->block_waves != 1 && out->block_waves != 2 && out->block_waves != 4 &&
        out->block_waves != 8)
        return set_error(SAL_ERR_INVALID_ARG, "block_waves must be 0, 1, 2, 4 or 8");
    if (out->element_rule != SAL_RULE_CENTROID && out->element_rule != SAL_RULE_FOUR_NODES)
        return set_error(SAL_ERR_INVALID_ARG, "element_rule must be SAL_RULE_CENTROID or SAL_RULE_FOUR_NODES");
    return SAL_OK;
}

LabelScratch context_scratch(const sal_context *ctx) {
    return LabelScratch{ctx->counters, ctx->flag_list, ctx->rc_pairs, ctx->rc_out,
                        ctx->rc_res,   ctx->rc_seg,    ctx->rc_pair_cap};
}

sal_status enqueue_label_on(sal_context *ctx, const sal_surface_set *set, int64_t n,
                            const int64_t *n_dev, const float *x, const float *y, const float *z,
                            const sal_label_options &opt, int32_t *labels, void *winding,
                            hipEvent_t ev_mid, hipStream_t stream, unsigned long long *masks) {
    return enqueue_label_with(ctx, set, n, n_dev, x, y, z, opt, labels, winding, ev_mid, stream,
                              masks, context_scratch(ctx));
}

sal_status enqueue_label_with(sal_context *ctx, const sal_surface_set *set, int64_t n,
                              const int64_t *n_dev, const float *x, const float *y,
                              const float *z, const sal_label_options &opt, int32_t *labels,
                              void *winding, hipEvent_t ev_mid, hipStream_t stream,
                              unsigned long long *masks, const LabelScratch &sc) {
    PairloopArgs a{};
    a.rec32 = set->rec32;
    a.rec64 = set->rec64;
    a.surf = set->surf;
    a.n_surf = set->n_surf;
    a.x = x;
    a.y = y;
    a.z = z;
    a.n = n;
    a.n_dev = n_dev;
    a.kappa = (float)opt.kappa;
    a.threshold = opt.threshold;
    a.band = opt.recheck_band;
    a.labels = labels;
    a.winding = winding;
    a.winding_type = winding ? opt.winding_type : SAL_WINDING_NONE;
    if (!winding) a.winding = nullptr;
    a.masks = masks;
    a.cull = opt.cull_bounds ? 1 : 0;
    a.flag_list = sc.flag_list;
    a.counters = sc.counters;
    if (opt.precision == SAL_PREC_FP64) {
        SAL_HIP(launch_pairloop_f64(a, opt.block_waves, stream));
        if (ev_mid) SAL_HIP(hipEventRecord(ev_mid, stream));
        return SAL_OK;
    }
    SAL_HIP(launch_pairloop_f32(a, opt.points_per_lane, opt.block_waves, stream));
    if (ev_mid) SAL_HIP(hipEventRecord(ev_mid, stream));
    RecheckArgs r{};
    r.rec32 = set->rec32;
    r.rec64 = set->rec64;
    r.surf = set->surf;
    r.strip_off = set->strip_off;
    r.x = x;
    r.y = y;
    r.z = z;
    r.n = n;
    r.threshold = opt.threshold;
    r.kappa = (float)opt.kappa;
    r.labels = labels;
    r.winding = a.winding;
    r.winding_type = a.winding_type;
    r.masks = masks;
    r.flag_list = sc.flag_list;
    r.counters = sc.counters;
    r.n_surf = set->n_surf;
    r.pairs = sc.rc_pairs;
    r.pair_out = sc.rc_out;
    r.res = sc.rc_res;
    r.seg = sc.rc_seg;
    r.pair_cap = sc.rc_pair_cap;
    r.target_waves = (int64_t)ctx->n_cu * 32;
    const int64_t grid = n < (int64_t)ctx->n_cu * 8 ? n : (int64_t)ctx->n_cu * 8;
    SAL_HIP(launch_recheck_f64(r, (int)grid, stream));
    return SAL_OK;
}

sal_status enqueue_label(sal_context *ctx, const sal_surface_set *set, int64_t n, const float *x,
                         const float *y, const float *z, const sal_label_options &opt_in,
                         int32_t *labels, void *winding, hipEvent_t ev_start, hipEvent_t ev_mid,
                         int *shape, unsigned long long *masks) {
    sal_label_options opt = opt_in;
    sal_status ts = tune_launch(ctx, set, n, x, y, z, labels, &opt);
    if (ts != SAL_OK) return ts;
    if (ev_start) SAL_HIP(hipEventRecord(ev_start, ctx->stream));
    if (shape) {
        shape[0] = opt.points_per_lane;
        shape[1] = opt.block_waves;
    }
    return enqueue_label_on(ctx, set, n, nullptr, x, y, z, opt, labels, winding, ev_mid,
                            ctx->stream, masks);
}

}  // namespace sal

using namespace sal;

#define SAL_GUARD_BEGIN try {
#define SAL_GUARD_END                                                          \
    }                                                                          \
    catch (const std::bad_alloc &) {                                           \
        return set_error(SAL_ERR_OUT_OF_MEMORY, "host allocation failed");     \
    }                                                                          \
    catch (const std::exception &ex) {                                         \
        return set_error(SAL_ERR_INTERNAL, ex.what());                         \
    }                                                                          \
    catch (...) {                                                              \
        return set_error(SAL_ERR_INTERNAL, "unknown exception");               \
    }

extern "C" {

const char *sal_status_string(sal_status s) {
    switch (s) {
        case SAL_OK: return "ok";
        case SAL_ERR_INVALID_ARG: return "invalid argument";
        case SAL_ERR_NOT_CLOSED: return "surface not closed";
        case SAL_ERR_ORIENTATION: return "surface orientation";
        case SAL_ERR_OUT_OF_MEMORY: return "out of memory";
        case SAL_ERR_DEVICE: return "device error";
        case SAL_ERR_CAPACITY: return "capacity exceeded";
        case SAL_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *sal_last_error_message(void) { return g_last_error.c_str(); }

int sal_abi_version(void) { return SAL_ABI_VERSION; }

void sal_debug_fail_allocation(int64_t n) { g_fail_countdown.store(n > 0 ? n : 0); }

void sal_label_options_default(sal_label_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = SAL_PREC_FP32_RECHECK;
    o->winding_type = SAL_WINDING_NONE;
    o->threshold = 0.5;
    o->recheck_band = 1e-3;
    o->kappa = 0.0;
    o->points_per_lane = 0;
    o->block_waves = 0;
    o->use_graph = 0;
    o->element_rule = SAL_RULE_CENTROID;
}

sal_status sal_context_create(int device, void *stream, sal_context **out) {
    SAL_GUARD_BEGIN
    g_last_error.clear();
    if (!out) return set_error(SAL_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return set_error(SAL_ERR_DEVICE, "no HIP device available");
    if (device < 0 || device >= count) return set_error(SAL_ERR_INVALID_ARG, "device out of range");
    SAL_HIP(hipSetDevice(device));
    auto *ctx = new sal_context();
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->n_cu = prop.multiProcessorCount;
    if (ctx->n_cu <= 0) ctx->n_cu = 256;
    // set-up of sal_label_points_noalloc: its scratch array's address on
    // this device (looked up once per device; a failure shows there)
    (void)noalloc_scratch(device);
    for (auto &ev : ctx->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) { sal_context_destroy(ctx); return hip_error(e, "hipEventCreate"); }
    }
    e = dev_malloc((void **)&ctx->counters, kNumCounters * sizeof(unsigned long long));
    if (e != hipSuccess) { sal_context_destroy(ctx); return hip_error(e, "hipMalloc(counters)"); }
    e = dev_malloc((void **)&ctx->tune_counters, kNumCounters * sizeof(unsigned long long));
    if (e != hipSuccess) { sal_context_destroy(ctx); return hip_error(e, "hipMalloc(counters)"); }
    e = dev_malloc((void **)&ctx->batch_next, sizeof(unsigned int) * 4);
    if (e != hipSuccess) { sal_context_destroy(ctx); return hip_error(e, "hipMalloc(batch counter)"); }
    e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { sal_context_destroy(ctx); return hip_error(e, "hipStreamCreate"); }
    *out = ctx;
    return SAL_OK;
    SAL_GUARD_END
}

sal_status sal_context_set_stream(sal_context *ctx, void *stream) {
    if (!ctx) return set_error(SAL_ERR_INVALID_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)stream;
    return SAL_OK;
}

void sal_context_destroy(sal_context *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &ev : ctx->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->flag_list) (void)hipFree(ctx->flag_list);
    if (ctx->rc_pairs) (void)hipFree(ctx->rc_pairs);
    if (ctx->rc_out) (void)hipFree(ctx->rc_out);
    if (ctx->rc_res) (void)hipFree(ctx->rc_res);
    if (ctx->rc_seg) (void)hipFree(ctx->rc_seg);
    if (ctx->counters) (void)hipFree(ctx->counters);
    if (ctx->tune_counters) (void)hipFree(ctx->tune_counters);
    if (ctx->batch_graph) (void)hipGraphExecDestroy(ctx->batch_graph);
    if (ctx->batch_items) (void)hipFree(ctx->batch_items);
    if (ctx->batch_insts) (void)hipFree(ctx->batch_insts);
    if (ctx->batch_partial) (void)hipFree(ctx->batch_partial);
    if (ctx->batch_mask) (void)hipFree(ctx->batch_mask);
    if (ctx->batch_next) (void)hipFree(ctx->batch_next);
    if (ctx->batch_counters) (void)hipFree(ctx->batch_counters);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
}

sal_status sal_surface_set_create(sal_context *ctx, const sal_surface_desc *s, int32_t n,
                                  uint32_t flags, sal_surface_set **out) {
    SAL_GUARD_BEGIN
    g_last_error.clear();
    if (out) *out = nullptr;
    if (flags & ~SAL_SURF_AUTO_ORIENT) return set_error(SAL_ERR_INVALID_ARG, "unknown flag bits");
    return build_surface_set(ctx, s, n, flags, out);
    SAL_GUARD_END
}

void sal_surface_set_destroy(sal_surface_set *set) { destroy_surface_set(set); }

sal_status sal_surface_set_get_info(const sal_surface_set *set, sal_surface_set_info *info) {
    if (!set || !info) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
    info->n_surfaces = set->n_surf;
    info->n_triangles = set->n_tri;
    info->n_strips = set->n_strips;
    info->device_bytes = set->bytes;
    return SAL_OK;
}

sal_status sal_label_points(sal_context *ctx, const sal_surface_set *set, int64_t n,
                            const float *x, const float *y, const float *z,
                            const sal_label_options *opt_in, int32_t *labels, void *winding,
                            sal_label_stats *stats) {
    SAL_GUARD_BEGIN
    g_last_error.clear();
    if (!ctx || !set) return set_error(SAL_ERR_INVALID_ARG, "ctx or set is NULL");
    if (n < 0) return set_error(SAL_ERR_INVALID_ARG, "n_points < 0");
    if (set->device != ctx->device)
        return set_error(SAL_ERR_INVALID_ARG, "surface set lives on another device");
    sal_label_options opt;
    sal_status st = resolve_options(opt_in, &opt);
    if (st != SAL_OK) return st;
    if (winding && opt.winding_type == SAL_WINDING_NONE)
        return set_error(SAL_ERR_INVALID_ARG, "winding buffer given with SAL_WINDING_NONE");
    if (n > 0 && (!x || !y || !z || !labels))
        return set_error(SAL_ERR_INVALID_ARG, "NULL point or label buffer");
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n == 0) return SAL_OK;
    SAL_HIP(hipSetDevice(ctx->device));
    // every argument is checked before anything is enqueued
    if (opt.cull_bounds && (st = ensure_surface_balls(ctx, set)) != SAL_OK) return st;
    if (opt.precision == SAL_PREC_FP32_RECHECK) {
        st = ensure_flag_capacity(ctx, n);
        if (st != SAL_OK) return st;
    }
    SAL_HIP(launch_fill_u64(ctx->counters, 0ull, kNumCounters, ctx->stream));
    int shape[2] = {0, 0};
    st = enqueue_label(ctx, set, n, x, y, z, opt, labels, winding, stats ? ctx->ev[0] : nullptr,
                       stats ? ctx->ev[1] : nullptr, shape);
    if (st != SAL_OK) return st;
    if (stats) {
        SAL_HIP(hipEventRecord(ctx->ev[2], ctx->stream));
        SAL_HIP(hipEventSynchronize(ctx->ev[2]));
        unsigned long long c[kNumCounters];
        SAL_HIP(hipMemcpy(c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost));
        stats->n_points = n;
        stats->n_pairs = n * set->n_tri;
        stats->n_recheck_points = (int64_t)c[kCntFlagged];
        stats->n_recheck_pairs = (int64_t)c[kCntRecheck];
        stats->n_band_flags = (int64_t)c[kCntBand];
        stats->n_cond_flags = (int64_t)c[kCntCond];
        stats->n_exact_fallbacks = (int64_t)c[kCntExact];
        stats->n_recheck_f64_terms = (int64_t)c[kCntRecheckF64];
        stats->n_pairs_culled = (int64_t)c[kCntCulled];
        SAL_HIP(hipEventElapsedTime(&stats->ms_pairloop, ctx->ev[0], ctx->ev[1]));
        SAL_HIP(hipEventElapsedTime(&stats->ms_total, ctx->ev[0], ctx->ev[2]));
        stats->ms_recheck = stats->ms_total - stats->ms_pairloop;
        stats->points_per_lane = shape[0];
        stats->block_waves = shape[1];
    }
    return SAL_OK;
    SAL_GUARD_END
}

}  // extern "C"
