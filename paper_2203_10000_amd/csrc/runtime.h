// Host-side objects behind the opaque handles of sal.h.
#pragma once

#include <vector>

#include "sal_internal.h"

// Device scratch owned by a context; grows, never shrinks.
struct sal_context {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev[8] = {};
    sal::FlagEntry *flag_list = nullptr;
    int64_t flag_cap = 0;
    // pair-major recheck scratch (grows with the flag list)
    sal::RecheckPair *rc_pairs = nullptr;
    sal::RecheckOut *rc_out = nullptr;
    unsigned long long *rc_res = nullptr;
    sal::RecheckSeg *rc_seg = nullptr;
    int64_t rc_pair_cap = 0;
    unsigned long long *counters = nullptr;  // sal::kNumCounters
    unsigned long long *tune_counters = nullptr;
    int n_cu = 0;
    // batched form
    void *batch_items = nullptr;
    int64_t batch_items_bytes = 0;
    void *batch_insts = nullptr;
    int64_t batch_insts_bytes = 0;
    double *batch_partial = nullptr;
    uint64_t *batch_mask = nullptr;
    int64_t batch_slots = 0;
    unsigned int *batch_next = nullptr;
    unsigned long long *batch_counters = nullptr;
    int64_t batch_counters_n = 0;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t batch_graph = nullptr;
    uint64_t batch_graph_key = 0;
    std::vector<uint64_t> batch_graph_fields;   // the fields hashed into batch_graph_key
    int64_t batch_graph_points = 0;
    uint64_t batch_items_key = 0;   // batch whose work list the item buffers hold (0: none)
    std::vector<uint64_t> batch_items_fields;   // the fields hashed into batch_items_key
    int64_t batch_n_items = 0;
};

struct sal_surface_set {
    uint64_t uid = 0;      // unique per creation (graph cache keys)
    int device = 0;
    int n_surf = 0;
    int64_t n_tri = 0, n_strips = 0, n_rec = 0, bytes = 0;
    sal::Rec32 *rec32 = nullptr;
    sal::Rec64 *rec64 = nullptr;
    sal::SurfaceDev *surf = nullptr;        // n_surf entries, then the two tuner entries
    sal::SurfaceDev *tune_surf = nullptr;   // surf + n_surf: [0] float32 trials, [1] FP64 trials,
                                            // [2] float32 screening trials
    int64_t *strip_off = nullptr;
    std::vector<sal::SurfaceDev> host_table;
    std::vector<int64_t> host_strip_off;   // record index of every strip head
    std::vector<int32_t> host_strip_tris;  // triangles of every strip
    bool balls_ready = false;              // ball_w of every surface known
};

namespace sal {

sal_status build_surface_set(sal_context *ctx, const sal_surface_desc *desc, int32_t n,
                             uint32_t flags, sal_surface_set **out);
void destroy_surface_set(sal_surface_set *set);

// Finds the winding number of each surface's ball centre (plain FP64 form,
// one launch per surface, synchronising the stream) the first time culling
// is asked for; until then no ball is used.
sal_status ensure_surface_balls(sal_context *ctx, const sal_surface_set *set);

// Grows the context scratch to hold a flag list of n entries.
sal_status ensure_flag_capacity(sal_context *ctx, int64_t n);

// Validated options with defaults applied.
sal_status resolve_options(const sal_label_options *in, sal_label_options *out);

// Enqueues one labeling pass (pair loop, and recheck in the float32 form) of
// n points; counters must be cleared by the caller.  The launch shape is
// resolved first (tune_launch); then ev_start (before the pair loop) and
// ev_after_pairloop are recorded when non-null, so that timings bracketed by
// them leave out any tuning.
sal_status enqueue_label(sal_context *ctx, const sal_surface_set *set, int64_t n, const float *x,
                         const float *y, const float *z, const sal_label_options &opt,
                         int32_t *labels, void *winding, hipEvent_t ev_start,
                         hipEvent_t ev_after_pairloop, int *shape = nullptr,
                         unsigned long long *masks = nullptr);

// The device scratch one labeling pass works in: the counters, the flag list
// (one entry per point at most) and the pair-major recheck buffers.
struct LabelScratch {
    unsigned long long *counters;
    FlagEntry *flag_list;
    RecheckPair *rc_pairs;
    RecheckOut *rc_out;
    unsigned long long *rc_res;
    RecheckSeg *rc_seg;
    int64_t rc_pair_cap;
};

// The context's own scratch (sized by ensure_flag_capacity).
LabelScratch context_scratch(const sal_context *ctx);

// The launches of one labeling pass with a resolved launch shape and the
// given scratch, on `stream`; the counters must be cleared by the caller.
sal_status enqueue_label_with(sal_context *ctx, const sal_surface_set *set, int64_t n,
                              const int64_t *n_dev, const float *x, const float *y,
                              const float *z, const sal_label_options &opt, int32_t *labels,
                              void *winding, hipEvent_t ev_mid, hipStream_t stream,
                              unsigned long long *masks, const LabelScratch &sc);

// Address of the allocation-free entry point's scratch array on `device`
// (looked up once per device, with the device current); nullptr on error.
void *noalloc_scratch(int device);

// The launches of one labeling pass with a resolved launch shape, on
// `stream`.  With n_dev set the point count is read on the device and n is the
// capacity the grids are sized for (the form a captured graph uses).
sal_status enqueue_label_on(sal_context *ctx, const sal_surface_set *set, int64_t n,
                            const int64_t *n_dev, const float *x, const float *y, const float *z,
                            const sal_label_options &opt, int32_t *labels, void *winding,
                            hipEvent_t ev_mid, hipStream_t stream,
                            unsigned long long *masks = nullptr);

// Resolves points_per_lane / block_waves left at 0 by timing the candidates
// on a prefix of the points against a prefix of the strips (the tuner table
// entries), so a trial costs a bounded number of pairs; the first use of a
// size bucket synchronises the stream.  Cached per process.
sal_status tune_launch(sal_context *ctx, const sal_surface_set *set, int64_t n, const float *x,
                       const float *y, const float *z, int32_t *labels, sal_label_options *opt);

}  // namespace sal
