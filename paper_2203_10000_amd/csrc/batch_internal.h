// Batched labeling data shared by batch.hip and batch.cpp.
#pragma once

#include "sal_internal.h"

namespace sal {

// One instance as the kernels see it.
struct BatchInst {
    const Rec32 *rec32;
    const Rec64 *rec64;
    const SurfaceDev *surf;
    const int64_t *strip_off;
    const float *x, *y, *z;
    int32_t *labels;
    int64_t n;             // points
    int64_t point_base;    // first global point id
    int64_t slot_base;     // first partial slot
    int32_t n_surf;
    int32_t splits_total;  // sum over surfaces of the strip-range splits
    int32_t split_off[kMaxSurfaces + 1];
    int32_t surf_label[kMaxSurfaces];
};

// (instance, 64-point block, surface, strip range) -> partial slot.
struct BatchItem {
    int32_t inst;
    int32_t surf;
    int64_t block;
    int64_t rec_begin, rec_end;
    int64_t slot;
};

struct BatchArgs {
    const BatchItem *items;
    int64_t n_items;
    const BatchInst *insts;
    int n_inst;
    int64_t total_points;
    unsigned int *next_item;
    double *partial;        // [slots][64]
    uint64_t *slot_mask;    // [slots]: conditioning flags (float32 form) or
                            // points on the surface (plain FP64 form)
    float kappa;
    double threshold, band;
    FlagEntry *flag_list;   // capacity total_points
    unsigned long long *counters;       // kCntFlagged = list length
    unsigned long long *inst_counters;  // [n_inst][kNumCounters]
    int fp64;               // plain FP64 form: FP64 walk, no float32 pass, no recheck
};

hipError_t launch_batch(const BatchArgs &a, int persistent_blocks, int recheck_blocks,
                        hipStream_t s);

}  // namespace sal
