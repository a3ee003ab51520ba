// Tetrahedral-mesh data shared by the mesh kernels (mesh.hip) and the host
// orchestration (mesh.cpp).
#pragma once

#include "sal_internal.h"

namespace sal {

constexpr int kMaxLevels = 3;   // refinement levels 1..3 above the lattice

// Per-level arrays.  Level 0 is the lattice (keys implicit from the index);
// level l >= 1 holds blocks of 8 children appended in split order.
//   child[l][i] = -1 for a leaf, else b: its children are level l+1 entries
//   8b .. 8b+7 (in the order of ChildTables::list).
struct LevelPtrs {
    uint64_t *key[kMaxLevels + 1];
    int32_t *label[kMaxLevels + 1];
    int32_t *child[kMaxLevels + 1];
    uint8_t *flag[kMaxLevels + 1];
    int64_t n[kMaxLevels + 1];
    const int64_t *n_dev;   // device copy of the level sizes; when set it replaces n
    int inherit;            // splits give the children their parent's label
};

// Per-round figures kept on the device by the captured refine round.
struct RoundStat {
    int64_t n_leaves, n_boundary, n_labeled, n_recheck_pairs;
};

// Device-resident state of the captured refine round: every size the round
// needs lives here, so one captured graph serves every round.  The plan step
// turns `status` nonzero (sticky) instead of writing past a capacity; the
// steps that change the mesh then do nothing.
struct RoundState {
    int64_t n[kMaxLevels + 1];           // entries per level
    int64_t cap[kMaxLevels + 1];         // capacity per level
    int64_t base_block[kMaxLevels + 1];  // first child block of each level's splits
    int64_t kid_off[kMaxLevels + 1];     // each level's children in the labeling scratch
    int64_t n_kids;                      // children made this round
    int64_t kid_cap;                     // labeling scratch capacity
    int64_t n_leaves;
    int32_t status;                      // 0 ok, 1 out of capacity, 2 beyond the deepest level
    int32_t round;                       // rounds completed
    RoundStat stat[kMaxLevels + 1];
};

struct LatticeGeom {
    double origin[3];
    double h;
    int32_t cells[3];
};

// Children of a tetrahedron with permutation index q: list[q][r] = (sub-cell
// code dx + 2 dy + 4 dz, child q') for r = 0..7; rank[q][code][q'] = r or -1.
struct ChildTables {
    int8_t list[6][8][2];
    int8_t rank[6][8][6];
};

// Source of a compaction: nonzero flags, or leaves (child < 0).
struct CompactSrc {
    const uint8_t *flag;    // entries with flag & mask != 0 (mask 0: any bit) ...
    const int32_t *child;   // ... or, without flag, the leaves (child < 0)
    uint8_t mask;
};

hipError_t launch_lattice_centroids(const LatticeGeom &g, int64_t n0, float *cx, float *cy,
                                    float *cz, hipStream_t s);
hipError_t launch_mark(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                       hipStream_t s);
int64_t compact_blocks(int64_t n);
hipError_t launch_compact(const CompactSrc &src, int64_t n, int64_t *block_scratch,
                          int64_t *total, int32_t *out, hipStream_t s);
hipError_t launch_split(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                        const int32_t *list, int64_t count, int64_t base_block, float *cx,
                        float *cy, float *cz, hipStream_t s);
hipError_t launch_export(const LevelPtrs &L, const LatticeGeom &g, int l, const int32_t *list,
                         int64_t count, int64_t out_base, uint64_t *keys, int32_t *labels,
                         float *cx, float *cy, float *cz, hipStream_t s);
// Device-sized forms for the captured refine round (sizes read from
// RoundState / compaction totals; fixed grids stride over them).
hipError_t launch_round_begin(RoundState *rs, unsigned long long *counters, hipStream_t s);
hipError_t launch_clear_flags_dev(uint8_t *flag, const int64_t *n_dev, hipStream_t s);
hipError_t launch_compact_dev(const CompactSrc &src, const int64_t *n_dev, int64_t cap,
                              int64_t *block_scratch, int64_t *total, int32_t *out, hipStream_t s);
hipError_t launch_plan(RoundState *rs, const int64_t *totals, hipStream_t s);
hipError_t launch_split_dev(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                            const int32_t *list, const int64_t *totals, const RoundState *rs,
                            float *cx, float *cy, float *cz, hipStream_t s);
hipError_t launch_commit(const RoundState *rs, const int64_t *totals, int l,
                         const int32_t *scratch_labels, int32_t *level_labels, hipStream_t s);
hipError_t launch_round_end(RoundState *rs, const unsigned long long *counters, hipStream_t s);

// Four-node rule (node enclosure masks).
hipError_t launch_lattice_nodes(const LatticeGeom &g, int64_t n_nodes, float *x, float *y, float *z,
                               hipStream_t s);
hipError_t launch_elem_from_nodes0(const LatticeGeom &g, int64_t n0,
                                   const unsigned long long *node0, const SurfaceDev *surf,
                                   int32_t *label0, hipStream_t s);
hipError_t launch_midpoints(const LevelPtrs &L, const LatticeGeom &g, int l, const int32_t *list,
                            int64_t count, float *mx, float *my, float *mz, uint64_t *mkey,
                            hipStream_t s);
// Node table (open addressing; keys ~0 = empty; the host keeps it at most
// half full).
hipError_t launch_node_insert(const uint64_t *mkey, int64_t n, unsigned long long *tkeys,
                              int64_t cap, int64_t *slot, int32_t *new_list,
                              unsigned long long *n_new, hipStream_t s);
hipError_t launch_node_gather(const int32_t *new_list, const unsigned long long *n_new,
                              int64_t n_cap, const float *mx, const float *my, const float *mz,
                              float *x, float *y, float *z, hipStream_t s);
hipError_t launch_node_store(const int32_t *new_list, const unsigned long long *n_new,
                             int64_t n_cap, const int64_t *slot, const unsigned long long *masks,
                             unsigned long long *tmasks, hipStream_t s);
hipError_t launch_node_fetch(const int64_t *slot, int64_t n, const unsigned long long *tmasks,
                             unsigned long long *out, hipStream_t s);
hipError_t launch_node_rehash(const unsigned long long *okeys, const unsigned long long *omasks,
                              int64_t ocap, unsigned long long *tkeys, unsigned long long *tmasks,
                              int64_t cap, hipStream_t s);
hipError_t launch_child_masks(const LevelPtrs &L, const LatticeGeom &g, int l,
                              const int32_t *list, int64_t count, int64_t base_block,
                              const unsigned long long *node0,
                              const unsigned long long *vmask_parent,
                              const unsigned long long *mid_masks,
                              unsigned long long *vmask_child, const SurfaceDev *surf,
                              hipStream_t s);

// Conforming transition refinement (conform.hip).
// Flags of a leaf during the closure (in LevelPtrs::flag): bits 0-5 the
// hanging edges, bit 6 a node at a quarter point, bit 7 split 1 -> 8.
// cells_new: one bit per level-0 cell, set for the cells a vertex added to
// `fresh` touches (unused when fresh is null).
hipError_t launch_insert_range(const LevelPtrs &L, const LatticeGeom &g, int l, int64_t first,
                               int64_t count, unsigned long long *set, int64_t cap,
                               unsigned long long *fresh, int64_t fcap, uint32_t *cells_new,
                               unsigned long long *n_new, unsigned long long *overflow,
                               hipStream_t s);
hipError_t launch_pattern_full(const LevelPtrs &L, const LatticeGeom &g, int l, int64_t first,
                               int64_t count, const unsigned long long *set, int64_t cap,
                               hipStream_t s);
hipError_t launch_pattern_fresh(const LevelPtrs &L, const LatticeGeom &g, int l, int64_t count,
                                const unsigned long long *fresh, int64_t fcap,
                                const uint32_t *cells_new, hipStream_t s);
// hist: 4 counters (leaves cut into 1, 2, 3, 4 tetrahedra), accumulated.
hipError_t launch_tet_counts(const LevelPtrs &L, int l, const int32_t *list, int64_t count,
                             int32_t *counts, unsigned long long *hist, hipStream_t s);
// rocPRIM device-wide primitives: with tmp == nullptr they only set *tmp_bytes.
hipError_t exclusive_sum_i32(const int32_t *in, int64_t *out, int64_t n, void *tmp,
                             size_t *tmp_bytes, hipStream_t s);
hipError_t sort_keys_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, size_t *tmp_bytes,
                         hipStream_t s);
hipError_t launch_emit(const LevelPtrs &L, const LatticeGeom &g, int l, const int32_t *list,
                       int64_t count, const int64_t *offsets, int64_t *tets, int32_t *labels,
                       hipStream_t s);
// Distinct keys of a sorted array, in order; with tmp == nullptr it only sets
// *tmp_bytes.
hipError_t launch_unique(const int64_t *sorted, int64_t n, int32_t *head, int64_t *pos,
                         int64_t *nodes, void *tmp, size_t *tmp_bytes, hipStream_t s);
hipError_t launch_node_ids(const int64_t *tet_keys, int64_t n, const int64_t *nodes, int64_t n_nodes,
                           int32_t *ids, hipStream_t s);
hipError_t launch_node_xyz(const LatticeGeom &g, const int64_t *nodes, int64_t n, float *xyz,
                           hipStream_t s);

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);

}  // namespace sal
