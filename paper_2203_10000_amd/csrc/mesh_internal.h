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
    const uint8_t *flag;
    const int32_t *child;
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
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);

}  // namespace sal
