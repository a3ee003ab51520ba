// Device helpers for the Kuhn lattice shared by the mesh passes: tetrahedron
// keys, permutations and vertices (paper section 2.1.1).
//
// A level-l tetrahedron is (cell c, permutation q of the axes); q indexes the
// six permutations (p0, p1, p2) in lexicographic order.  Its vertices, in that
// level's integer units, are x0 = c, x1 = x0 + e_p0, x2 = x1 + e_p1,
// x3 = c + (1, 1, 1).  Key: level in bits 60-63, q in 57-59, and 19 bits per
// cell coordinate.  Level-0 entries carry no key array: entry i is cell i / 6
// (x fastest), permutation i % 6.
#pragma once
#include <hip/hip_runtime.h>

#include "mesh_internal.h"

namespace sal {

__device__ __forceinline__ void perm_of(int q, int &p0, int &p1, int &p2) {
    // lexicographic permutations of (x, y, z)
    p0 = q >> 1;
    const int a = p0 == 0 ? 1 : 0;
    const int b = p0 == 2 ? 1 : 2;
    if (q & 1) { p1 = b; p2 = a; } else { p1 = a; p2 = b; }
}

__device__ __forceinline__ int q_of(int p0, int p1, int p2) { return 2 * p0 + (p1 > p2 ? 1 : 0); }

__device__ __forceinline__ uint64_t make_key(int l, int q, int64_t i, int64_t j, int64_t k) {
    return ((uint64_t)l << 60) | ((uint64_t)q << 57) | ((uint64_t)i << 38) | ((uint64_t)j << 19) |
           (uint64_t)k;
}

__device__ __forceinline__ void split_key(uint64_t key, int &l, int &q, int64_t c[3]) {
    l = (int)(key >> 60);
    q = (int)((key >> 57) & 7u);
    c[0] = (int64_t)((key >> 38) & 0x7ffffu);
    c[1] = (int64_t)((key >> 19) & 0x7ffffu);
    c[2] = (int64_t)(key & 0x7ffffu);
}

__device__ __forceinline__ uint64_t entry_key(const LevelPtrs &L, const LatticeGeom &g, int l,
                                              int64_t i) {
    if (l > 0) return L.key[l][i];
    const int q = (int)(i % 6);
    int64_t cell = i / 6;
    const int64_t cx = cell % g.cells[0];
    cell /= g.cells[0];
    const int64_t cy = cell % g.cells[1];
    const int64_t cz = cell / g.cells[1];
    return make_key(0, q, cx, cy, cz);
}

// origin + scale * t in double with the product and the sum rounded
// separately (never fused into one FMA), then rounded once more to float: the
// coordinates a host computes with plain double arithmetic.
__device__ __forceinline__ float lattice_coord(double origin, double scale, double t) {
#pragma clang fp contract(off)
    const double p = scale * t;
    return (float)(origin + p);
}

// Vertices x0..x3 of (cell c, permutation q) in that level's integer units.
__device__ __forceinline__ void kuhn_vertices(int q, const int64_t c[3], int64_t X[4][3]) {
    int p0, p1, p2;
    perm_of(q, p0, p1, p2);
    for (int a = 0; a < 3; ++a) {
        X[0][a] = c[a];
        X[3][a] = c[a] + 1;
    }
    for (int a = 0; a < 3; ++a) X[1][a] = X[0][a];
    X[1][p0] += 1;
    for (int a = 0; a < 3; ++a) X[2][a] = X[1][a];
    X[2][p1] += 1;
}

}  // namespace sal
