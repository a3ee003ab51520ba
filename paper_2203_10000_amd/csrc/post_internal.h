// Post-processing of the conforming mesh (paper section 2.2): shared state
// and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mesh_internal.h"
#include "sal.h"

namespace sal {

// The conforming mesh as the post-processing passes see it (device arrays
// owned by the mesh).
struct SmoothCache;
struct ConformView {
    LatticeGeom g;
    int64_t n_tets, n_nodes;
    const int32_t *ids;      // [n_tets][4]
    const int32_t *labels;   // [n_tets]
    const int64_t *keys;     // [n_nodes] finest-grid node keys, ascending
    float *xyz;              // [n_nodes][3]
    SmoothCache **cache;     // edge graph and node classes, built on first use
};

// Edge graph of the conforming mesh over the nodes renumbered in Morton
// order (rank r is node order[r]): rows by rank, neighbours by ascending
// rank; bit 31 of a column marks an interface edge (the tetrahedra around
// it carry two or more labels).  Lists, row segments and working positions
// are in rank space too.
struct SmoothCache {
    int64_t n_nodes = 0, n_edges = 0, n_surface_edges = 0;
    int64_t *rowptr = nullptr;   // [n_nodes + 1]
    uint32_t *cols = nullptr;    // [2 n_edges]
    uint8_t *cls = nullptr;      // [n_nodes] 0 fixed, 1 interface, 2 volume
    int32_t *order = nullptr;    // [n_nodes] node id of each Morton rank
    int32_t *list[2] = {};       // nodes of the surface and of the volume phase
    uint64_t *seg[2] = {};       // their row segments
    uint32_t *head[2] = {};      // the first kTaubinGroup * kTaubinUnroll columns of each
                                 // listed row at a fixed stride (see launch_row_heads)
    int64_t n_list[2] = {};
    int64_t n_entries[2] = {};   // row entries read per half step of each phase
    float4 *pos[2] = {};         // [n_nodes] working positions (w unused)
    double *partials = nullptr;  // per-block sums
    int64_t partials_cap = 0;
    double *sum = nullptr;       // [1]
};
void smooth_cache_free(SmoothCache *c);

// Defined with the mesh: false when the mesh is not conforming yet.
bool conform_view(sal_tet_mesh *m, ConformView *v);
int mesh_device(const sal_tet_mesh *m);

constexpr int kSmoothThreads = 256;
#ifndef SAL_TAUBIN_GROUP
#define SAL_TAUBIN_GROUP 2
#endif
#ifndef SAL_TAUBIN_UNROLL
#define SAL_TAUBIN_UNROLL 8
#endif
constexpr int kTaubinGroup = SAL_TAUBIN_GROUP;     // lanes per node in a half step (power of 2)
constexpr int kTaubinUnroll = SAL_TAUBIN_UNROLL;   // entries per lane loaded together
#ifndef SAL_TAUBIN_WINDOW
#define SAL_TAUBIN_WINDOW 256
#endif
constexpr int kTaubinWindow = SAL_TAUBIN_WINDOW;   // positions a half-step block may stage in LDS

// Edge graph construction.
// *bad_labels counts tetrahedra with a label outside [-1, 254].
hipError_t launch_edge_occurrences(const int32_t *ids, const int32_t *labels, int64_t n_tets,
                                   uint64_t *keys, unsigned long long *bad_labels, hipStream_t s);
hipError_t sort_keys_u64(const uint64_t *in, uint64_t *out, int64_t n, int end_bit, void *tmp,
                         size_t *tmp_bytes, hipStream_t s);
// Per sorted occurrence: 1 where its edge (key >> 8) starts.
hipError_t launch_edge_heads(const uint64_t *keys, int64_t n, int32_t *head, hipStream_t s);
hipError_t exclusive_sum_head(const int32_t *head, int64_t *pos, int64_t n, void *tmp,
                              size_t *tmp_bytes, hipStream_t s);
hipError_t launch_edge_directed(const uint64_t *keys, const int32_t *head, const int64_t *pos,
                                int64_t n, int64_t n_edges, int64_t *start, const int32_t *rank,
                                uint64_t *dkeys, unsigned long long *n_surf, hipStream_t s);
// order[r]: the node of Morton rank r; rank[i]: the rank of node i.  With
// tmp == nullptr it only sets *tmp_bytes.
hipError_t launch_morton_order(const int64_t *keys, int64_t n, uint64_t *code, uint64_t *code_sorted,
                               int32_t *ids, int32_t *order, int32_t *rank, void *tmp,
                               size_t *tmp_bytes, hipStream_t s);
hipError_t launch_csr(const uint64_t *dkeys, int64_t n2, int64_t n_nodes, int64_t *rowptr,
                      uint32_t *cols, hipStream_t s);
hipError_t launch_node_class(const int64_t *rowptr, const uint32_t *cols, const int64_t *keys,
                             const int32_t *order, int64_t n_nodes, const LatticeGeom &g, uint8_t *cls,
                             hipStream_t s);

// Iterations.
hipError_t launch_pack_pos(const float *xyz, const int32_t *order, int64_t n, float4 *a, float4 *b,
                           hipStream_t s);
hipError_t launch_unpack_pos(const float4 *p, const int32_t *order, int64_t n, float *xyz,
                             hipStream_t s);
// sum of |p_i|^2 over the list (block partials, then one fixed-order sum)
hipError_t launch_norm_sq(const float4 *p, const int32_t *list, int64_t n, double *partials,
                          double *sum, hipStream_t s);
// sum of the row lengths of the listed nodes
hipError_t launch_row_entries(const int64_t *rowptr, const int32_t *list, int64_t n, double *partials,
                              double *sum, hipStream_t s);
// out_i = in_i + coef (m_i - in_i) over the listed nodes, m_i the mean of in
// over node i and its neighbours (interface edges only when surface_only);
// *sum = sum of |out_i - in_i|^2.
hipError_t launch_taubin_half(const float4 *in, float4 *out, const uint64_t *seg,
                              const uint32_t *head, const uint32_t *cols, const int32_t *list,
                              int64_t n, double coef, int surface_only, double *partials,
                              double *sum, hipStream_t s);
// seg[t] = (rowptr[list[t]] << 32) | row length (rows below 2^32 entries)
hipError_t launch_row_segments(const int64_t *rowptr, const int32_t *list, int64_t n, uint64_t *seg,
                               hipStream_t s);
// head[(t G + g) U + u] = column q = g + u G of row list[t] (0 past the row's
// end), G = kTaubinGroup, U = kTaubinUnroll: each lane of a node's group
// reads its first U columns as contiguous 16-byte loads, without waiting for
// the row segment.  [n][G U] entries.
hipError_t launch_row_heads(const int64_t *rowptr, const uint32_t *cols, const int32_t *list,
                            int64_t n, uint32_t *head, hipStream_t s);
// Inflation (inflate.hip): triangles of the surface set (9 floats, sorted
// vertices), binned on the level-0 lattice.
hipError_t launch_strip_triangles(const Rec64 *rec, const int64_t *strip_off, const int64_t *tri_base,
                                  int64_t n_strips, float *tri, hipStream_t s);
// pass 0 counts the triangles of each bin into count; pass 1 (count zeroed,
// start its exclusive sum) places them into items.
hipError_t launch_bin_triangles(const float *tri, int64_t n_tri, const LatticeGeom &g, int pass,
                                int32_t *count, const int64_t *start, int32_t *items, hipStream_t s);
hipError_t exclusive_sum_bins(const int32_t *count, int64_t *start, int64_t n, void *tmp, size_t *tmp_bytes,
                              hipStream_t s);
// binned[9 r + c] = tri[9 items[r] + c]: the triangles of every bin, in bin order.
hipError_t launch_gather_binned(const float *tri, const int32_t *items, int64_t n_items, float *binned,
                                hipStream_t s);
// Moves the listed (interface) nodes; out must hold every position on entry.
// sums[0] = nodes moved, sums[1] = triangle tests.  bin_tri: the binned
// triangles (launch_gather_binned), bin k's entries at [bin_start[k], bin_start[k + 1]).
hipError_t launch_inflate(const float4 *in, float4 *out, const uint64_t *seg, const uint32_t *cols,
                          const int32_t *list, int64_t n, const int32_t *order, const int64_t *keys,
                          const float *bin_tri, const int64_t *bin_start, const LatticeGeom &g,
                          double zeta, double *partials, double *sums, hipStream_t s);
int64_t inflate_blocks(int64_t n);

// Builds the edge graph on first use (smooth.cpp).
sal_status ensure_smooth_graph(const ConformView &v, hipStream_t s);

int64_t smooth_blocks(int64_t n);   // blocks of the one-thread-per-item kernels
int64_t taubin_blocks(int64_t n);   // blocks of a half step over n nodes

}  // namespace sal
