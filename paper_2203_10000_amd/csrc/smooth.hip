// Taubin smoothing of the conforming mesh (paper section 2.2.1): the edge
// graph, the node classes and the half steps.
//
// Each half step is a sparse gather: per moved node, its row of neighbour
// ids and their positions (float4, one 16-byte load each), the mean over the
// node and its neighbours in double, and one position written back.  It is
// bound by memory traffic; the arithmetic is a few double operations per
// neighbour.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "post_internal.h"

namespace sal {
namespace {

constexpr int kEdgeA[6] = {0, 0, 0, 1, 1, 2};
constexpr int kEdgeB[6] = {1, 2, 3, 2, 3, 3};
constexpr uint32_t kSurfBit = 1u << 31;

inline unsigned grid_of(int64_t n) { return (unsigned)((n + kSmoothThreads - 1) / kSmoothThreads); }

// Occurrence of edge e of tetrahedron t: (low id << 36) | (high id << 8) |
// (label + 1), ids below 2^28 and labels in [-1, 254] (checked by the host).
__global__ void k_edge_occurrences(const int32_t *__restrict__ ids, const int32_t *__restrict__ labels,
                                   int64_t n_tets, uint64_t *__restrict__ keys,
                                   unsigned long long *__restrict__ bad_labels) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= 6 * n_tets) return;
    const int64_t t = jj / 6;
    const int e = (int)(jj - 6 * t);
    const uint32_t a = (uint32_t)ids[4 * t + kEdgeA[e]], b = (uint32_t)ids[4 * t + kEdgeB[e]];
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    const int32_t lab = labels[t];
    if (e == 0 && (lab < -1 || lab > 254)) atomicAdd(bad_labels, 1ull);
    keys[jj] = (lo << 36) | (hi << 8) | (uint64_t)(uint8_t)(lab + 1);
}

// Morton code of a node (its three 21-bit finest-grid coordinates
// interleaved): numbering the nodes in this order keeps the neighbours of a
// node close in memory in every direction.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

__global__ void k_morton_codes(const int64_t *__restrict__ keys, int64_t n, uint64_t *__restrict__ code,
                               int32_t *__restrict__ ids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = (uint64_t)keys[i];
    code[i] = (spread3(k >> 42) << 2) | (spread3(k >> 21) << 1) | spread3(k);
    ids[i] = (int32_t)i;
}

__global__ void k_rank_of(const int32_t *__restrict__ order, int64_t n, int32_t *__restrict__ rank) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    rank[order[r]] = (int32_t)r;
}

__global__ void k_edge_heads(const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ head) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    head[i] = (i == 0 || (keys[i] >> 8) != (keys[i - 1] >> 8)) ? 1 : 0;
}

__global__ void k_edge_starts(const int32_t *__restrict__ head, const int64_t *__restrict__ pos,
                              int64_t n, int64_t *__restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !head[i]) return;
    start[pos[i]] = i;
}

// Both directions of edge e in Morton ranks: (row << 32) | (col << 1) |
// interface, where the edge is an interface edge when its occurrences carry
// different labels (sorted, so the first and the last differ).
__global__ void k_edge_emit(const uint64_t *__restrict__ keys, const int64_t *__restrict__ start,
                            int64_t n, int64_t n_edges, const int32_t *__restrict__ rank,
                            uint64_t *__restrict__ dkeys, unsigned long long *__restrict__ n_surf) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t surf = 0;
    if (e < n_edges) {
        const int64_t s = start[e];
        const int64_t last = (e + 1 < n_edges ? start[e + 1] : n) - 1;
        const uint64_t k = keys[s];
        surf = (k & 0xffu) != (keys[last] & 0xffu) ? 1u : 0u;
        const uint64_t a = (uint64_t)rank[k >> 36], b = (uint64_t)rank[(k >> 8) & ((1ull << 28) - 1)];
        dkeys[2 * e] = (a << 32) | (b << 1) | surf;
        dkeys[2 * e + 1] = (b << 32) | (a << 1) | surf;
    }
    // one counter update per block
    __shared__ unsigned int block_count;
    if (threadIdx.x == 0) block_count = 0;
    __syncthreads();
    const unsigned long long m = __ballot(surf != 0);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&block_count, (unsigned int)__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0 && block_count) atomicAdd(n_surf, (unsigned long long)block_count);
}

// Row pointers from the sorted directed keys (rows without an entry get an
// empty range) and the columns with the interface bit.
__global__ void k_csr(const uint64_t *__restrict__ dkeys, int64_t n2, int64_t n_nodes,
                      int64_t *__restrict__ rowptr, uint32_t *__restrict__ cols) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n2) return;
    const uint64_t d = dkeys[k];
    const int64_t r = (int64_t)(d >> 32);
    cols[k] = (uint32_t)((d >> 1) & 0x7fffffffu) | ((d & 1u) ? kSurfBit : 0u);
    const int64_t prev = k == 0 ? -1 : (int64_t)(dkeys[k - 1] >> 32);
    for (int64_t q = prev + 1; q <= r; ++q) rowptr[q] = k;
    if (k == n2 - 1)
        for (int64_t q = r + 1; q <= n_nodes; ++q) rowptr[q] = n2;
}

// Per Morton rank: 0 on a face of the lattice box (never moves); 1 on an
// interface (surface phase); 2 any other node (volume phase).
__global__ void k_node_class(const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ cols,
                             const int64_t *__restrict__ keys, const int32_t *__restrict__ order,
                             int64_t n, LatticeGeom g, uint8_t *__restrict__ cls) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = (uint64_t)keys[order[i]];
    const int64_t f[3] = {(int64_t)((k >> 42) & 0x1fffffu), (int64_t)((k >> 21) & 0x1fffffu),
                          (int64_t)(k & 0x1fffffu)};
    bool box = false;
    for (int a = 0; a < 3; ++a) box |= f[a] == 0 || f[a] == ((int64_t)g.cells[a] << kMaxLevels);
    bool surf = false;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) surf |= (cols[q] & kSurfBit) != 0;
    cls[i] = box ? 0 : (surf ? 1 : 2);
}

// Positions in Morton rank order (rank r holds node order[r]).
__global__ void k_pack_pos(const float *__restrict__ xyz, const int32_t *__restrict__ order, int64_t n,
                           float4 *__restrict__ a, float4 *__restrict__ b) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t i = order[r];
    const float4 p = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], 0.0f);
    a[r] = p;
    b[r] = p;
}

__global__ void k_unpack_pos(const float4 *__restrict__ p, const int32_t *__restrict__ order, int64_t n,
                             float *__restrict__ xyz) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t i = order[r];
    const float4 q = p[r];
    xyz[3 * i] = q.x;
    xyz[3 * i + 1] = q.y;
    xyz[3 * i + 2] = q.z;
}

// Fixed-order block sum of one double per thread into partials[blockIdx.x].
__device__ __forceinline__ void block_sum(double v, double *partials) {
    __shared__ double red[kSmoothThreads];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kSmoothThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// As block_sum, into partials[at] (the block's tile in a remapped grid).
__device__ __forceinline__ void block_sum_at(double v, double *partials, int64_t at) {
    __shared__ double red[kSmoothThreads];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kSmoothThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[at] = red[0];
}

__global__ __launch_bounds__(kSmoothThreads) void k_norm_sq(const float4 *__restrict__ p,
                                                           const int32_t *__restrict__ list,
                                                           int64_t n, double *__restrict__ partials) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (t < n) {
        const float4 q = p[list[t]];
        v = (double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z;
    }
    block_sum(v, partials);
}

__global__ __launch_bounds__(kSmoothThreads) void k_row_entries(const int64_t *__restrict__ rowptr,
                                                               const int32_t *__restrict__ list,
                                                               int64_t n, double *__restrict__ partials) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (t < n) {
        const int32_t i = list[t];
        v = (double)(rowptr[i + 1] - rowptr[i]);
    }
    block_sum(v, partials);
}

// One block: thread j sums partials j, j + 1024, ... in order, then a tree.
__global__ __launch_bounds__(1024) void k_sum_partials(const double *__restrict__ partials, int64_t nb,
                                                       double *__restrict__ out) {
    __shared__ double red[1024];
    double v = 0.0;
    for (int64_t j = threadIdx.x; j < nb; j += 1024) v += partials[j];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Row segment of each listed node: (first entry << 32) | length, so a half
// step reads it with the node id instead of after it.
__global__ void k_row_segments(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ list,
                               int64_t n, uint64_t *__restrict__ seg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t i = list[t];
    const int64_t b = rowptr[i];
    seg[t] = ((uint64_t)b << 32) | (uint64_t)(rowptr[i + 1] - b);
}

// Fixed-stride copy of the first G U columns of each listed row, lane-major
// (see launch_row_heads).
__global__ void k_row_heads(const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ cols,
                            const int32_t *__restrict__ list, int64_t n, uint32_t *__restrict__ head) {
    constexpr int G = kTaubinGroup, U = kTaubinUnroll;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (t, g, u)
    if (k >= n * G * U) return;
    const int64_t t = k / (G * U);
    const int g = (int)(k / U % G), u = (int)(k % U);
    const int32_t i = list[t];
    const int64_t b = rowptr[i], len = rowptr[i + 1] - b;
    const int64_t q = g + (int64_t)u * G;
    head[k] = q < len ? cols[b + q] : 0u;
}

// kTaubinGroup lanes per node, each taking every kTaubinGroup-th entry of
// the row.  The first kTaubinUnroll entries of a lane come from the row
// heads, loaded with the node id and row segment (not after the segment),
// then all their position gathers are issued together: a node costs two
// dependent memory round trips, not two per neighbour (the heads took the
// surface half step on c3 from 0.46 to 0.36 ms and the volume one from 1.30
// to 1.19 ms, same results); longer rows finish in a plain loop over the row
// segment.  The group's double sums are combined by a fixed butterfly and
// its first lane writes the node.
__global__ __launch_bounds__(kSmoothThreads) void k_taubin_half(
    const float4 *__restrict__ in, float4 *__restrict__ out, const uint64_t *__restrict__ seg,
    const uint32_t *__restrict__ head, const uint32_t *__restrict__ cols,
    const int32_t *__restrict__ list, int64_t n, double coef, int surface_only,
    double *__restrict__ partials) {
#pragma clang fp contract(off)
    constexpr int G = kTaubinGroup, U = kTaubinUnroll;
    const int lane = (int)(threadIdx.x & (G - 1));
    // Workgroups go to the 8 XCDs round-robin; tile = the block's place in a
    // grid where each XCD takes one contiguous eighth of the nodes (Morton
    // order), so the neighbour positions a node gathers sit in the L2 of the
    // XCD that gathers them (the grid is a multiple of 8 blocks).
    const int64_t per = (int64_t)gridDim.x / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    const int64_t t = (tile * blockDim.x + threadIdx.x) / G;
    // The block's nodes are consecutive list entries, so their Morton ranks
    // span [list[first], list[last]]; when that range is short, the positions
    // in it are staged in LDS with coalesced loads and every neighbour inside
    // it (most of them: neighbours are close in Morton order) is read from LDS
    // instead of by its own gather.  On c3 a 256-position window took the
    // volume half step from 1.19 to 1.06 ms and the surface one from 0.36 to
    // 0.34 ms (512 and 1024 positions: the same volume time, no surface gain).
    __shared__ float4 win[kTaubinWindow];
    const int64_t tb0 = tile * (blockDim.x / G);
    int64_t w0 = 0, wn = 0;
    if (tb0 < n) {
        const int64_t tb1 = (tb0 + blockDim.x / G < n ? tb0 + blockDim.x / G : n) - 1;
        w0 = list[tb0];
        wn = (int64_t)list[tb1] - w0 + 1;
        if (wn <= 0 || wn > kTaubinWindow) wn = 0;   // (the list is ascending: wn >= 1)
    }
    for (int64_t k = threadIdx.x; k < wn; k += blockDim.x) win[k] = in[w0 + k];
    __syncthreads();
    auto pos = [&](uint32_t j) -> float4 {
        const uint64_t o = (uint64_t)((int64_t)j - w0);
        return o < (uint64_t)wn ? win[o] : in[j];
    };
    double sx = 0.0, sy = 0.0, sz = 0.0;
    int cnt = 0;
    int32_t i = 0;
    if (t < n) {
        i = list[t];
        const uint64_t sg = seg[t];
        const int64_t beg = (int64_t)(sg >> 32), len = (int64_t)(sg & 0xffffffffu);
        const uint32_t need = surface_only ? kSurfBit : 0u;
        // the lane's first U columns: contiguous in `head`, independent of the
        // row segment (0 past the row's end)
        static_assert(U % 4 == 0, "row heads are read as 16-byte vectors");
        uint32_t c[U];
        const uint4 *hv = (const uint4 *)(head + (t * G + lane) * U);
#pragma unroll
        for (int v = 0; v < U / 4; ++v) {
            const uint4 w = hv[v];
            c[4 * v] = w.x;
            c[4 * v + 1] = w.y;
            c[4 * v + 2] = w.z;
            c[4 * v + 3] = w.w;
        }
        float4 p[U];
        unsigned use = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = lane + (int64_t)u * G;
            const bool ok = q < len && (c[u] & need) == need;
            use |= ok ? 1u << u : 0u;
            p[u] = ok ? pos(c[u] & ~kSurfBit) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (use >> u & 1u) {
                sx += (double)p[u].x;
                sy += (double)p[u].y;
                sz += (double)p[u].z;
                ++cnt;
            }
        }
        for (int64_t q = lane + (int64_t)U * G; q < len; q += G) {
            const uint32_t cq = cols[beg + q];
            if ((cq & need) != need) continue;
            const float4 pq = pos(cq & ~kSurfBit);
            sx += (double)pq.x;
            sy += (double)pq.y;
            sz += (double)pq.z;
            ++cnt;
        }
    }
    for (int off = G / 2; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off, G);
        sy += __shfl_xor(sy, off, G);
        sz += __shfl_xor(sz, off, G);
        cnt += __shfl_xor(cnt, off, G);
    }
    double d2 = 0.0;
    if (t < n && lane == 0) {
        const float4 xi = pos((uint32_t)i);
        // mean over the node and its neighbours, then the step toward it
        const double inv = (double)(cnt + 1);
        const double mx = (sx + (double)xi.x) / inv, my = (sy + (double)xi.y) / inv,
                     mz = (sz + (double)xi.z) / inv;
        float4 o;
        o.x = (float)((double)xi.x + coef * (mx - (double)xi.x));
        o.y = (float)((double)xi.y + coef * (my - (double)xi.y));
        o.z = (float)((double)xi.z + coef * (mz - (double)xi.z));
        o.w = 0.0f;
        out[i] = o;
        const double dx = (double)o.x - xi.x, dy = (double)o.y - xi.y, dz = (double)o.z - xi.z;
        d2 = dx * dx + dy * dy + dz * dz;
    }
    block_sum_at(d2, partials, tile);
}

}  // namespace

int64_t smooth_blocks(int64_t n) { return (n + kSmoothThreads - 1) / kSmoothThreads; }
// Blocks of a half step, rounded up to a multiple of the 8 XCDs (the
// trailing blocks find no node and add 0 to the stopping sum).
int64_t taubin_blocks(int64_t n) {
    const int64_t b = (n * kTaubinGroup + kSmoothThreads - 1) / kSmoothThreads;
    return (b + 7) / 8 * 8;
}

hipError_t launch_edge_occurrences(const int32_t *ids, const int32_t *labels, int64_t n_tets,
                                   uint64_t *keys, unsigned long long *bad_labels, hipStream_t s) {
    if (n_tets <= 0) return hipSuccess;
    k_edge_occurrences<<<grid_of(6 * n_tets), kSmoothThreads, 0, s>>>(ids, labels, n_tets, keys,
                                                                       bad_labels);
    return hipGetLastError();
}

hipError_t sort_keys_u64(const uint64_t *in, uint64_t *out, int64_t n, int end_bit, void *tmp,
                         size_t *tmp_bytes, hipStream_t s) {
    return rocprim::radix_sort_keys(tmp, *tmp_bytes, in, out, (size_t)n, 0u, (unsigned)end_bit, s);
}

hipError_t launch_edge_heads(const uint64_t *keys, int64_t n, int32_t *head, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_edge_heads<<<grid_of(n), kSmoothThreads, 0, s>>>(keys, n, head);
    return hipGetLastError();
}

hipError_t exclusive_sum_head(const int32_t *head, int64_t *pos, int64_t n, void *tmp,
                              size_t *tmp_bytes, hipStream_t s) {
    return rocprim::exclusive_scan(tmp, *tmp_bytes, head, pos, (int64_t)0, (size_t)n,
                                   rocprim::plus<int64_t>(), s);
}

hipError_t launch_edge_directed(const uint64_t *keys, const int32_t *head, const int64_t *pos,
                                int64_t n, int64_t n_edges, int64_t *start, const int32_t *rank,
                                uint64_t *dkeys, unsigned long long *n_surf, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_edge_starts<<<grid_of(n), kSmoothThreads, 0, s>>>(head, pos, n, start);
    k_edge_emit<<<grid_of(n_edges), kSmoothThreads, 0, s>>>(keys, start, n, n_edges, rank, dkeys,
                                                           n_surf);
    return hipGetLastError();
}

hipError_t launch_csr(const uint64_t *dkeys, int64_t n2, int64_t n_nodes, int64_t *rowptr,
                      uint32_t *cols, hipStream_t s) {
    if (n2 <= 0) return hipSuccess;
    k_csr<<<grid_of(n2), kSmoothThreads, 0, s>>>(dkeys, n2, n_nodes, rowptr, cols);
    return hipGetLastError();
}

hipError_t launch_morton_order(const int64_t *keys, int64_t n, uint64_t *code, uint64_t *code_sorted,
                               int32_t *ids, int32_t *order, int32_t *rank, void *tmp,
                               size_t *tmp_bytes, hipStream_t s) {
    if (!tmp)
        return rocprim::radix_sort_pairs(tmp, *tmp_bytes, code, code_sorted, ids, order, (size_t)n,
                                         0u, 63u, s);
    if (n <= 0) return hipSuccess;
    k_morton_codes<<<grid_of(n), kSmoothThreads, 0, s>>>(keys, n, code, ids);
    hipError_t e = rocprim::radix_sort_pairs(tmp, *tmp_bytes, code, code_sorted, ids, order,
                                             (size_t)n, 0u, 63u, s);
    if (e != hipSuccess) return e;
    k_rank_of<<<grid_of(n), kSmoothThreads, 0, s>>>(order, n, rank);
    return hipGetLastError();
}

hipError_t launch_node_class(const int64_t *rowptr, const uint32_t *cols, const int64_t *keys,
                             const int32_t *order, int64_t n_nodes, const LatticeGeom &g, uint8_t *cls,
                             hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    k_node_class<<<grid_of(n_nodes), kSmoothThreads, 0, s>>>(rowptr, cols, keys, order, n_nodes, g, cls);
    return hipGetLastError();
}

hipError_t launch_pack_pos(const float *xyz, const int32_t *order, int64_t n, float4 *a, float4 *b,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_pack_pos<<<grid_of(n), kSmoothThreads, 0, s>>>(xyz, order, n, a, b);
    return hipGetLastError();
}

hipError_t launch_unpack_pos(const float4 *p, const int32_t *order, int64_t n, float *xyz,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_unpack_pos<<<grid_of(n), kSmoothThreads, 0, s>>>(p, order, n, xyz);
    return hipGetLastError();
}

hipError_t launch_norm_sq(const float4 *p, const int32_t *list, int64_t n, double *partials,
                          double *sum, hipStream_t s) {
    const int64_t nb = smooth_blocks(n);
    if (nb > 0) k_norm_sq<<<(unsigned)nb, kSmoothThreads, 0, s>>>(p, list, n, partials);
    k_sum_partials<<<1, 1024, 0, s>>>(partials, nb, sum);
    return hipGetLastError();
}

hipError_t launch_row_entries(const int64_t *rowptr, const int32_t *list, int64_t n, double *partials,
                              double *sum, hipStream_t s) {
    const int64_t nb = smooth_blocks(n);
    if (nb > 0) k_row_entries<<<(unsigned)nb, kSmoothThreads, 0, s>>>(rowptr, list, n, partials);
    k_sum_partials<<<1, 1024, 0, s>>>(partials, nb, sum);
    return hipGetLastError();
}

hipError_t launch_row_segments(const int64_t *rowptr, const int32_t *list, int64_t n, uint64_t *seg,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_row_segments<<<grid_of(n), kSmoothThreads, 0, s>>>(rowptr, list, n, seg);
    return hipGetLastError();
}

hipError_t launch_row_heads(const int64_t *rowptr, const uint32_t *cols, const int32_t *list,
                            int64_t n, uint32_t *head, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_row_heads<<<grid_of(n * kTaubinGroup * kTaubinUnroll), kSmoothThreads, 0, s>>>(rowptr, cols,
                                                                                   list, n, head);
    return hipGetLastError();
}

hipError_t launch_taubin_half(const float4 *in, float4 *out, const uint64_t *seg,
                              const uint32_t *head, const uint32_t *cols, const int32_t *list,
                              int64_t n, double coef, int surface_only, double *partials,
                              double *sum, hipStream_t s) {
    const int64_t nb = taubin_blocks(n);
    if (nb > 0)
        k_taubin_half<<<(unsigned)nb, kSmoothThreads, 0, s>>>(in, out, seg, head, cols, list, n,
                                                              coef, surface_only, partials);
    k_sum_partials<<<1, 1024, 0, s>>>(partials, nb, sum);
    return hipGetLastError();
}

}  // namespace sal
