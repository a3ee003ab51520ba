// Kuhn lattice, label-boundary marking, compaction and 1 -> 8 split
// (paper sections 2.1.1-2.1.3).  These passes are index arithmetic and
// gathers, bound by memory traffic, not by arithmetic.
//
// Geometry in lattice units: a level-l tetrahedron is (cell c, permutation
// pi = (p0, p1, p2) of the axes) = {1 >= f[p0] >= f[p1] >= f[p2] >= 0},
// f = u 2^l - c; its vertices are x0 = c, x1 = x0 + e_p0, x2 = x1 + e_p1,
// x3 = c + (1, 1, 1) (scaled by 2^-l).
//
// Same-level face neighbours (each shares the three other vertices):
//   opposite x0: cell + e_p0, (p1, p2, p0)     opposite x1: cell, (p1, p0, p2)
//   opposite x2: cell, (p0, p2, p1)            opposite x3: cell - e_p2, (p2, p0, p1)
// Parent of a level-(l+1) tetrahedron (cell c', pi'): cell c' >> 1 and the
// permutation sorting U_a = 4 (c'_a & 1) + w_a in decreasing order, where
// w[pi'0] = 3, w[pi'1] = 2, w[pi'2] = 1 (U / 8 is the child's centroid in the
// parent cell).
#include <hip/hip_runtime.h>

#include "kuhn_dev.h"
#include "mesh_internal.h"

namespace sal {
namespace {

// Centroid: origin + h 2^-l (c + offset), each coordinate by lattice_coord.
__device__ __forceinline__ void centroid(const LatticeGeom &g, int l, int q, const int64_t c[3],
                                         float &x, float &y, float &z) {
    int p0, p1, p2;
    perm_of(q, p0, p1, p2);
    double off[3];
    off[p0] = 0.75;
    off[p1] = 0.5;
    off[p2] = 0.25;
    const double hl = ldexp(g.h, -l);
    x = lattice_coord(g.origin[0], hl, (double)c[0] + off[0]);
    y = lattice_coord(g.origin[1], hl, (double)c[1] + off[1]);
    z = lattice_coord(g.origin[2], hl, (double)c[2] + off[2]);
}

__global__ void k_lattice_centroids(LatticeGeom g, int64_t n0, float *__restrict__ cx,
                                    float *__restrict__ cy, float *__restrict__ cz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n0) return;
    const int q = (int)(i % 6);
    int64_t cell = i / 6;
    int64_t c[3];
    c[0] = cell % g.cells[0];
    cell /= g.cells[0];
    c[1] = cell % g.cells[1];
    c[2] = cell / g.cells[1];
    centroid(g, 0, q, c, cx[i], cy[i], cz[i]);
}

// The leaf containing the level-l tetrahedron (c, q): its (level, index), or
// level -1 when (c, q) is itself refined (then its descendants are leaves).
__device__ __forceinline__ void resolve(const LevelPtrs &L, const LatticeGeom &g,
                                        const ChildTables &T, int l, int q, const int64_t c[3],
                                        int &lv_out, int64_t &idx_out) {
    int qa[kMaxLevels + 1];
    int64_t ca[kMaxLevels + 1][3];
    int rank[kMaxLevels + 1];
    qa[l] = q;
    ca[l][0] = c[0]; ca[l][1] = c[1]; ca[l][2] = c[2];
    for (int lv = l; lv > 0; --lv) {
        int p0, p1, p2;
        perm_of(qa[lv], p0, p1, p2);
        int w[3];
        w[p0] = 3; w[p1] = 2; w[p2] = 1;
        int U[3];
        int dcode = 0;
        for (int a = 0; a < 3; ++a) {
            const int d = (int)(ca[lv][a] & 1);
            U[a] = 4 * d + w[a];
            dcode |= d << a;
            ca[lv - 1][a] = ca[lv][a] >> 1;
        }
        // axes in decreasing U
        int s0 = 0, s1 = 1, s2 = 2, tmp;
        if (U[s1] > U[s0]) { tmp = s0; s0 = s1; s1 = tmp; }
        if (U[s2] > U[s1]) { tmp = s1; s1 = s2; s2 = tmp; }
        if (U[s1] > U[s0]) { tmp = s0; s0 = s1; s1 = tmp; }
        qa[lv - 1] = q_of(s0, s1, s2);
        rank[lv] = T.rank[qa[lv - 1]][dcode][qa[lv]];
    }
    int64_t idx = ((ca[0][2] * g.cells[1] + ca[0][1]) * g.cells[0] + ca[0][0]) * 6 + qa[0];
    for (int lv = 0;; ++lv) {
        const int32_t ch = L.child[lv][idx];
        if (ch < 0) { lv_out = lv; idx_out = idx; return; }
        if (lv == l) { lv_out = -1; idx_out = -1; return; }
        idx = 8 * (int64_t)ch + rank[lv + 1];
    }
}

// Section 2.1.3 (Fig. 3): a leaf is on a tissue boundary when a leaf sharing a
// 2-D part of one of its faces carries another label.  Each leaf looks across
// its four faces at the same level; when the other side is a leaf (or lies in
// a coarser leaf) with another label, both are flagged.  When the other side
// is finer, its leaves find this one the same way, so every pair is seen.
__device__ __forceinline__ int64_t level_n(const LevelPtrs &L, int l) {
    return L.n_dev ? L.n_dev[l] : L.n[l];
}

__device__ void mark_one(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                         int64_t i) {
    if (L.child[l][i] >= 0) return;
    const int32_t lab = L.label[l][i];
    int q, lk;
    int64_t c[3];
    split_key(entry_key(L, g, l, i), lk, q, c);
    int p0, p1, p2;
    perm_of(q, p0, p1, p2);
    const int64_t lim[3] = {(int64_t)g.cells[0] << l, (int64_t)g.cells[1] << l,
                            (int64_t)g.cells[2] << l};
    bool mine = false;
    for (int f = 0; f < 4; ++f) {
        int64_t nc[3] = {c[0], c[1], c[2]};
        int nq;
        if (f == 0) { nc[p0] += 1; nq = q_of(p1, p2, p0); }
        else if (f == 1) { nq = q_of(p1, p0, p2); }
        else if (f == 2) { nq = q_of(p0, p2, p1); }
        else { nc[p2] -= 1; nq = q_of(p2, p0, p1); }
        if (nc[0] < 0 || nc[1] < 0 || nc[2] < 0 || nc[0] >= lim[0] || nc[1] >= lim[1] ||
            nc[2] >= lim[2])
            continue;   // domain boundary
        int lv;
        int64_t j;
        resolve(L, g, T, l, nq, nc, lv, j);
        if (lv < 0) continue;
        if (L.label[lv][j] != lab) {
            mine = true;
            L.flag[lv][j] = 1;
        }
    }
    if (mine) L.flag[l][i] = 1;
}

__global__ void k_mark(LevelPtrs L, LatticeGeom g, ChildTables T, int l) {
    const int64_t n = level_n(L, l);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        mark_one(L, g, T, l, i);
}

// ------------------------------------------------------------- compaction
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ bool pred(const CompactSrc &s, int64_t i) {
    return s.flag ? (s.flag[i] & (s.mask ? s.mask : 0xffu)) != 0 : s.child[i] < 0;
}

// Each thread owns kScanItems consecutive entries of its tile: one 16-byte
// load of flag bytes (or four of int32 children) instead of one narrow load
// per entry.  Returns the entries' predicate bits (bit j: entry first + j).
// The wide loads need the whole run inside [0, n) and a 16-byte aligned
// base; otherwise (the tail, or a misaligned array) entries are read one by one.
static_assert(kScanItems == 16, "one 16-byte flag load per thread");
__device__ __forceinline__ uint32_t pred_bits(const CompactSrc &s, int64_t first, int64_t n) {
    uint32_t bits = 0;
    const bool whole = first + kScanItems <= n;
    if (s.flag) {
        const uint32_t mk = s.mask ? s.mask : 0xffu;
        if (whole && (((uintptr_t)(s.flag + first)) & 15u) == 0) {
            const uint4 w = *(const uint4 *)(s.flag + first);
            const uint32_t m4 = mk * 0x01010101u;
            const uint32_t words[4] = {w.x & m4, w.y & m4, w.z & m4, w.w & m4};
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    bits |= (((words[q] >> (8 * b)) & 0xffu) != 0u ? 1u : 0u) << (4 * q + b);
        } else {
            for (int j = 0; j < kScanItems; ++j)
                if (first + j < n && (s.flag[first + j] & mk) != 0) bits |= 1u << j;
        }
    } else {
        if (whole && (((uintptr_t)(s.child + first)) & 15u) == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int4 c = *(const int4 *)(s.child + first + 4 * q);
                bits |= (c.x < 0 ? 1u : 0u) << (4 * q);
                bits |= (c.y < 0 ? 1u : 0u) << (4 * q + 1);
                bits |= (c.z < 0 ? 1u : 0u) << (4 * q + 2);
                bits |= (c.w < 0 ? 1u : 0u) << (4 * q + 3);
            }
        } else {
            for (int j = 0; j < kScanItems; ++j)
                if (first + j < n && s.child[first + j] < 0) bits |= 1u << j;
        }
    }
    return bits;
}

__global__ __launch_bounds__(kScanThreads) void k_count(CompactSrc s, int64_t n,
                                                        const int64_t *__restrict__ n_dev,
                                                        int64_t *__restrict__ block_counts) {
    __shared__ int red[kScanThreads];
    if (n_dev) n = *n_dev;
    const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    red[threadIdx.x] = first < n ? __popc(pred_bits(s, first, n)) : 0;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_counts[blockIdx.x] = red[0];
}

// Exclusive scan of n_blocks counts in one workgroup; total -> *total.
__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t *__restrict__ counts, int64_t n_blocks,
                                                     int64_t *__restrict__ total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n_blocks + 1023) / 1024;
    const int64_t b0 = t * per, b1 = b0 + per < n_blocks ? b0 + per : n_blocks;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += counts[b];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;   // exclusive prefix of this thread's chunk
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t c = counts[b];
        counts[b] = run;
        run += c;
    }
    if (t == 1023) *total = part[1023];
}

// Ordered scatter of one tile: thread t owns the kScanItems consecutive
// entries starting at tile + t kScanItems (so thread order is index order);
// a scan of the per-thread counts across the workgroup gives each thread its
// place, the tile's indices are staged in LDS in index order, then written
// out contiguously (coalesced writes).
constexpr int kScanWaves = kScanThreads / 64;

__global__ __launch_bounds__(kScanThreads) void k_scatter(CompactSrc s, int64_t n,
                                                          const int64_t *__restrict__ n_dev,
                                                          const int64_t *__restrict__ offsets,
                                                          int32_t *__restrict__ out) {
    __shared__ int32_t buf[kScanTile];
    __shared__ int wave_total[kScanWaves];
    if (n_dev) n = *n_dev;
    const int lane = (int)(threadIdx.x & 63u);
    const int wv = (int)(threadIdx.x >> 6);
    const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t bits = first < n ? pred_bits(s, first, n) : 0u;
    const int cnt = __popc(bits);
    // inclusive scan of the counts over the wavefront's lanes
    int inc = cnt;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wave_total[wv] = inc;
    __syncthreads();
    int run = 0, total = 0;
    for (int w = 0; w < kScanWaves; ++w) {
        if (w < wv) run += wave_total[w];
        total += wave_total[w];
    }
    int pos = run + inc - cnt;
    while (bits) {
        const int j = __builtin_ctz(bits);
        bits &= bits - 1u;
        buf[pos++] = (int32_t)(first + j);
    }
    __syncthreads();
    const int64_t o = offsets[blockIdx.x];
    for (int j = (int)threadIdx.x; j < total; j += kScanThreads) out[o + j] = buf[j];
}

// Section 2.1.2: each listed leaf of level l becomes 8 level-(l+1) tetrahedra
// (red refinement); they are appended as one block, their centroids written
// to the labeling scratch.  jj = 8 (list position) + child rank.
__device__ void split_one(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                          const int32_t *__restrict__ list, int64_t jj, int64_t base_block,
                          float *__restrict__ cx, float *__restrict__ cy, float *__restrict__ cz) {
    const int64_t j = jj >> 3;
    const int r = (int)(jj & 7);
    const int64_t i = list[j];
    int q, lk;
    int64_t c[3];
    split_key(entry_key(L, g, l, i), lk, q, c);
    const int64_t b = base_block + j;
    if (r == 0) L.child[l][i] = (int32_t)b;
    const int dcode = T.list[q][r][0];
    const int cq = T.list[q][r][1];
    int64_t cc[3];
    for (int a = 0; a < 3; ++a) cc[a] = 2 * c[a] + ((dcode >> a) & 1);
    const int64_t o = 8 * b + r;
    L.key[l + 1][o] = make_key(l + 1, cq, cc[0], cc[1], cc[2]);
    L.child[l + 1][o] = -1;
    L.label[l + 1][o] = L.inherit ? L.label[l][i] : -2;
    if (cx) centroid(g, l + 1, cq, cc, cx[jj], cy[jj], cz[jj]);
}

__global__ void k_split(LevelPtrs L, LatticeGeom g, ChildTables T, int l,
                        const int32_t *__restrict__ list, int64_t count, int64_t base_block,
                        float *__restrict__ cx, float *__restrict__ cy, float *__restrict__ cz) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= count * 8) return;
    split_one(L, g, T, l, list, jj, base_block, cx, cy, cz);
}

// ------------------------------------------------------- four-node rule
// Section 2.1.3 as printed: the solid-angle test is applied to the nodes, and
// a tetrahedron belongs to a surface when all four of its nodes are enclosed.
// Node enclosure masks: level-0 nodes in a dense (nx+1)(ny+1)(nz+1) grid,
// nodes added by a split (edge midpoints) carried per child tetrahedron as
// the masks of its four vertices (x0..x3 in its own Kuhn order).

__device__ __forceinline__ int32_t mask_label(const SurfaceDev *surf, uint64_t m) {
    return m ? surf[63 - __builtin_clzll(m)].label : 0;
}

__global__ void k_lattice_nodes(LatticeGeom g, int64_t n_nodes, float *__restrict__ x,
                                float *__restrict__ y, float *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const int64_t nx1 = g.cells[0] + 1, ny1 = g.cells[1] + 1;
    const int64_t u = i % nx1, v = (i / nx1) % ny1, w = i / (nx1 * ny1);
    x[i] = lattice_coord(g.origin[0], g.h, (double)u);
    y[i] = lattice_coord(g.origin[1], g.h, (double)v);
    z[i] = lattice_coord(g.origin[2], g.h, (double)w);
}

__device__ __forceinline__ int64_t node0_index(const LatticeGeom &g, const int64_t X[3]) {
    return (X[2] * (g.cells[1] + 1) + X[1]) * (int64_t)(g.cells[0] + 1) + X[0];
}

// Level-0 labels from the node grid.
__global__ void k_elem_from_nodes0(LatticeGeom g, int64_t n0,
                                   const unsigned long long *__restrict__ node0,
                                   const SurfaceDev *__restrict__ surf,
                                   int32_t *__restrict__ label0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n0) return;
    const int q = (int)(i % 6);
    int64_t cell = i / 6;
    int64_t c[3];
    c[0] = cell % g.cells[0];
    cell /= g.cells[0];
    c[1] = cell % g.cells[1];
    c[2] = cell / g.cells[1];
    int64_t X[4][3];
    kuhn_vertices(q, c, X);
    uint64_t m = ~0ull;
    for (int v = 0; v < 4; ++v) m &= node0[node0_index(g, X[v])];
    label0[i] = mask_label(surf, m);
}

// The six edge midpoints of every listed level-l leaf (edges 01, 02, 03, 12,
// 13, 23), in millimetres, into the labeling scratch: origin + h 2^-(l+1)
// (X_a + X_b), products and sums rounded once in double, then to float.
__global__ void k_midpoints(LevelPtrs L, LatticeGeom g, int l, const int32_t *__restrict__ list,
                            int64_t count, float *__restrict__ mx, float *__restrict__ my,
                            float *__restrict__ mz, uint64_t *__restrict__ mkey) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= count * 6) return;
    const int64_t j = jj / 6;
    const int e = (int)(jj - j * 6);
    int q, lk;
    int64_t c[3];
    split_key(entry_key(L, g, l, list[j]), lk, q, c);
    int64_t X[4][3];
    kuhn_vertices(q, c, X);
    const int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
    const double hl = ldexp(g.h, -(l + 1));
    float *out[3] = {mx, my, mz};
    for (int a = 0; a < 3; ++a)
        out[a][jj] = lattice_coord(g.origin[a], hl, (double)(X[ea[e]][a] + X[eb[e]][a]));
    // node key: coordinates on the level-kMaxLevels grid, 21 bits each
    const int sh = kMaxLevels - (l + 1);
    uint64_t key = 0;
    for (int a = 0; a < 3; ++a)
        key = (key << 21) | (uint64_t)((X[ea[e]][a] + X[eb[e]][a]) << sh);
    mkey[jj] = key;
}

// ------------------------------------------------------------ node table
// Open-addressing hash table of the nodes labeled after a split (keys on the
// finest grid, linear probing), so a node shared by several split leaves, or
// labeled in an earlier round, is labeled once.
constexpr uint64_t kEmptyKey = ~0ull;

__device__ __forceinline__ uint64_t node_hash(uint64_t k) {
    // splitmix64 finaliser
    k ^= k >> 30;
    k *= 0xbf58476d1ce4e5b9ull;
    k ^= k >> 27;
    k *= 0x94d049bb133111ebull;
    k ^= k >> 31;
    return k;
}

// Inserts every midpoint key; the thread whose insert creates the entry lists
// the midpoint as a new node.  slot[jj] = the key's table slot.
__global__ void k_node_insert(const uint64_t *__restrict__ mkey, int64_t n,
                              unsigned long long *__restrict__ tkeys, int64_t cap,
                              int64_t *__restrict__ slot, int32_t *__restrict__ new_list,
                              unsigned long long *__restrict__ n_new) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= n) return;
    const uint64_t key = mkey[jj];
    uint64_t h = node_hash(key) & (uint64_t)(cap - 1);
    for (int64_t probe = 0; probe < cap; ++probe) {
        const unsigned long long prev = atomicCAS(&tkeys[h], kEmptyKey, key);
        if (prev == kEmptyKey) {
            slot[jj] = (int64_t)h;
            new_list[atomicAdd(n_new, 1ull)] = (int32_t)jj;
            return;
        }
        if (prev == key) {
            slot[jj] = (int64_t)h;
            return;
        }
        h = (h + 1) & (uint64_t)(cap - 1);
    }
    slot[jj] = -1;   // table full (the host keeps it at most half full)
}

// The new nodes' coordinates, compacted for labeling.
__global__ void k_node_gather(const int32_t *__restrict__ new_list,
                              const unsigned long long *__restrict__ n_new,
                              const float *__restrict__ mx, const float *__restrict__ my,
                              const float *__restrict__ mz, float *__restrict__ x,
                              float *__restrict__ y, float *__restrict__ z) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)*n_new) return;
    const int32_t jj = new_list[t];
    x[t] = mx[jj];
    y[t] = my[jj];
    z[t] = mz[jj];
}

__global__ void k_node_store(const int32_t *__restrict__ new_list,
                             const unsigned long long *__restrict__ n_new,
                             const int64_t *__restrict__ slot,
                             const unsigned long long *__restrict__ masks,
                             unsigned long long *__restrict__ tmasks) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)*n_new) return;
    tmasks[slot[new_list[t]]] = masks[t];
}

// Midpoint masks from the table, in midpoint order.
__global__ void k_node_fetch(const int64_t *__restrict__ slot, int64_t n,
                             const unsigned long long *__restrict__ tmasks,
                             unsigned long long *__restrict__ out) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= n) return;
    const int64_t sl = slot[jj];
    out[jj] = sl >= 0 ? tmasks[sl] : 0ull;
}

// Re-inserts the entries of an old table into a larger one.
__global__ void k_node_rehash(const unsigned long long *__restrict__ okeys,
                              const unsigned long long *__restrict__ omasks, int64_t ocap,
                              unsigned long long *__restrict__ tkeys,
                              unsigned long long *__restrict__ tmasks, int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ocap) return;
    const uint64_t key = okeys[i];
    if (key == kEmptyKey) return;
    uint64_t h = node_hash(key) & (uint64_t)(cap - 1);
    for (int64_t probe = 0; probe < cap; ++probe) {
        if (atomicCAS(&tkeys[h], kEmptyKey, key) == kEmptyKey) {
            tmasks[h] = omasks[i];
            return;
        }
        h = (h + 1) & (uint64_t)(cap - 1);
    }
}

// Vertex masks and labels of the 8 children of every listed level-l leaf:
// each child vertex is one of the parent's 10 nodes at level l + 1 (2 X_i, or
// X_a + X_b for an edge), matched by integer coordinates.
__global__ void k_child_masks(LevelPtrs L, LatticeGeom g, int l, const int32_t *__restrict__ list,
                              int64_t count, int64_t base_block,
                              const unsigned long long *__restrict__ node0,
                              const unsigned long long *__restrict__ vmask_parent,
                              const unsigned long long *__restrict__ mid_masks,
                              unsigned long long *__restrict__ vmask_child,
                              const SurfaceDev *__restrict__ surf) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= count * 8) return;
    const int64_t j = jj >> 3;
    const int r = (int)(jj & 7);
    const int64_t i = list[j];
    int q, lk;
    int64_t c[3];
    split_key(entry_key(L, g, l, i), lk, q, c);
    int64_t X[4][3];
    kuhn_vertices(q, c, X);
    int64_t N[10][3];
    uint64_t M[10];
    for (int v = 0; v < 4; ++v) {
        for (int a = 0; a < 3; ++a) N[v][a] = 2 * X[v][a];
        M[v] = l == 0 ? node0[node0_index(g, X[v])] : vmask_parent[4 * i + v];
    }
    const int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
    for (int e = 0; e < 6; ++e) {
        for (int a = 0; a < 3; ++a) N[4 + e][a] = X[ea[e]][a] + X[eb[e]][a];
        M[4 + e] = mid_masks[6 * j + e];
    }
    const int64_t o = 8 * (base_block + j) + r;
    int cq, clk;
    int64_t cc[3];
    split_key(L.key[l + 1][o], clk, cq, cc);
    int64_t Y[4][3];
    kuhn_vertices(cq, cc, Y);
    uint64_t all = ~0ull;
    for (int v = 0; v < 4; ++v) {
        uint64_t mv = 0;
        for (int n = 0; n < 10; ++n)
            if (N[n][0] == Y[v][0] && N[n][1] == Y[v][1] && N[n][2] == Y[v][2]) mv = M[n];
        vmask_child[4 * o + v] = mv;
        all &= mv;
    }
    L.label[l + 1][o] = mask_label(surf, all);
}

// ------------------------------------------------- captured refine round
// These kernels take every size from RoundState or the compaction totals, so
// the same launch sequence serves every round; fixed grids stride over them.
constexpr int kDevGrid = 2048;

__global__ void k_round_begin(RoundState *rs, unsigned long long *counters) {
    const int t = threadIdx.x;
    if (t < kNumCounters) counters[t] = 0ull;
    if (t == 0) rs->n_kids = 0;
}

__global__ void k_clear_flags_dev(uint8_t *__restrict__ flag, const int64_t *__restrict__ n_dev) {
    const int64_t n = *n_dev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) flag[i] = 0;
}

// One thread: sizes of this round's splits (levels deepest first, as the
// host-driven round orders them), capacity checks, new level sizes.
__global__ void k_plan(RoundState *rs, const int64_t *__restrict__ totals) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    rs->n_kids = 0;
    if (rs->status) return;
    if (rs->round > kMaxLevels) { rs->status = 2; return; }
    int64_t cnt[kMaxLevels + 1];
    int64_t boundary = 0;
    for (int l = 0; l <= kMaxLevels; ++l) {
        cnt[l] = totals[l];
        boundary += cnt[l];
    }
    if (cnt[kMaxLevels] > 0) { rs->status = 2; return; }
    int64_t run = 0;
    for (int l = kMaxLevels - 1; l >= 0; --l) {
        if (rs->n[l + 1] + 8 * cnt[l] > rs->cap[l + 1]) { rs->status = 1; return; }
        rs->kid_off[l] = run;
        run += 8 * cnt[l];
    }
    if (run > rs->kid_cap) { rs->status = 1; return; }
    for (int l = kMaxLevels - 1; l >= 0; --l) {
        rs->base_block[l] = rs->n[l + 1] / 8;
        rs->n[l + 1] += 8 * cnt[l];
    }
    rs->n_kids = run;
    rs->n_leaves += 7 * boundary;
    RoundStat &st = rs->stat[rs->round];
    st.n_leaves = rs->n_leaves;
    st.n_boundary = boundary;
    st.n_labeled = run;
}

__global__ void k_split_dev(LevelPtrs L, LatticeGeom g, ChildTables T, int l,
                            const int32_t *__restrict__ list, const int64_t *__restrict__ totals,
                            const RoundState *__restrict__ rs, float *__restrict__ cx,
                            float *__restrict__ cy, float *__restrict__ cz) {
    if (rs->status) return;
    const int64_t n = 8 * totals[l];
    const int64_t base_block = rs->base_block[l];
    const int64_t off = rs->kid_off[l];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; jj < n; jj += stride)
        split_one(L, g, T, l, list, jj, base_block, cx + off, cy + off, cz + off);
}

// Copies the children's labels from the labeling scratch into level l + 1.
__global__ void k_commit(const RoundState *__restrict__ rs, const int64_t *__restrict__ totals,
                         int l, const int32_t *__restrict__ scratch_labels,
                         int32_t *__restrict__ level_labels) {
    if (rs->status) return;
    const int64_t n = 8 * totals[l];
    const int32_t *src = scratch_labels + rs->kid_off[l];
    int32_t *dst = level_labels + 8 * rs->base_block[l];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
        dst[j] = src[j];
}

__global__ void k_round_end(RoundState *rs, const unsigned long long *__restrict__ counters) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (rs->status) return;
    rs->stat[rs->round].n_recheck_pairs = (int64_t)counters[kCntRecheck];
    rs->round += 1;
}

__global__ void k_export(LevelPtrs L, LatticeGeom g, int l, const int32_t *__restrict__ list,
                         int64_t count, int64_t out_base, uint64_t *__restrict__ keys,
                         int32_t *__restrict__ labels, float *__restrict__ cx,
                         float *__restrict__ cy, float *__restrict__ cz) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const int64_t i = list[j];
    const int64_t o = out_base + j;
    const uint64_t key = entry_key(L, g, l, i);
    if (keys) keys[o] = key;
    if (labels) labels[o] = L.label[l][i];
    if (cx || cy || cz) {
        int q, lk;
        int64_t c[3];
        split_key(key, lk, q, c);
        float x, y, z;
        centroid(g, l, q, c, x, y, z);
        if (cx) cx[o] = x;
        if (cy) cy[o] = y;
        if (cz) cz[o] = z;
    }
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

hipError_t launch_lattice_nodes(const LatticeGeom &g, int64_t n_nodes, float *x, float *y, float *z,
                               hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    k_lattice_nodes<<<grid_for(n_nodes, 256), 256, 0, s>>>(g, n_nodes, x, y, z);
    return hipGetLastError();
}

hipError_t launch_elem_from_nodes0(const LatticeGeom &g, int64_t n0,
                                   const unsigned long long *node0, const SurfaceDev *surf,
                                   int32_t *label0, hipStream_t s) {
    if (n0 <= 0) return hipSuccess;
    k_elem_from_nodes0<<<grid_for(n0, 256), 256, 0, s>>>(g, n0, node0, surf, label0);
    return hipGetLastError();
}

hipError_t launch_midpoints(const LevelPtrs &L, const LatticeGeom &g, int l, const int32_t *list,
                            int64_t count, float *mx, float *my, float *mz, uint64_t *mkey,
                            hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_midpoints<<<grid_for(count * 6, 256), 256, 0, s>>>(L, g, l, list, count, mx, my, mz, mkey);
    return hipGetLastError();
}

hipError_t launch_node_insert(const uint64_t *mkey, int64_t n, unsigned long long *tkeys,
                              int64_t cap, int64_t *slot, int32_t *new_list,
                              unsigned long long *n_new, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_node_insert<<<grid_for(n, 256), 256, 0, s>>>(mkey, n, tkeys, cap, slot, new_list, n_new);
    return hipGetLastError();
}

hipError_t launch_node_gather(const int32_t *new_list, const unsigned long long *n_new,
                              int64_t n_cap, const float *mx, const float *my, const float *mz,
                              float *x, float *y, float *z, hipStream_t s) {
    if (n_cap <= 0) return hipSuccess;
    k_node_gather<<<grid_for(n_cap, 256), 256, 0, s>>>(new_list, n_new, mx, my, mz, x, y, z);
    return hipGetLastError();
}

hipError_t launch_node_store(const int32_t *new_list, const unsigned long long *n_new,
                             int64_t n_cap, const int64_t *slot, const unsigned long long *masks,
                             unsigned long long *tmasks, hipStream_t s) {
    if (n_cap <= 0) return hipSuccess;
    k_node_store<<<grid_for(n_cap, 256), 256, 0, s>>>(new_list, n_new, slot, masks, tmasks);
    return hipGetLastError();
}

hipError_t launch_node_fetch(const int64_t *slot, int64_t n, const unsigned long long *tmasks,
                             unsigned long long *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_node_fetch<<<grid_for(n, 256), 256, 0, s>>>(slot, n, tmasks, out);
    return hipGetLastError();
}

hipError_t launch_node_rehash(const unsigned long long *okeys, const unsigned long long *omasks,
                              int64_t ocap, unsigned long long *tkeys, unsigned long long *tmasks,
                              int64_t cap, hipStream_t s) {
    if (ocap <= 0) return hipSuccess;
    k_node_rehash<<<grid_for(ocap, 256), 256, 0, s>>>(okeys, omasks, ocap, tkeys, tmasks, cap);
    return hipGetLastError();
}

hipError_t launch_child_masks(const LevelPtrs &L, const LatticeGeom &g, int l,
                              const int32_t *list, int64_t count, int64_t base_block,
                              const unsigned long long *node0,
                              const unsigned long long *vmask_parent,
                              const unsigned long long *mid_masks,
                              unsigned long long *vmask_child, const SurfaceDev *surf,
                              hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_child_masks<<<grid_for(count * 8, 256), 256, 0, s>>>(L, g, l, list, count, base_block, node0,
                                                          vmask_parent, mid_masks, vmask_child,
                                                          surf);
    return hipGetLastError();
}

hipError_t launch_lattice_centroids(const LatticeGeom &g, int64_t n0, float *cx, float *cy,
                                    float *cz, hipStream_t s) {
    if (n0 <= 0) return hipSuccess;
    k_lattice_centroids<<<grid_for(n0, 256), 256, 0, s>>>(g, n0, cx, cy, cz);
    return hipGetLastError();
}

hipError_t launch_mark(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                       hipStream_t s) {
    if (L.n_dev) {
        k_mark<<<kDevGrid, 256, 0, s>>>(L, g, T, l);
        return hipGetLastError();
    }
    if (L.n[l] <= 0) return hipSuccess;
    k_mark<<<grid_for(L.n[l], 256), 256, 0, s>>>(L, g, T, l);
    return hipGetLastError();
}

int64_t compact_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_compact(const CompactSrc &src, int64_t n, int64_t *block_scratch,
                          int64_t *total, int32_t *out, hipStream_t s) {
    const int64_t nb = compact_blocks(n);
    if (nb <= 0) return launch_fill_u64((unsigned long long *)total, 0ull, 1, s);
    k_count<<<(unsigned)nb, kScanThreads, 0, s>>>(src, n, nullptr, block_scratch);
    k_scan_blocks<<<1, 1024, 0, s>>>(block_scratch, nb, total);
    k_scatter<<<(unsigned)nb, kScanThreads, 0, s>>>(src, n, nullptr, block_scratch, out);
    return hipGetLastError();
}

hipError_t launch_round_begin(RoundState *rs, unsigned long long *counters, hipStream_t s) {
    k_round_begin<<<1, 64, 0, s>>>(rs, counters);
    return hipGetLastError();
}

hipError_t launch_clear_flags_dev(uint8_t *flag, const int64_t *n_dev, hipStream_t s) {
    k_clear_flags_dev<<<kDevGrid, 256, 0, s>>>(flag, n_dev);
    return hipGetLastError();
}

// Tiles for `cap` entries; tiles past the device-side size count nothing.
hipError_t launch_compact_dev(const CompactSrc &src, const int64_t *n_dev, int64_t cap,
                              int64_t *block_scratch, int64_t *total, int32_t *out, hipStream_t s) {
    const int64_t nb = compact_blocks(cap);
    if (nb <= 0) return launch_fill_u64((unsigned long long *)total, 0ull, 1, s);
    k_count<<<(unsigned)nb, kScanThreads, 0, s>>>(src, cap, n_dev, block_scratch);
    k_scan_blocks<<<1, 1024, 0, s>>>(block_scratch, nb, total);
    k_scatter<<<(unsigned)nb, kScanThreads, 0, s>>>(src, cap, n_dev, block_scratch, out);
    return hipGetLastError();
}

hipError_t launch_plan(RoundState *rs, const int64_t *totals, hipStream_t s) {
    k_plan<<<1, 64, 0, s>>>(rs, totals);
    return hipGetLastError();
}

hipError_t launch_split_dev(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                            const int32_t *list, const int64_t *totals, const RoundState *rs,
                            float *cx, float *cy, float *cz, hipStream_t s) {
    k_split_dev<<<kDevGrid, 256, 0, s>>>(L, g, T, l, list, totals, rs, cx, cy, cz);
    return hipGetLastError();
}

hipError_t launch_commit(const RoundState *rs, const int64_t *totals, int l,
                         const int32_t *scratch_labels, int32_t *level_labels, hipStream_t s) {
    k_commit<<<kDevGrid, 256, 0, s>>>(rs, totals, l, scratch_labels, level_labels);
    return hipGetLastError();
}

hipError_t launch_round_end(RoundState *rs, const unsigned long long *counters, hipStream_t s) {
    k_round_end<<<1, 64, 0, s>>>(rs, counters);
    return hipGetLastError();
}

hipError_t launch_split(const LevelPtrs &L, const LatticeGeom &g, const ChildTables &T, int l,
                        const int32_t *list, int64_t count, int64_t base_block, float *cx,
                        float *cy, float *cz, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_split<<<grid_for(count * 8, 256), 256, 0, s>>>(L, g, T, l, list, count, base_block, cx, cy,
                                                    cz);
    return hipGetLastError();
}

hipError_t launch_export(const LevelPtrs &L, const LatticeGeom &g, int l, const int32_t *list,
                         int64_t count, int64_t out_base, uint64_t *keys, int32_t *labels,
                         float *cx, float *cy, float *cz, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_export<<<grid_for(count, 256), 256, 0, s>>>(L, g, l, list, count, out_base, keys, labels,
                                                  cx, cy, cz);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_u8<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace sal
