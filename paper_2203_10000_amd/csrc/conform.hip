// Conforming transition refinement of the leaf set (paper section 2.1.2,
// Fig. 2c-e) and the conforming mesh it gives: explicit tetrahedra over
// numbered nodes.
//
// A leaf edge is *hanging* when its midpoint is a vertex of another leaf; a
// node at a quarter point means a neighbour two or more levels finer.  The
// patterns the paper splits are one hanging edge (2 tetrahedra), two hanging
// edges of one face (3) and the three edges of one face (4); a leaf with any
// other pattern is split into its 8 children (labels kept) and the patterns
// are found again (closure, driven from mesh.cpp).  Nodes are points of the
// finest grid (level kMaxLevels), keyed by 21-bit coordinates.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "kuhn_dev.h"
#include "mesh_internal.h"

namespace sal {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr unsigned kDeep = 1u << 6;   // an edge has a node at a quarter point
constexpr unsigned kRed = 1u << 7;    // pattern not split by the paper: split 1 -> 8

// The four vertices of leaf (l, i) on the finest grid.
__device__ __forceinline__ void leaf_fine_vertices(const LevelPtrs &L, const LatticeGeom &g, int l,
                                                   int64_t i, int64_t F[4][3]) {
    int lk, q;
    int64_t c[3];
    split_key(entry_key(L, g, l, i), lk, q, c);
    kuhn_vertices(q, c, F);
    const int sh = kMaxLevels - l;
    for (int v = 0; v < 4; ++v)
        for (int a = 0; a < 3; ++a) F[v][a] <<= sh;
}

__device__ __forceinline__ uint64_t fine_key(const int64_t f[3]) {
    return ((uint64_t)f[0] << 42) | ((uint64_t)f[1] << 21) | (uint64_t)f[2];
}

__device__ __forceinline__ uint64_t set_hash(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ bool set_find(const unsigned long long *tkeys, int64_t cap, uint64_t key) {
    uint64_t h = set_hash(key) & (uint64_t)(cap - 1);
    for (int64_t probe = 0; probe < cap; ++probe) {
        const uint64_t k = tkeys[h];
        if (k == key) return true;
        if (k == kEmpty) return false;
        h = (h + 1) & (uint64_t)(cap - 1);
    }
    return false;
}

// Inserts key; *added tells whether it was new.  False when the table is full.
// A slot only ever changes from empty to a key, so a key read with a plain
// load is final: most inserts find their key already there (a vertex is
// shared by many leaves) and need no atomic; an empty slot is claimed with a
// compare-and-swap.
__device__ __forceinline__ bool set_insert(unsigned long long *tkeys, int64_t cap, uint64_t key,
                                           bool *added) {
    uint64_t h = set_hash(key) & (uint64_t)(cap - 1);
    for (int64_t probe = 0; probe < cap; ++probe) {
        unsigned long long cur = __atomic_load_n(&tkeys[h], __ATOMIC_RELAXED);
        if (cur == kEmpty) cur = atomicCAS(&tkeys[h], kEmpty, key);
        if (cur == kEmpty || cur == key) {
            if (added) *added = cur == kEmpty;
            return true;
        }
        h = (h + 1) & (uint64_t)(cap - 1);
    }
    return false;
}

// Sets the bit of every level-0 cell whose closure holds the finest-grid
// point f (up to 8 cells for a point on cell corners).
__device__ __forceinline__ void mark_cells(uint32_t *__restrict__ bits, const LatticeGeom &g,
                                           const int64_t f[3]) {
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t c = f[a] >> kMaxLevels, last = g.cells[a] - 1;
        const bool on_face = (f[a] & ((1 << kMaxLevels) - 1)) == 0;
        hi[a] = c < last ? c : last;
        lo[a] = on_face && c > 0 ? c - 1 : c;
        if (lo[a] > last) lo[a] = last;
    }
    for (int64_t z = lo[2]; z <= hi[2]; ++z)
        for (int64_t y = lo[1]; y <= hi[1]; ++y)
            for (int64_t x = lo[0]; x <= hi[0]; ++x) {
                const int64_t cell = (z * g.cells[1] + y) * g.cells[0] + x;
                atomicOr(&bits[cell >> 5], 1u << (cell & 31));
            }
}

// Inserts the vertices of entries [first, first + count) of level l (leaves
// or not: an inner entry's vertices are those of its corner children).  Keys
// that were not in the set are counted in *n_new and, when `fresh` is given,
// also put in that second set (the vertices new in this closure round), with
// the bits of the level-0 cells they touch set in `cells_new`.
__global__ void k_insert_range(LevelPtrs L, LatticeGeom g, int l, int64_t first, int64_t count,
                               unsigned long long *__restrict__ set, int64_t cap,
                               unsigned long long *__restrict__ fresh, int64_t fcap,
                               uint32_t *__restrict__ cells_new,
                               unsigned long long *__restrict__ n_new,
                               unsigned long long *__restrict__ overflow) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool added = false;
    if (jj < 4 * count) {
        int64_t F[4][3];
        leaf_fine_vertices(L, g, l, first + (jj >> 2), F);
        const uint64_t key = fine_key(F[jj & 3]);
        if (set_insert(set, cap, key, &added)) {
            if (added && fresh) {
                if (set_insert(fresh, fcap, key, nullptr))
                    mark_cells(cells_new, g, F[jj & 3]);
                else
                    atomicAdd(overflow, 1ull);
            }
        } else {
            atomicAdd(overflow, 1ull);
        }
    }
    // one counter update per block
    __shared__ unsigned int block_new;
    if (threadIdx.x == 0) block_new = 0;
    __syncthreads();
    const unsigned long long mask = __ballot(added);
    if ((threadIdx.x & 63) == 0 && mask) atomicAdd(&block_new, (unsigned int)__popcll(mask));
    __syncthreads();
    if (threadIdx.x == 0 && block_new) atomicAdd(n_new, (unsigned long long)block_new);
}

constexpr int kEdgeA[6] = {0, 0, 0, 1, 1, 2};
constexpr int kEdgeB[6] = {1, 2, 3, 2, 3, 3};

__device__ __forceinline__ bool allowed_pattern(unsigned bits) {
    const int n = __popc(bits);
    if (n <= 1) return true;
    if (n > 3) return false;
    unsigned verts = 0;
    for (int e = 0; e < 6; ++e)
        if (bits >> e & 1u) verts |= (1u << kEdgeA[e]) | (1u << kEdgeB[e]);
    return __popc(verts) == 3;   // two edges sharing a vertex, or the edges of one face
}

// Hanging-edge bits (0-5) and the quarter-point flag (bit 6) of a level-l
// leaf against a vertex set.
__device__ __forceinline__ unsigned leaf_hits(const int64_t F[4][3], int l,
                                              const unsigned long long *set, int64_t cap) {
    unsigned bits = 0;
    for (int e = 0; e < 6; ++e) {
        const int a = kEdgeA[e], b = kEdgeB[e];
        if (l < kMaxLevels) {
            int64_t m[3];
            for (int x = 0; x < 3; ++x) m[x] = (F[a][x] + F[b][x]) >> 1;
            if (set_find(set, cap, fine_key(m))) bits |= 1u << e;
        }
        if (l + 2 <= kMaxLevels && !(bits & kDeep)) {
            int64_t q1[3], q2[3];
            for (int x = 0; x < 3; ++x) {
                q1[x] = (3 * F[a][x] + F[b][x]) >> 2;
                q2[x] = (F[a][x] + 3 * F[b][x]) >> 2;
            }
            if (set_find(set, cap, fine_key(q1)) || set_find(set, cap, fine_key(q2))) bits |= kDeep;
        }
    }
    return bits;
}

__device__ __forceinline__ uint8_t with_red(unsigned f) {
    return (uint8_t)(((f & kDeep) || !allowed_pattern(f & 63u)) ? f | kRed : f);
}

// Full pattern of entries [first, first + count) of level l against the
// vertex set: flag = hanging bits | deep | red for a leaf, 0 for an inner
// entry.
__global__ void k_pattern_full(LevelPtrs L, LatticeGeom g, int l, int64_t first, int64_t count,
                               const unsigned long long *__restrict__ set, int64_t cap) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const int64_t i = first + j;
    if (L.child[l][i] >= 0) {
        L.flag[l][i] = 0;
        return;
    }
    int64_t F[4][3];
    leaf_fine_vertices(L, g, l, i, F);
    L.flag[l][i] = with_red(leaf_hits(F, l, set, cap));
}

// Update of entries [0, count) of level l after a closure round: the vertex
// set only grows, so a leaf's new pattern is its old one plus what the
// vertices added in this round (the `fresh` set) hit.  Entries split in the
// round are inner now and lose their flag.  Every point a leaf tests lies in
// the closure of its level-0 cell, so a leaf whose cell got no new vertex
// keeps its pattern without probing the set.
__global__ void k_pattern_fresh(LevelPtrs L, LatticeGeom g, int l, int64_t count,
                                const unsigned long long *__restrict__ fresh, int64_t fcap,
                                const uint32_t *__restrict__ cells_new) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint8_t old = L.flag[l][i];
    if (L.child[l][i] >= 0) {
        if (old) L.flag[l][i] = 0;
        return;
    }
    int64_t cell;
    if (l == 0) {
        cell = i / 6;
    } else {
        int lk, q;
        int64_t c[3];
        split_key(L.key[l][i], lk, q, c);
        cell = ((c[2] >> l) * g.cells[1] + (c[1] >> l)) * g.cells[0] + (c[0] >> l);
    }
    if (!((cells_new[cell >> 5] >> (cell & 31)) & 1u)) return;
    int64_t F[4][3];
    leaf_fine_vertices(L, g, l, i, F);
    const unsigned f = old | leaf_hits(F, l, fresh, fcap);
    if (f != old) L.flag[l][i] = with_red(f);
}

// Tetrahedra per listed leaf: one plus its number of hanging edges; hist[k]
// counts the leaves cut into k + 1 pieces (one atomic per block and bin).
__global__ void k_tet_counts(LevelPtrs L, int l, const int32_t *__restrict__ list, int64_t count,
                             int32_t *__restrict__ counts, unsigned long long *__restrict__ hist) {
    __shared__ unsigned int bins[4];
    if (threadIdx.x < 4) bins[threadIdx.x] = 0;
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) {
        const int c = 1 + __popc((unsigned)L.flag[l][list[j]] & 63u);
        counts[j] = c;
        atomicAdd(&bins[(c < 4 ? c : 4) - 1], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 4 && bins[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)bins[threadIdx.x]);
}

__device__ __forceinline__ void put_tet(int64_t *__restrict__ out, int64_t slot, const int64_t a[3],
                                        const int64_t b[3], const int64_t c[3], const int64_t d[3]) {
    // positive orientation: det(b - a, c - a, d - a) > 0, else swap a and b
    const int64_t u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const int64_t v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const int64_t w[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
    const int64_t det = u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                        u[2] * (v[0] * w[1] - v[1] * w[0]);
    int64_t *o = out + 4 * slot;
    o[0] = (int64_t)fine_key(det > 0 ? a : b);
    o[1] = (int64_t)fine_key(det > 0 ? b : a);
    o[2] = (int64_t)fine_key(c);
    o[3] = (int64_t)fine_key(d);
}

// The tetrahedra of every listed leaf at offsets[j] (first output slot).
__global__ void k_emit(LevelPtrs L, LatticeGeom g, int l, const int32_t *__restrict__ list,
                       int64_t count,
                       const int64_t *__restrict__ offsets, int64_t *__restrict__ tets,
                       int32_t *__restrict__ labels) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const int64_t i = list[j];
    int64_t F[4][3];
    leaf_fine_vertices(L, g, l, i, F);
    const unsigned b = L.flag[l][i] & 63u;
    const int n = __popc(b);
    const int64_t o = offsets[j];
    const int32_t lab = L.label[l][i];
    for (int t = 0; t <= n; ++t) labels[o + t] = lab;
    if (n == 0) {
        put_tet(tets, o, F[0], F[1], F[2], F[3]);
        return;
    }
    int ed[3], k = 0;
    for (int e = 0; e < 6; ++e)
        if (b >> e & 1u) ed[k++] = e;
    if (n == 1) {
        const int x = kEdgeA[ed[0]], y = kEdgeB[ed[0]];
        int r[2], m = 0;
        for (int v = 0; v < 4; ++v)
            if (v != x && v != y) r[m++] = v;
        int64_t mid[3];
        for (int a = 0; a < 3; ++a) mid[a] = (F[x][a] + F[y][a]) >> 1;
        put_tet(tets, o, F[x], mid, F[r[0]], F[r[1]]);
        put_tet(tets, o + 1, mid, F[y], F[r[0]], F[r[1]]);
        return;
    }
    if (n == 2) {
        const int e0a = kEdgeA[ed[0]], e0b = kEdgeB[ed[0]];
        const int e1a = kEdgeA[ed[1]], e1b = kEdgeB[ed[1]];
        const int a = (e0a == e1a || e0a == e1b) ? e0a : e0b;   // the shared vertex
        const int bv = e0a + e0b - a, cv = e1a + e1b - a;
        const int d = 6 - a - bv - cv;
        int64_t m1[3], m2[3];
        for (int x = 0; x < 3; ++x) {
            m1[x] = (F[a][x] + F[bv][x]) >> 1;
            m2[x] = (F[a][x] + F[cv][x]) >> 1;
        }
        put_tet(tets, o, F[a], m1, m2, F[d]);
        // the quadrilateral (m1, b, c, m2) is cut along the diagonal through
        // its smallest node key, a property of the face alone
        const uint64_t km1 = fine_key(m1), kb = fine_key(F[bv]), kc = fine_key(F[cv]),
                       km2 = fine_key(m2);
        const uint64_t low = min(min(km1, kb), min(kc, km2));
        if (low == km1 || low == kc) {
            put_tet(tets, o + 1, m1, F[bv], F[cv], F[d]);
            put_tet(tets, o + 2, m1, F[cv], m2, F[d]);
        } else {
            put_tet(tets, o + 1, m1, F[bv], m2, F[d]);
            put_tet(tets, o + 2, F[bv], F[cv], m2, F[d]);
        }
        return;
    }
    // three edges of one face (a < b < c), apex d
    unsigned vm = 0;
    for (int q = 0; q < 3; ++q) vm |= (1u << kEdgeA[ed[q]]) | (1u << kEdgeB[ed[q]]);
    int fv[3], m = 0, d = 0;
    for (int v = 0; v < 4; ++v) {
        if (vm >> v & 1u) fv[m++] = v;
        else d = v;
    }
    int64_t mab[3], mbc[3], mca[3];
    for (int x = 0; x < 3; ++x) {
        mab[x] = (F[fv[0]][x] + F[fv[1]][x]) >> 1;
        mbc[x] = (F[fv[1]][x] + F[fv[2]][x]) >> 1;
        mca[x] = (F[fv[2]][x] + F[fv[0]][x]) >> 1;
    }
    put_tet(tets, o, F[fv[0]], mab, mca, F[d]);
    put_tet(tets, o + 1, mab, F[fv[1]], mbc, F[d]);
    put_tet(tets, o + 2, mca, mbc, F[fv[2]], F[d]);
    put_tet(tets, o + 3, mab, mbc, mca, F[d]);
}

__global__ void k_head_flags(const int64_t *__restrict__ sorted, int64_t n, int32_t *__restrict__ head) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    head[i] = (i == 0 || sorted[i] != sorted[i - 1]) ? 1 : 0;
}

__global__ void k_unique_scatter(const int64_t *__restrict__ sorted, const int32_t *__restrict__ head,
                                 const int64_t *__restrict__ pos, int64_t n,
                                 int64_t *__restrict__ nodes) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (head[i]) nodes[pos[i]] = sorted[i];
}

__global__ void k_node_ids(const int64_t *__restrict__ tet_keys, int64_t n,
                           const int64_t *__restrict__ nodes, int64_t n_nodes,
                           int32_t *__restrict__ ids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t key = tet_keys[i];
    int64_t lo = 0, hi = n_nodes - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (nodes[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    ids[i] = (int32_t)lo;
}

__global__ void k_node_xyz(LatticeGeom g, const int64_t *__restrict__ nodes, int64_t n,
                           float *__restrict__ xyz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = (uint64_t)nodes[i];
    const int64_t f[3] = {(int64_t)((k >> 42) & 0x1fffffu), (int64_t)((k >> 21) & 0x1fffffu),
                          (int64_t)(k & 0x1fffffu)};
    const double hf = ldexp(g.h, -kMaxLevels);
    for (int a = 0; a < 3; ++a)
        xyz[3 * i + a] = lattice_coord(g.origin[a], hf, (double)f[a]);
}

inline unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_insert_range(const LevelPtrs &L, const LatticeGeom &g, int l, int64_t first,
                               int64_t count, unsigned long long *set, int64_t cap,
                               unsigned long long *fresh, int64_t fcap, uint32_t *cells_new,
                               unsigned long long *n_new, unsigned long long *overflow,
                               hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_insert_range<<<grid_of(4 * count), 256, 0, s>>>(L, g, l, first, count, set, cap, fresh, fcap,
                                                      cells_new, n_new, overflow);
    return hipGetLastError();
}

hipError_t launch_pattern_full(const LevelPtrs &L, const LatticeGeom &g, int l, int64_t first,
                               int64_t count, const unsigned long long *set, int64_t cap,
                               hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_pattern_full<<<grid_of(count), 256, 0, s>>>(L, g, l, first, count, set, cap);
    return hipGetLastError();
}

hipError_t launch_pattern_fresh(const LevelPtrs &L, const LatticeGeom &g, int l, int64_t count,
                                const unsigned long long *fresh, int64_t fcap,
                                const uint32_t *cells_new, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_pattern_fresh<<<grid_of(count), 256, 0, s>>>(L, g, l, count, fresh, fcap, cells_new);
    return hipGetLastError();
}

hipError_t launch_tet_counts(const LevelPtrs &L, int l, const int32_t *list, int64_t count,
                             int32_t *counts, unsigned long long *hist, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_tet_counts<<<grid_of(count), 256, 0, s>>>(L, l, list, count, counts, hist);
    return hipGetLastError();
}

hipError_t exclusive_sum_i32(const int32_t *in, int64_t *out, int64_t n, void *tmp,
                             size_t *tmp_bytes, hipStream_t s) {
    return rocprim::exclusive_scan(tmp, *tmp_bytes, in, out, (int64_t)0, (size_t)n,
                                   rocprim::plus<int64_t>(), s);
}

hipError_t launch_emit(const LevelPtrs &L, const LatticeGeom &g, int l, const int32_t *list,
                       int64_t count, const int64_t *offsets, int64_t *tets, int32_t *labels,
                       hipStream_t s) {
    if (count <= 0) return hipSuccess;
    k_emit<<<grid_of(count), 256, 0, s>>>(L, g, l, list, count, offsets, tets, labels);
    return hipGetLastError();
}

hipError_t sort_keys_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, size_t *tmp_bytes,
                         hipStream_t s) {
    return rocprim::radix_sort_keys(tmp, *tmp_bytes, in, out, (size_t)n, 0u, 64u, s);
}

hipError_t launch_unique(const int64_t *sorted, int64_t n, int32_t *head, int64_t *pos,
                         int64_t *nodes, void *tmp, size_t *tmp_bytes, hipStream_t s) {
    if (!tmp)
        return rocprim::exclusive_scan(tmp, *tmp_bytes, head, pos, (int64_t)0, (size_t)n,
                                       rocprim::plus<int64_t>(), s);
    if (n <= 0) return hipSuccess;
    k_head_flags<<<grid_of(n), 256, 0, s>>>(sorted, n, head);
    hipError_t e = rocprim::exclusive_scan(tmp, *tmp_bytes, head, pos, (int64_t)0, (size_t)n,
                                           rocprim::plus<int64_t>(), s);
    if (e != hipSuccess) return e;
    k_unique_scatter<<<grid_of(n), 256, 0, s>>>(sorted, head, pos, n, nodes);
    return hipGetLastError();
}

hipError_t launch_node_ids(const int64_t *tet_keys, int64_t n, const int64_t *nodes, int64_t n_nodes,
                           int32_t *ids, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_node_ids<<<grid_of(n), 256, 0, s>>>(tet_keys, n, nodes, n_nodes, ids);
    return hipGetLastError();
}

hipError_t launch_node_xyz(const LatticeGeom &g, const int64_t *nodes, int64_t n, float *xyz,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_node_xyz<<<grid_of(n), 256, 0, s>>>(g, nodes, n, xyz);
    return hipGetLastError();
}

}  // namespace sal
