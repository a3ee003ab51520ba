// Inflation of the compartment boundaries (paper section 2.2.2): interface
// nodes slide along the incident edge whose crossing with a surface triangle
// is nearest, by zeta times that distance.
//
// Triangles are binned on the level-0 lattice (one bin per cell); an edge
// tests only the triangles of the bins its bounding box covers.  Each
// crossing is the Moller-Trumbore construction in double with the products
// and sums rounded one by one, on the triangle's vertices in lexicographic
// order, so the parameter depends on the geometry alone.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_scan.hpp>

#include "post_internal.h"

namespace sal {
namespace {

constexpr uint32_t kSurfBit = 1u << 31;
constexpr int kInflateGroup = 8;   // lanes per node

inline unsigned grid_of(int64_t n) { return (unsigned)((n + kSmoothThreads - 1) / kSmoothThreads); }

__device__ __forceinline__ bool lex_less(const double *a, const double *b) {
    if (a[0] != b[0]) return a[0] < b[0];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[2] < b[2];
}

// Triangles of strip s: (v_k, v_k+1, v_k+2) with v_0, v_1 in the head record
// and v_k+2 the vertex of the k-th record after it; stored with sorted
// vertices, in float32 (the surface vertices are float32 values, so this
// loses nothing and halves the bytes each test reads).
__global__ void k_strip_triangles(const Rec64 *__restrict__ rec, const int64_t *__restrict__ strip_off,
                                  const int64_t *__restrict__ tri_base, int64_t n_strips,
                                  float *__restrict__ tri) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_strips) return;
    const int64_t h = strip_off[s];
    int64_t m;
    memcpy(&m, &rec[h].v[6], 8);
    double w[3][3];
    for (int c = 0; c < 3; ++c) {
        w[0][c] = rec[h].v[c];
        w[1][c] = rec[h].v[3 + c];
    }
    for (int64_t k = 0; k < m; ++k) {
        for (int c = 0; c < 3; ++c) w[2][c] = rec[h + 1 + k].v[c];
        const double *p[3] = {w[0], w[1], w[2]};
        // sort three
        if (lex_less(p[1], p[0])) { const double *x = p[0]; p[0] = p[1]; p[1] = x; }
        if (lex_less(p[2], p[1])) { const double *x = p[1]; p[1] = p[2]; p[2] = x; }
        if (lex_less(p[1], p[0])) { const double *x = p[0]; p[0] = p[1]; p[1] = x; }
        float *o = tri + 9 * (tri_base[s] + k);
        for (int v = 0; v < 3; ++v)
            for (int c = 0; c < 3; ++c) o[3 * v + c] = (float)p[v][c];
        for (int c = 0; c < 3; ++c) {
            w[0][c] = w[1][c];
            w[1][c] = w[2][c];
        }
    }
}

__device__ __forceinline__ int bin_of(double x, double o, double h, int n) {
    const double f = floor((x - o) / h);
    return f < 0.0 ? 0 : (f >= (double)n ? n - 1 : (int)f);
}

struct BinBox {
    int lo[3], hi[3];
};

__device__ __forceinline__ BinBox box_bins(const double lo[3], const double hi[3], const LatticeGeom &g) {
    BinBox b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = bin_of(lo[a], g.origin[a], g.h, g.cells[a]);
        b.hi[a] = bin_of(hi[a], g.origin[a], g.h, g.cells[a]);
    }
    return b;
}

__device__ __forceinline__ int64_t bin_index(int x, int y, int z, const LatticeGeom &g) {
    return ((int64_t)z * g.cells[1] + y) * g.cells[0] + x;
}

// pass 0: count triangles per bin; pass 1: place them (cursor per bin).
__global__ void k_bin_triangles(const float *__restrict__ tri, int64_t n_tri, LatticeGeom g, int pass,
                                int32_t *__restrict__ count, const int64_t *__restrict__ start,
                                int32_t *__restrict__ items) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    const float *v = tri + 9 * t;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = fmin(fmin((double)v[a], (double)v[3 + a]), (double)v[6 + a]);
        hi[a] = fmax(fmax((double)v[a], (double)v[3 + a]), (double)v[6 + a]);
    }
    const BinBox b = box_bins(lo, hi, g);
    for (int z = b.lo[2]; z <= b.hi[2]; ++z)
        for (int y = b.lo[1]; y <= b.hi[1]; ++y)
            for (int x = b.lo[0]; x <= b.hi[0]; ++x) {
                const int64_t k = bin_index(x, y, z, g);
                const int32_t slot = atomicAdd(&count[k], 1);
                if (pass == 1) items[start[k] + slot] = (int32_t)t;
            }
}

// The triangles of each bin copied in bin order (9 floats per entry), so the
// tests of a bin read their triangles at consecutive addresses instead of
// through the item list (one dependent load less per test).
__global__ void k_gather_binned(const float *__restrict__ tri, const int32_t *__restrict__ items,
                                int64_t n_items, float *__restrict__ binned) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (entry, coordinate)
    if (k >= 9 * n_items) return;
    const int64_t r = k / 9;
    binned[k] = tri[9 * (int64_t)items[r] + (k - 9 * r)];
}

// Segment p -> p + d against triangle tv (9 floats): t in [0, 1], or -1.
__device__ __forceinline__ double crossing(const double p[3], const double d[3], const float *tv) {
#pragma clang fp contract(off)
    double v[9];
    for (int k = 0; k < 9; ++k) v[k] = (double)tv[k];
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double h[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    const double a = (e1[0] * h[0] + e1[1] * h[1]) + e1[2] * h[2];
    if (a == 0.0) return -1.0;
    const double f = 1.0 / a;
    const double s[3] = {p[0] - v[0], p[1] - v[1], p[2] - v[2]};
    const double u = f * ((s[0] * h[0] + s[1] * h[1]) + s[2] * h[2]);
    if (!(u >= 0.0 && u <= 1.0)) return -1.0;
    const double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    const double w = f * ((d[0] * q[0] + d[1] * q[1]) + d[2] * q[2]);
    if (!(w >= 0.0 && u + w <= 1.0)) return -1.0;
    const double t = f * ((e2[0] * q[0] + e2[1] * q[1]) + e2[2] * q[2]);
    return (t >= 0.0 && t <= 1.0) ? t : -1.0;
}

// kInflateGroup lanes per interface node, each taking every
// kInflateGroup-th entry of the row; per entry the nearest crossing over the
// triangles of the covered bins; the group keeps the entry with the
// smallest (distance, neighbour key) and its first lane writes the moved
// node into `out` (which holds every position on entry).
// Five wavefronts per SIMD (96 VGPRs, 12 bytes spilled) instead of the four
// that 102 VGPRs allow: on c3 the call took 15.2 ms against 16.5 ms; six
// (84 bytes spilled) measured the same as five.
__global__ __launch_bounds__(kSmoothThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_inflate(
    const float4 *__restrict__ in, float4 *__restrict__ out, const uint64_t *__restrict__ seg,
    const uint32_t *__restrict__ cols, const int32_t *__restrict__ list, int64_t n,
    const int32_t *__restrict__ order, const int64_t *__restrict__ keys,
    const float *__restrict__ bin_tri, const int64_t *__restrict__ bin_start, LatticeGeom g,
    double zeta, double *__restrict__ partials) {
#pragma clang fp contract(off)
    constexpr int G = kInflateGroup;
    const int lane = (int)(threadIdx.x & (G - 1));
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    double best_d = INFINITY;
    int64_t best_key = INT64_MAX;
    int32_t best_j = -1;
    double tests = 0.0;
    int32_t i = 0;
    if (t < n) {
        i = list[t];
        const float4 xi = in[i];
        const double p[3] = {(double)xi.x, (double)xi.y, (double)xi.z};
        const uint64_t sg = seg[t];
        const int64_t beg = (int64_t)(sg >> 32), len = (int64_t)(sg & 0xffffffffu);
        for (int64_t q = lane; q < len; q += G) {
            const int32_t j = (int32_t)(cols[beg + q] & ~kSurfBit);
            const float4 xj = in[j];
            const double qj[3] = {(double)xj.x, (double)xj.y, (double)xj.z};
            const double d[3] = {qj[0] - p[0], qj[1] - p[1], qj[2] - p[2]};
            // bounding box of the segment, widened far beyond rounding so a
            // crossing on a bin face finds the triangles of both bins
            double lo[3], hi[3];
            const double pad = 1e-9 * g.h;
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(p[a], qj[a]) - pad;
                hi[a] = fmax(p[a], qj[a]) + pad;
            }
            const BinBox b = box_bins(lo, hi, g);
            double tmin = INFINITY;
            for (int z = b.lo[2]; z <= b.hi[2]; ++z)
                for (int y = b.lo[1]; y <= b.hi[1]; ++y)
                    for (int x = b.lo[0]; x <= b.hi[0]; ++x) {
                        const int64_t k = bin_index(x, y, z, g);
                        for (int64_t r = bin_start[k], e = bin_start[k + 1]; r < e; ++r) {
                            const double tt = crossing(p, d, bin_tri + 9 * r);
                            tests += 1.0;
                            if (tt >= 0.0 && tt < tmin) tmin = tt;
                        }
                    }
            if (tmin <= 1.0) {
                const double len2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                const double dist = tmin * sqrt(len2);
                const int64_t kj = keys[order[j]];
                if (dist < best_d || (dist == best_d && kj < best_key)) {
                    best_d = dist;
                    best_key = kj;
                    best_j = j;
                }
            }
        }
    }
    for (int off = G / 2; off > 0; off >>= 1) {
        const double od = __shfl_xor(best_d, off, G);
        const int64_t ok = __shfl_xor(best_key, off, G);
        const int32_t oj = __shfl_xor(best_j, off, G);
        if (od < best_d || (od == best_d && ok < best_key)) {
            best_d = od;
            best_key = ok;
            best_j = oj;
        }
    }
    double moved = 0.0;
    if (t < n && lane == 0 && best_j >= 0) {
        const float4 xi = in[i];
        const float4 xj = in[best_j];
        const double p[3] = {(double)xi.x, (double)xi.y, (double)xi.z};
        const double d[3] = {(double)xj.x - p[0], (double)xj.y - p[1], (double)xj.z - p[2]};
        const double len = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        float4 o;
        o.x = (float)(p[0] + zeta * best_d * (d[0] / len));
        o.y = (float)(p[1] + zeta * best_d * (d[1] / len));
        o.z = (float)(p[2] + zeta * best_d * (d[2] / len));
        o.w = 0.0f;
        out[i] = o;
        moved = 1.0;
    }
    // block sums of moved nodes and triangle tests
    __shared__ double red[2][kSmoothThreads];
    red[0][threadIdx.x] = moved;
    red[1][threadIdx.x] = tests;
    __syncthreads();
    for (int w = kSmoothThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0];
        partials[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(1024) void k_sum_pairs(const double *__restrict__ partials, int64_t nb,
                                                    double *__restrict__ out) {
    __shared__ double red[2][1024];
    double a = 0.0, b = 0.0;
    for (int64_t j = threadIdx.x; j < nb; j += 1024) {
        a += partials[2 * j];
        b += partials[2 * j + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

}  // namespace

int64_t inflate_blocks(int64_t n) { return (n * kInflateGroup + kSmoothThreads - 1) / kSmoothThreads; }

hipError_t launch_strip_triangles(const Rec64 *rec, const int64_t *strip_off, const int64_t *tri_base,
                                  int64_t n_strips, float *tri, hipStream_t s) {
    if (n_strips <= 0) return hipSuccess;
    k_strip_triangles<<<grid_of(n_strips), kSmoothThreads, 0, s>>>(rec, strip_off, tri_base, n_strips, tri);
    return hipGetLastError();
}

hipError_t launch_bin_triangles(const float *tri, int64_t n_tri, const LatticeGeom &g, int pass,
                                int32_t *count, const int64_t *start, int32_t *items, hipStream_t s) {
    if (n_tri <= 0) return hipSuccess;
    k_bin_triangles<<<grid_of(n_tri), kSmoothThreads, 0, s>>>(tri, n_tri, g, pass, count, start, items);
    return hipGetLastError();
}

hipError_t exclusive_sum_bins(const int32_t *count, int64_t *start, int64_t n, void *tmp, size_t *tmp_bytes,
                              hipStream_t s) {
    return rocprim::exclusive_scan(tmp, *tmp_bytes, count, start, (int64_t)0, (size_t)n,
                                   rocprim::plus<int64_t>(), s);
}

hipError_t launch_gather_binned(const float *tri, const int32_t *items, int64_t n_items, float *binned,
                                hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_gather_binned<<<grid_of(9 * n_items), kSmoothThreads, 0, s>>>(tri, items, n_items, binned);
    return hipGetLastError();
}

hipError_t launch_inflate(const float4 *in, float4 *out, const uint64_t *seg, const uint32_t *cols,
                          const int32_t *list, int64_t n, const int32_t *order, const int64_t *keys,
                          const float *bin_tri, const int64_t *bin_start, const LatticeGeom &g,
                          double zeta, double *partials, double *sums, hipStream_t s) {
    const int64_t nb = inflate_blocks(n);
    if (nb > 0)
        k_inflate<<<(unsigned)nb, kSmoothThreads, 0, s>>>(in, out, seg, cols, list, n, order, keys,
                                                          bin_tri, bin_start, g, zeta, partials);
    k_sum_pairs<<<1, 1024, 0, s>>>(partials, nb, sums);
    return hipGetLastError();
}

}  // namespace sal
