// Recheck of the (point, surface) pairs the float32 pass could not certify,
// and the final label of those points: every triangle term is recomputed,
// in float32 where float32 certifies it and in double (with the exact-sign
// guard) where it does not (recheck_mixed.h).
//
// One workgroup per flagged point (grid-stride over the device-side count, so
// no host round trip sizes the launch).  For each flagged surface the 256
// threads take the surface's strips round-robin, each sums its strips in
// double along the strip, and an LDS tree reduces the 256 partial sums in a
// fixed order: the result does not depend on timing.
#include <hip/hip_runtime.h>

#include "pairloop_f32.h"
#include "recheck_mixed.h"
#include "sal_internal.h"

namespace sal {
namespace {

constexpr double kInv2Pi = 0.15915494309189533577;
constexpr int kThreads = 256;

// ---------------------------------------------------------- pair-major form
// Flagged (point, surface) pairs are grouped by surface (a counting sort),
// each group padded to a multiple of 64; a wavefront takes 64 pairs of one
// surface and walks its strips with scalar record loads, as the pair loop
// does, keeping the float32 terms float32 certifies and recomputing the
// others in double per lane.  Every pair's sum is a sequential per-lane sum
// with per-lane path choices, so the result does not depend on which pairs
// share a wavefront (the order of the groups is not deterministic).

using f32::lane_id;
using f32::CRec32;
using f32::CSurf;

__global__ void k_rc_clear(RecheckSeg *seg) {
    const int t = threadIdx.x;
    if (t < kMaxSurfaces) {
        seg->count[t] = 0ull;
        seg->cursor[t] = 0ull;
    }
    if (t == 0) {
        seg->total = 0ull;
        seg->overflow = 0ull;
    }
}

__device__ __forceinline__ int64_t flagged_count(const RecheckArgs &a) {
    const int64_t c = (int64_t)a.counters[kCntFlagged];
    return c < a.n ? c : a.n;
}

// Certified bits of every flagged point; pairs per surface.
__global__ void k_rc_count(RecheckArgs a) {
    const int64_t count = flagged_count(a);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const FlagEntry e = a.flag_list[i];
        a.res[i] = e.enc & ~e.flg;
        uint64_t f = e.flg;
        while (f) {
            const int k = __builtin_ctzll(f);
            f &= f - 1;
            atomicAdd(&a.seg->count[k], 1ull);
        }
    }
}

// One thread per surface: padded group offsets, the padding entries, and the
// capacity check.
__global__ void k_rc_scan(RecheckArgs a) {
    __shared__ unsigned long long padded[kMaxSurfaces];
    const int k = threadIdx.x;
    const unsigned long long c = k < a.n_surf ? a.seg->count[k] : 0ull;
    if (k < kMaxSurfaces) padded[k] = (c + 63ull) & ~63ull;
    __syncthreads();
    if (k >= kMaxSurfaces) return;
    unsigned long long off = 0, total = 0;
    for (int j = 0; j < kMaxSurfaces; ++j) {
        if (j < k) off += padded[j];
        total += padded[j];
    }
    a.seg->off[k] = off;
    if (k == 0) {
        // Few pairs: cut each surface into strip ranges so that chunks x
        // splits wavefronts fill the GPU; the partial sums need splits slots
        // per pair, so splits <= capacity / pairs.
        const unsigned long long chunks = total / 64ull;
        unsigned long long sp = 1;
        if (chunks > 0) {
            sp = ((unsigned long long)a.target_waves + chunks - 1) / chunks;
            if (sp > 16) sp = 16;
            const unsigned long long room = (unsigned long long)a.pair_cap / total;
            if (sp > room) sp = room;
            if (sp < 1) sp = 1;
        }
        a.seg->total = total;
        a.seg->splits = sp;
        a.seg->overflow = total > (unsigned long long)a.pair_cap ? 1ull : 0ull;
    }
    if (total > (unsigned long long)a.pair_cap) return;
    for (unsigned long long q = off + c; q < off + padded[k]; ++q) {
        RecheckPair pr;
        pr.entry = -1;
        pr.surf = k;
        a.pairs[q] = pr;
    }
}

__global__ void k_rc_scatter(RecheckArgs a) {
    if (a.seg->overflow) return;
    const int64_t count = flagged_count(a);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        uint64_t f = a.flag_list[i].flg;
        while (f) {
            const int k = __builtin_ctzll(f);
            f &= f - 1;
            const unsigned long long pos = a.seg->off[k] + atomicAdd(&a.seg->cursor[k], 1ull);
            RecheckPair pr;
            pr.entry = (int32_t)i;
            pr.surf = k;
            a.pairs[pos] = pr;
        }
    }
}

constexpr int kPairWaves = 4;   // wavefronts per workgroup of k_rc_pairs

__global__ __launch_bounds__(64 * kPairWaves) void k_rc_pairs(RecheckArgs a) {
    if (a.seg->overflow) return;
    const int64_t splits = (int64_t)a.seg->splits;
    const int64_t items = (int64_t)(a.seg->total / 64ull) * splits;
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * kPairWaves +
                         __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int64_t n_waves = (int64_t)gridDim.x * kPairWaves;
    const CRec32 *rec = (const CRec32 *)a.rec32;
    const CSurf *surf = (const CSurf *)a.surf;
    const float kap = a.kappa;
    const float branch_cut = mixed::kPiF - 0.25f * kap;
    unsigned n_exact = 0, n_f64 = 0;
    for (int64_t it = wave; it < items; it += n_waves) {
        const int64_t c = it / splits;     // 64-pair chunk
        const int64_t j = it - c * splits; // strip range of the surface
        const RecheckPair pr = a.pairs[c * 64 + lane];
        const int k = __builtin_amdgcn_readfirstlane(pr.surf);
        const bool valid = pr.entry >= 0;
        float px = 0.0f, py = 0.0f, pz = 0.0f;
        if (valid) {
            const int64_t idx = a.flag_list[pr.entry].idx;
            px = a.x[idx];
            py = a.y[idx];
            pz = a.z[idx];
        }
        double S = 0.0;
        int on = 0;
        const int64_t sb = surf[k].strip_begin, n_strips = surf[k].strip_end - sb;
        const int64_t s_lo = sb + n_strips * j / splits, s_hi = sb + n_strips * (j + 1) / splits;
        const int64_t rec_end = s_hi < surf[k].strip_end ? a.strip_off[s_hi] : surf[k].rec_end;
        for (int64_t r = s_lo < s_hi ? a.strip_off[s_lo] : rec_end; r < rec_end;) {
            const CRec32 *h = rec + r;
            const int m = __float_as_int(h->v[6]);
            float x0 = h->v[0], x1 = h->v[1], x2 = h->v[2];   // raw older vertex
            float y0 = h->v[3], y1 = h->v[4], y2 = h->v[5];   // raw newer vertex
            float ax = x0 - px, ay = x1 - py, az = x2 - pz;
            float bx = y0 - px, by = y1 - py, bz = y2 - pz;
            float ar = __builtin_amdgcn_sqrtf(fmaf(ax, ax, fmaf(ay, ay, az * az)));
            float br = __builtin_amdgcn_sqrtf(fmaf(bx, bx, fmaf(by, by, bz * bz)));
            float e01 = fmaf(ax, bx, fmaf(ay, by, az * bz));
            float rr01 = ar * br;
            float accf = 0.0f, accn = 0.0f;
            double accd = 0.0;
            for (int t = 1; t <= m; ++t) {
                const CRec32 *q = rec + r + t;
                const float z0 = q->v[0], z1 = q->v[1], z2 = q->v[2];
                const float q3 = q->v[3], q4 = q->v[4], q5 = q->v[5], q6 = q->v[6], q7 = q->v[7];
                const float cx = z0 - px, cy = z1 - py, cz = z2 - pz;
                const float cr = __builtin_amdgcn_sqrtf(fmaf(cx, cx, fmaf(cy, cy, cz * cz)));
                const float e02 = fmaf(ax, cx, fmaf(ay, cy, az * cz));
                const float e12 = fmaf(bx, cx, fmaf(by, cy, bz * cz));
                const float nn = fmaf(cx, q3, fmaf(cy, q4, cz * q5));   // 32 N
                const float mm = rr01 * cr;
                const float dd = fmaf(e12, ar, fmaf(e02, br, fmaf(e01, cr, mm)));
                const float lim = fmaf(q7, cr, fmaf(kap, mm, fabsf(nn)));
                // Per-lane choice (not wave-uniform as in the pair loop): a pair's
                // terms must not depend on which pairs share its wavefront.
                if (__builtin_expect(dd > lim, 1)) {   // the common case as the fall-through path
                    const float u = nn * __builtin_amdgcn_rcpf(dd);
                    const float s2 = u * u;
                    accf = fmaf(u, fmaf(fmaf(mixed::kA2, s2, mixed::kA1), s2, mixed::kA0), accf);
                } else {
                    const float n1 = nn * (1.0f / kNScale);
                    const float ang = atan2f(n1, dd);
                    const float thr = fmaf(cr, kap * q6, kap * mm);
                    const bool ill = fmaxf(fabsf(n1), fabsf(dd)) <= thr;
                    const bool cut = fabsf(ang) > branch_cut;
                    if (valid && (ill || cut)) {
                        const mixed::F64Term d = mixed::f64_triangle(
                            x0, x1, x2, y0, y1, y2, a.rec64[r + t].v, px, py, pz);
                        accd += d.half;
                        on |= d.on;
                        n_exact += d.exact;
                        n_f64 += 1;
                    } else {
                        accn += ang;
                    }
                }
                ax = bx; ay = by; az = bz; ar = br;
                bx = cx; by = cy; bz = cz; br = cr;
                e01 = e12;
                rr01 = ar * cr;
                x0 = y0; x1 = y1; x2 = y2;
                y0 = z0; y1 = z1; y2 = z2;
            }
            S += accd + (double)accf + (double)accn;
            r += m + 1;
        }
        if (valid) {
            RecheckOut o;
            o.sum = S;
            o.on = on;
            o.pad = 0u;
            a.pair_out[(c * 64 + lane) * splits + j] = o;
        }
    }
    if (n_exact) atomicAdd(&a.counters[kCntExact], (unsigned long long)n_exact);
    if (n_f64) atomicAdd(&a.counters[kCntRecheckF64], (unsigned long long)n_f64);
}

// Per pair: the decision of section 2.1.3 for its surface, into the point's
// enclosed bits (and the winding output).
__global__ void k_rc_pair_final(RecheckArgs a) {
    if (a.seg->overflow) return;
    const int64_t total = (int64_t)a.seg->total;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
        const RecheckPair pr = a.pairs[q];
        if (pr.entry < 0) continue;
        const int64_t splits = (int64_t)a.seg->splits;
        double sum = 0.0;
        int on = 0;
        for (int64_t j = 0; j < splits; ++j) {   // the strip ranges in order
            const RecheckOut o = a.pair_out[q * splits + j];
            sum += o.sum;
            on |= o.on;
        }
        const double w = sum * kInv2Pi;
        if (on || w >= a.threshold) atomicOr(&a.res[pr.entry], 1ull << pr.surf);
        if (a.winding) {
            const int64_t idx = a.flag_list[pr.entry].idx;
            const int64_t off = (int64_t)pr.surf * a.n + idx;
            if (a.winding_type == SAL_WINDING_F64) ((double *)a.winding)[off] = w;
            else ((float *)a.winding)[off] = (float)w;
        }
    }
}

// Per flagged point: the label from its enclosed bits (section 2.1: the
// enclosing surface latest in the list wins; 0 = box).
__global__ void k_rc_entry_final(RecheckArgs a) {
    if (a.seg->overflow) return;
    const int64_t count = flagged_count(a);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long pairs = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const FlagEntry e = a.flag_list[i];
        const unsigned long long enc = a.res[i];
        a.labels[e.idx] = enc ? a.surf[63 - __builtin_clzll(enc)].label : 0;
        if (a.masks) a.masks[e.idx] = enc;
        pairs += (unsigned long long)__popcll(e.flg);
    }
    if (pairs) atomicAdd(&a.counters[kCntRecheck], pairs);
}

// ---------------------------------------------------------- per-point form
// Runs only when the pairs did not fit the pair-major scratch.
__global__ __launch_bounds__(kThreads) void k_recheck_f64(RecheckArgs a) {
    __shared__ double red[kThreads];
    const int tid = threadIdx.x;
    if (!a.seg->overflow) return;
    int64_t count = (int64_t)a.counters[kCntFlagged];
    if (count > a.n) count = a.n;
    unsigned n_exact = 0, n_f64 = 0;
    const float branch_cut = mixed::kPiF - 0.25f * a.kappa;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const FlagEntry e = a.flag_list[i];
        const float praw[3] = {a.x[e.idx], a.y[e.idx], a.z[e.idx]};
        const double p[3] = {praw[0], praw[1], praw[2]};
        uint64_t enc = e.enc;
        uint64_t f = e.flg;
        while (f) {
            const int k = __builtin_ctzll(f);
            f &= f - 1;
            const SurfaceDev sd = a.surf[k];
            double part = 0.0;
            int on = 0;
            for (int64_t s = sd.strip_begin + tid; s < sd.strip_end; s += kThreads) {
                const int64_t r = a.strip_off[s];
                const int m = __float_as_int(a.rec32[r].v[6]);
                part += mixed::strip_sum(a.rec32, a.rec64, r, m, praw, p, a.kappa, branch_cut,
                                         &on, &n_exact, &n_f64);
            }
            red[tid] = part;
            on = __syncthreads_or(on);
            for (int w = kThreads / 2; w > 0; w >>= 1) {
                if (tid < w) red[tid] += red[tid + w];
                __syncthreads();
            }
            const double wk = red[0] * kInv2Pi;
            __syncthreads();
            // Section 2.1.3: enclosed when s >= T (or when p lies on the surface).
            if (on || wk >= a.threshold) enc |= 1ull << k;
            else enc &= ~(1ull << k);
            if (tid == 0 && a.winding) {
                const int64_t o = (int64_t)k * a.n + e.idx;
                if (a.winding_type == SAL_WINDING_F64) ((double *)a.winding)[o] = wk;
                else ((float *)a.winding)[o] = (float)wk;
            }
        }
        if (tid == 0) {
            // Section 2.1: the enclosing surface latest in the list wins; 0 = box.
            const int32_t lab = enc ? a.surf[63 - __builtin_clzll(enc)].label : 0;
            a.labels[e.idx] = lab;
            if (a.masks) a.masks[e.idx] = enc;
            atomicAdd(&a.counters[kCntRecheck], (unsigned long long)__popcll(e.flg));
        }
    }
    if (n_exact) atomicAdd(&a.counters[kCntExact], (unsigned long long)n_exact);
    if (n_f64) atomicAdd(&a.counters[kCntRecheckF64], (unsigned long long)n_f64);
}

}  // namespace

hipError_t launch_recheck_f64(const RecheckArgs &a, int grid_blocks, hipStream_t s) {
    if (a.n <= 0 || grid_blocks <= 0) return hipSuccess;
    k_rc_clear<<<1, kMaxSurfaces, 0, s>>>(a.seg);
    k_rc_count<<<dim3(grid_blocks), 256, 0, s>>>(a);
    k_rc_scan<<<1, kMaxSurfaces, 0, s>>>(a);
    k_rc_scatter<<<dim3(grid_blocks), 256, 0, s>>>(a);
    k_rc_pairs<<<dim3(grid_blocks), 64 * kPairWaves, 0, s>>>(a);
    k_rc_pair_final<<<dim3(grid_blocks), 256, 0, s>>>(a);
    k_rc_entry_final<<<dim3(grid_blocks), 256, 0, s>>>(a);
    k_recheck_f64<<<dim3(grid_blocks), dim3(kThreads), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace sal
