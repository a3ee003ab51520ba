// Pair loop: winding numbers of every point against every triangle of every
// surface, the label decision, and the flags that send a (point, surface)
// pair to the FP64 recheck.  gfx950 (CDNA4), wave64.
//
// Work layout: one lane owns P points (registers); every lane of a wavefront
// walks the same triangle strips, so each strip record is fetched once per
// wavefront with a scalar load and used as an SGPR operand by all 64 lanes.
// No LDS, no barriers: wavefronts are independent and the record stream
// (tens of MB at most) stays in L2 / MALL.  This is not a dense contraction
// (three coordinates per point, transcendental terms, sign-sensitive
// cancellation near the surface), so it runs on the VALU, not on MFMA.
#include <hip/hip_runtime.h>

#include "pairloop_f32.h"
#include "sal_internal.h"
#include "pairloop_f64.h"

namespace sal {
namespace {

using namespace f32;

// CULL selects the form that tests each surface's box and ball first (see
// below); without it the kernel has no trace of the test, so its register
// budget (and occupancy) stays that of the plain walk.
template <int P, bool CULL>
__global__ __launch_bounds__(512) void k_pairloop_f32(PairloopArgs a) {
    const int64_t blk = (int64_t)blockIdx.x * blockDim.x * P;
    const int64_t n = a.n_dev ? *a.n_dev : a.n;
    if (blk >= n) return;   // whole workgroup past the end (grid sized for a capacity)
    const CRec32 *rec = (const CRec32 *)a.rec32;
    const CSurf *surf = (const CSurf *)a.surf;
    float px[P], py[P], pz[P];
    int64_t idx[P];
    bool valid[P], good[P];
    uint64_t good_mask[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        idx[j] = blk + (int64_t)j * blockDim.x + threadIdx.x;
        valid[j] = idx[j] < n;
        px[j] = valid[j] ? a.x[idx[j]] : 0.0f;
        py[j] = valid[j] ? a.y[idx[j]] : 0.0f;
        pz[j] = valid[j] ? a.z[idx[j]] : 0.0f;
        good[j] = valid[j] && finite3(px[j], py[j], pz[j]);
        if (!good[j]) { px[j] = 0.0f; py[j] = 0.0f; pz[j] = 0.0f; }
        good_mask[j] = ballot(good[j]);
    }
    const float kap = a.kappa;
    const float branch_cut = kPiF - 0.25f * kap;
    int32_t lab[P];
    uint64_t enc[P], flg[P];
#pragma unroll
    for (int j = 0; j < P; ++j) { lab[j] = 0; enc[j] = 0; flg[j] = 0; }
    uint32_t n_band = 0, n_cond = 0;
    const int lane = lane_id();

    for (int k = 0; k < a.n_surf; ++k) {
        double S[P];
        uint64_t cmask[P];
#pragma unroll
        for (int j = 0; j < P; ++j) { S[j] = 0.0; cmask[j] = 0; }

        // A point strictly outside the box of a closed surface's vertices is
        // outside its convex hull (w = 0 exactly); a point inside a ball the
        // surface does not cross has the winding number of the ball's centre.
        // When every point of the wavefront qualifies the walk is skipped and
        // S is set to give that w exactly (2 pi in double times kInv2Pi is
        // 1.0); nothing of the test stays live across the walk.
        bool skip = false;
        if (CULL) {
            bool out = true, in = surf[k].ball_w >= 0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                out = out && (!good[j] || px[j] < surf[k].lo[0] || px[j] > surf[k].hi[0] ||
                              py[j] < surf[k].lo[1] || py[j] > surf[k].hi[1] ||
                              pz[j] < surf[k].lo[2] || pz[j] > surf[k].hi[2]);
                const float dx = px[j] - surf[k].ball[0], dy = py[j] - surf[k].ball[1],
                            dz = pz[j] - surf[k].ball[2];
                in = in && (!good[j] || fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < surf[k].ball[3]);
            }
            const int fix = ballot(!out) == 0 ? 0 : (ballot(!in) == 0 ? surf[k].ball_w : -1);
            if (fix >= 0) {
                uint64_t n_good = 0;
#pragma unroll
                for (int j = 0; j < P; ++j) n_good += __popcll(good_mask[j]);
                skip = true;
#pragma unroll
                for (int j = 0; j < P; ++j) S[j] = fix ? kTwoPi : 0.0;
                // one atomic per skipped walk (a count carried through the
                // loop would hold a register)
                if (lane == 0 && n_good)
                    atomicAdd(&a.counters[kCntCulled], (unsigned long long)(n_good * (uint64_t)surf[k].n_tri));
            }
        }
        if (!skip)
            surface_sum<P>(rec, surf[k].rec_begin, surf[k].rec_end, px, py, pz, good_mask, kap, branch_cut,
                           S, cmask);

        // Section 2.1.3: enclosed when s = Omega / 4 pi >= T; later surfaces win.
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const double w = S[j] * kInv2Pi;
            const bool in = w >= a.threshold;
            const bool band = fabs(w - a.threshold) < a.band;
            const bool cond = (cmask[j] >> lane) & 1ull;
            n_band += __popcll(ballot(band) & good_mask[j]);
            n_cond += __popcll(cmask[j]);
            if (band || cond) flg[j] |= 1ull << k;
            if (in) { enc[j] |= 1ull << k; lab[j] = surf[k].label; }
            if (a.winding && valid[j]) {
                const int64_t o = (int64_t)k * n + idx[j];
                const double wv = good[j] ? w : __builtin_nan("");
                if (a.winding_type == SAL_WINDING_F64) ((double *)a.winding)[o] = wv;
                else ((float *)a.winding)[o] = (float)wv;
            }
        }
    }

#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (valid[j]) a.labels[idx[j]] = good[j] ? lab[j] : -1;
        if (a.masks && valid[j]) a.masks[idx[j]] = good[j] ? enc[j] : 0ull;
        append_flag(a, good[j] && flg[j] != 0, idx[j], enc[j], flg[j]);
    }
    if (lane == 0) {
        if (n_band) atomicAdd(&a.counters[kCntBand], (unsigned long long)n_band);
        if (n_cond) atomicAdd(&a.counters[kCntCond], (unsigned long long)n_cond);
    }
}

// ------------------------------------------------------------------ float64
// The plain FP64 form: one point per lane, every triangle in double with the
// exact-sign guard; labels are final.  Held to 128 VGPRs (4 waves per SIMD):
// the few spills this costs sit outside the triangle loop (measured on c2:
// 147 VGPRs / 3 waves 247 G pairs/s, 128 / 4 waves 259, 102 / 5 waves 53).
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_pairloop_f64(PairloopArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = a.n_dev ? *a.n_dev : a.n;
    if ((int64_t)blockIdx.x * blockDim.x >= n) return;
    const bool valid = i < n;
    float fx = valid ? a.x[i] : 0.0f, fy = valid ? a.y[i] : 0.0f, fz = valid ? a.z[i] : 0.0f;
    const bool good = valid && finite3(fx, fy, fz);
    if (!good) { fx = 0.0f; fy = 0.0f; fz = 0.0f; }
    const double p[3] = {fx, fy, fz};
    int32_t lab = 0;
    uint64_t enc = 0;
    unsigned n_exact = 0;
    const CRec64 *rec = (const CRec64 *)a.rec64;
    const CSurf *surf = (const CSurf *)a.surf;
    const uint64_t n_good = __popcll(ballot(good));
    uint64_t culled = 0;
    for (int k = 0; k < a.n_surf; ++k) {
        const int64_t rec_end = surf[k].rec_end;
        double S = 0.0;
        int on = 0;
        // every point of the wavefront strictly outside the box (w = 0
        // exactly) or inside the ball (w = ball_w exactly)
        bool skip = false;
        double wfix = 0.0;
        if (a.cull) {
            const int32_t bw = surf[k].ball_w;
            const bool out = !good || fx < surf[k].lo[0] || fx > surf[k].hi[0] || fy < surf[k].lo[1] ||
                             fy > surf[k].hi[1] || fz < surf[k].lo[2] || fz > surf[k].hi[2];
            const float dx = fx - surf[k].ball[0], dy = fy - surf[k].ball[1], dz = fz - surf[k].ball[2];
            const bool in = bw >= 0 && (!good || fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < surf[k].ball[3]);
            if (ballot(!out) == 0) {
                skip = true;
            } else if (ballot(!in) == 0) {
                skip = true;
                wfix = (double)bw;
            }
        }
        if (skip) culled += n_good * (uint64_t)surf[k].n_tri;
        else S = f64::surface_sum(rec, surf[k].rec_begin, rec_end, p[0], p[1], p[2], fx, fy, fz, on,
                                  n_exact);
        const double w = skip ? wfix : S * kInv2Pi;
        if (on || w >= a.threshold) {
            lab = surf[k].label;
            enc |= 1ull << k;
        }
        if (a.winding && valid) {
            const int64_t o = (int64_t)k * n + i;
            const double wv = good ? w : __builtin_nan("");
            if (a.winding_type == SAL_WINDING_F64) ((double *)a.winding)[o] = wv;
            else ((float *)a.winding)[o] = (float)wv;
        }
    }
    if (valid) a.labels[i] = good ? lab : -1;
    if (a.masks && valid) a.masks[i] = good ? enc : 0ull;
    const uint64_t any = ballot(n_exact != 0);
    if (any) atomicAdd(&a.counters[kCntExact], (unsigned long long)n_exact);
    if (culled && lane_id() == 0) atomicAdd(&a.counters[kCntCulled], (unsigned long long)culled);
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_pairloop_f32(const PairloopArgs &a, int ppl, int block_waves, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int threads = 64 * block_waves;
    const int64_t per_block = (int64_t)threads * ppl;
    const int64_t blocks = (a.n + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)blocks), b(threads);
    switch (ppl * 2 + (a.cull ? 1 : 0)) {
        case 2: k_pairloop_f32<1, false><<<g, b, 0, s>>>(a); break;
        case 3: k_pairloop_f32<1, true><<<g, b, 0, s>>>(a); break;
        case 4: k_pairloop_f32<2, false><<<g, b, 0, s>>>(a); break;
        case 5: k_pairloop_f32<2, true><<<g, b, 0, s>>>(a); break;
        case 8: k_pairloop_f32<4, false><<<g, b, 0, s>>>(a); break;
        case 9: k_pairloop_f32<4, true><<<g, b, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pairloop_f64(const PairloopArgs &a, int block_waves, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int threads = 64 * block_waves;
    const int64_t blocks = (a.n + threads - 1) / threads;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    k_pairloop_f64<<<dim3((unsigned)blocks), dim3(threads), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_fill_u64<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace sal
