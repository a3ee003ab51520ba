// Float32 strip walk shared by the single-instance and batched pair loops.
#pragma once

#include <hip/hip_runtime.h>

#include "sal_internal.h"

namespace sal {
namespace f32 {

constexpr double kInv2Pi = 0.15915494309189533577;
constexpr double kTwoPi = 6.283185307179586;   // 2 pi in double: kTwoPi * kInv2Pi == 1.0
constexpr float kPiF = 3.14159265358979323846f;

// atan(t) for |t| <= 1/32 given u = 32 t (the record normals carry the
// factor 32):  u (1/32 - u^2 / (3 32^3)), the Taylor series to t^3; the first
// omitted term, t^5 / 5, is below 2e-7 t.
constexpr float kA0 = 0.03125f;
constexpr float kA1 = -1.0172526042e-05f;   // -1 / (3 * 32768)
static_assert(kNScale == 32.0f, "series constants assume normals scaled by 32");

__device__ __forceinline__ uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of m below this lane.
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int64_t bcast_i64(int64_t v, int src) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Appends this lane's entry when `want` (wave-aggregated atomic).
__device__ __forceinline__ void append_flag(const PairloopArgs &a, bool want, int64_t idx,
                                            uint64_t enc, uint64_t flg) {
    const uint64_t m = ballot(want);
    if (m == 0) return;
    const int leader = __builtin_ctzll(m);
    int64_t base = 0;
    if (lane_id() == leader)
        base = (int64_t)atomicAdd(&a.counters[kCntFlagged], (unsigned long long)__popcll(m));
    base = bcast_i64(base, leader);
    if (want) {
        FlagEntry e;
        e.idx = idx;
        e.enc = enc;
        e.flg = flg;
        a.flag_list[base + lanes_below(m)] = e;
    }
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
    return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

// ------------------------------------------------------------------ float32
// Records are read through the constant address space: the address is the
// same for every lane, so each record is one scalar load into SGPRs.
typedef __attribute__((address_space(4))) const Rec32 CRec32;
typedef __attribute__((address_space(4))) const Rec64 CRec64;
typedef __attribute__((address_space(4))) const SurfaceDev CSurf;

struct Vtx {
    float x, y, z, r;   // vertex - p and its length
};

// The eight floats of one triangle record, held in SGPRs.
struct TriRec {
    float v[8];
};

// The load is volatile only to pin it where the source puts it: the compiler
// would otherwise sink a prefetch down to the end of the loop body, next to
// the copy that consumes it.  It is still one scalar load.
__device__ __forceinline__ TriRec load_rec(const CRec32 *p) {
    typedef float F8 __attribute__((ext_vector_type(8)));
    typedef __attribute__((address_space(4))) const volatile F8 VF8;
    const F8 w = *(const VF8 *)p;
    TriRec r;
#pragma unroll
    for (int c = 0; c < 8; ++c) r.v[c] = w[c];
    return r;
}

// One strip step for P points: the triangle (O, N, Z) with Z and its normal in
// record `rec`.  Z is written to the free slot F; the caller rotates the three
// slots (O, N, F) -> (N, F, O) instead of moving registers.
template <int P>
__device__ __forceinline__ void f32_step(const Vtx (&O)[P], const Vtx (&N)[P], Vtx (&F)[P],
                                         float (&e01)[P], float (&rr01)[P], float (&acc)[P],
                                         float (&accn)[P],
                                         const TriRec &rec, const float (&px)[P],
                                         const float (&py)[P], const float (&pz)[P],
                                         const uint64_t (&good_mask)[P], float kap,
                                         float branch_cut, uint64_t (&cmask)[P]) {
    const float q0 = rec.v[0], q1 = rec.v[1], q2 = rec.v[2];
    const float q3 = rec.v[3], q4 = rec.v[4], q5 = rec.v[5];
    const float q6 = rec.v[6], q7 = rec.v[7];
    float x2[P], y2[P], z2[P], r2[P], e02[P], e12[P], nn[P], mm[P], dd[P];
    uint64_t near = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        x2[j] = q0 - px[j];
        y2[j] = q1 - py[j];
        z2[j] = q2 - pz[j];
        r2[j] = __builtin_amdgcn_sqrtf(fmaf(x2[j], x2[j], fmaf(y2[j], y2[j], z2[j] * z2[j])));
        e02[j] = fmaf(O[j].x, x2[j], fmaf(O[j].y, y2[j], O[j].z * z2[j]));
        e12[j] = fmaf(N[j].x, x2[j], fmaf(N[j].y, y2[j], N[j].z * z2[j]));
        nn[j] = fmaf(x2[j], q3, fmaf(y2[j], q4, z2[j] * q5));            // 32 N
        mm[j] = rr01[j] * r2[j];                                         // |a||b||c|
        dd[j] = fmaf(e12[j], O[j].r, fmaf(e02[j], N[j].r, fmaf(e01[j], r2[j], mm[j])));
        // small-angle path: |N/D| < 1/32, D > kappa |a||b||c|, D > 5 |n| |c|
        const float lim = fmaf(q7, r2[j], fmaf(kap, mm[j], fabsf(nn[j])));
        near |= ballot(!(dd[j] > lim)) & good_mask[j];
    }
    // The hint lays the series out as the fall-through path (without it the
    // atan2 block fell through and the common path took three branches per
    // step: 2 % of the c2 launch time).
    if (__builtin_expect(near == 0, 1)) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const float u = nn[j] * __builtin_amdgcn_rcpf(dd[j]);
            acc[j] = fmaf(u, fmaf(kA1, u * u, kA0), acc[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const float n1 = nn[j] * (1.0f / kNScale);
            const float ang = atan2f(n1, dd[j]);
            const float thr = fmaf(r2[j], kap * q6, kap * mm[j]);
            const bool ill = fmaxf(fabsf(n1), fabsf(dd[j])) <= thr;
            const bool cut = fabsf(ang) > branch_cut;
            cmask[j] |= (ballot(ill) | ballot(cut)) & good_mask[j];
            accn[j] += ang;
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        rr01[j] = N[j].r * r2[j];
        e01[j] = e12[j];
        F[j].x = x2[j];
        F[j].y = y2[j];
        F[j].z = z2[j];
        F[j].r = r2[j];
    }
}


// Sums atan2(N, D) = Omega / 2 over the strips in records [rec_begin,
// rec_end) for the P points of this lane: S[j] += per-strip float32 sums,
// cmask[j] |= lanes whose pair is ill-conditioned.
template <int P>
__device__ __forceinline__ void surface_sum(const CRec32 *rec, int64_t rec_begin, int64_t rec_end,
                                            const float (&px)[P], const float (&py)[P],
                                            const float (&pz)[P], const uint64_t (&good_mask)[P],
                                            float kap, float branch_cut, double (&S)[P],
                                            uint64_t (&cmask)[P]) {
    for (int64_t r = rec_begin; r < rec_end;) {
        const CRec32 *h = rec + r;
        const int m = __float_as_int(h->v[6]);
        const float h0 = h->v[0], h1 = h->v[1], h2 = h->v[2];
        const float h3 = h->v[3], h4 = h->v[4], h5 = h->v[5];
        Vtx A[P], B[P], C[P];
        // Small-angle terms and full-atan2 terms go to separate float sums,
        // so the two paths do not merge one register (no copy per step).
        float e01[P], rr01[P], acc[P], accn[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            A[j].x = h0 - px[j]; A[j].y = h1 - py[j]; A[j].z = h2 - pz[j];
            B[j].x = h3 - px[j]; B[j].y = h4 - py[j]; B[j].z = h5 - pz[j];
            A[j].r = __builtin_amdgcn_sqrtf(fmaf(A[j].x, A[j].x, fmaf(A[j].y, A[j].y, A[j].z * A[j].z)));
            B[j].r = __builtin_amdgcn_sqrtf(fmaf(B[j].x, B[j].x, fmaf(B[j].y, B[j].y, B[j].z * B[j].z)));
            e01[j] = fmaf(A[j].x, B[j].x, fmaf(A[j].y, B[j].y, A[j].z * B[j].z));
            rr01[j] = A[j].r * B[j].r;
            acc[j] = 0.0f;
            accn[j] = 0.0f;
        }
        // Triangle records are prefetched one step ahead: each step first
        // waits for the scalar loads in flight (the record it is about to
        // use), then issues the load of the next record, then computes, so a
        // load overlaps a whole step.  The explicit wait orders the two
        // (scalar loads can return out of order, so any wait is a wait for
        // all of them).  Indices are clamped to the strip's last record.
        const CRec32 *tr = h + 1;
        const int last = m - 1;
        TriRec c0 = load_rec(tr), c1, c2;
        int t = 0;
        for (; t + 2 < m; t += 3) {
            __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
            c1 = load_rec(tr + (t + 1));
            __builtin_amdgcn_sched_barrier(0);     // keep the step's arithmetic below
            f32_step<P>(A, B, C, e01, rr01, acc, accn, c0, px, py, pz, good_mask, kap, branch_cut, cmask);
            __builtin_amdgcn_s_waitcnt(0xc07f);
            c2 = load_rec(tr + (t + 2));
            __builtin_amdgcn_sched_barrier(0);
            f32_step<P>(B, C, A, e01, rr01, acc, accn, c1, px, py, pz, good_mask, kap, branch_cut, cmask);
            __builtin_amdgcn_s_waitcnt(0xc07f);
            c0 = load_rec(tr + (t + 3 < last ? t + 3 : last));
            __builtin_amdgcn_sched_barrier(0);
            f32_step<P>(C, A, B, e01, rr01, acc, accn, c2, px, py, pz, good_mask, kap, branch_cut, cmask);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        if (t < m) {
            f32_step<P>(A, B, C, e01, rr01, acc, accn, c0, px, py, pz, good_mask, kap, branch_cut, cmask);
            if (t + 1 < m) {
                c1 = load_rec(tr + (t + 1));
                f32_step<P>(B, C, A, e01, rr01, acc, accn, c1, px, py, pz, good_mask, kap, branch_cut, cmask);
            }
        }
#pragma unroll
        for (int j = 0; j < P; ++j) S[j] += (double)acc[j] + (double)accn[j];
        r += m + 1;
    }
}

}  // namespace f32
}  // namespace sal
