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

#include "recheck_mixed.h"
#include "sal_internal.h"

namespace sal {
namespace {

constexpr double kInv2Pi = 0.15915494309189533577;
constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_recheck_f64(RecheckArgs a) {
    __shared__ double red[kThreads];
    const int tid = threadIdx.x;
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
            atomicAdd(&a.counters[kCntRecheck], (unsigned long long)__popcll(e.flg));
        }
    }
    if (n_exact) atomicAdd(&a.counters[kCntExact], (unsigned long long)n_exact);
    if (n_f64) atomicAdd(&a.counters[kCntRecheckF64], (unsigned long long)n_f64);
}

}  // namespace

hipError_t launch_recheck_f64(const RecheckArgs &a, int grid_blocks, hipStream_t s) {
    if (a.n <= 0 || grid_blocks <= 0) return hipSuccess;
    k_recheck_f64<<<dim3(grid_blocks), dim3(kThreads), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace sal
