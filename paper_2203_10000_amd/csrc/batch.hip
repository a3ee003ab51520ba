// Batched labeling: many independent (surface set, point set) instances in
// one persistent launch.
//
// Work item = (instance, block of 64 points, surface, strip range).  Items are
// ordered by cost, largest first, and every resident wavefront pulls the next
// item from a device counter until the list is exhausted (every wavefront
// exits when the counter passes the item count).  An item writes its 64
// float64 partial sums and a 64-bit lane mask to a slot (float32 form: the
// conditioning flags; plain FP64 form: the points found on the surface); the
// finalize pass adds the slots of each (point, surface) in split order, so
// results do not depend on which wavefront ran what.
#include <hip/hip_runtime.h>

#include "batch_internal.h"
#include "pairloop_f32.h"
#include "pairloop_f64.h"
#include "recheck_mixed.h"
#include "vos_f64.h"

namespace sal {
namespace {

using namespace f32;

typedef __attribute__((address_space(4))) const BatchItem CItem;
typedef __attribute__((address_space(4))) const BatchInst CInst;

__global__ __launch_bounds__(256) void k_batch_pairloop(BatchArgs a) {
    const CItem *items = (const CItem *)a.items;
    const CInst *insts = (const CInst *)a.insts;
    const int lane = lane_id();
    const float kap = a.kappa;
    const float branch_cut = kPiF - 0.25f * kap;
    for (;;) {
        // Every lane takes part in the atomic (only lane 0 adds 1), so the loop
        // has no lane-dependent branch; lane 0's old value is the claimed item.
        // (A lane-0-only `if` around the atomic let the compiler build a loop
        // that only lane 0 could leave.)
        const unsigned int got = atomicAdd(a.next_item, lane == 0 ? 1u : 0u);
        const unsigned int it = (unsigned int)__builtin_amdgcn_readfirstlane((int)got);
        if ((int64_t)it >= a.n_items) break;
        const CItem *item = items + it;
        const CInst *inst = insts + item->inst;
        const int64_t p = item->block * 64 + lane;
        const bool valid = p < inst->n;
        float px[1], py[1], pz[1];
        px[0] = valid ? inst->x[p] : 0.0f;
        py[0] = valid ? inst->y[p] : 0.0f;
        pz[0] = valid ? inst->z[p] : 0.0f;
        const bool good = valid && finite3(px[0], py[0], pz[0]);
        if (!good) { px[0] = 0.0f; py[0] = 0.0f; pz[0] = 0.0f; }
        const uint64_t gm[1] = {ballot(good)};
        double S[1] = {0.0};
        uint64_t cmask[1] = {0};
        surface_sum<1>((const CRec32 *)inst->rec32, item->rec_begin, item->rec_end, px, py, pz, gm,
                       kap, branch_cut, S, cmask);
        a.partial[item->slot * 64 + lane] = S[0];
        if (lane == 0) a.slot_mask[item->slot] = cmask[0];
    }
}

// The plain FP64 form of the same work list: every pair in double with the
// exact sign where double cannot certify it (the per-point FP64 walk), no
// float32 pass and so no recheck.  Occupancy as the per-point FP64 kernel.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_pairloop_f64(
    BatchArgs a) {
    const CItem *items = (const CItem *)a.items;
    const CInst *insts = (const CInst *)a.insts;
    const int lane = lane_id();
    for (;;) {
        // claim as in the float32 kernel: every lane executes the atomic
        const unsigned int got = atomicAdd(a.next_item, lane == 0 ? 1u : 0u);
        const unsigned int it = (unsigned int)__builtin_amdgcn_readfirstlane((int)got);
        if ((int64_t)it >= a.n_items) break;
        const CItem *item = items + it;
        const CInst *inst = insts + item->inst;
        const int64_t p = item->block * 64 + lane;
        const bool valid = p < inst->n;
        float fx = valid ? inst->x[p] : 0.0f, fy = valid ? inst->y[p] : 0.0f,
              fz = valid ? inst->z[p] : 0.0f;
        const bool good = valid && finite3(fx, fy, fz);
        if (!good) { fx = 0.0f; fy = 0.0f; fz = 0.0f; }
        int on = 0;
        unsigned n_exact = 0;
        const double S = f64::surface_sum((const CRec64 *)inst->rec64, item->rec_begin,
                                          item->rec_end, fx, fy, fz, fx, fy, fz, on, n_exact);
        a.partial[item->slot * 64 + lane] = S;
        const uint64_t on_mask = ballot(on != 0 && good);
        if (lane == 0) a.slot_mask[item->slot] = on_mask;
        if (n_exact && good)
            atomicAdd(&a.inst_counters[(int64_t)item->inst * kNumCounters + kCntExact],
                      (unsigned long long)n_exact);
    }
}

__device__ __forceinline__ int find_inst(const BatchInst *insts, int n_inst, int64_t gp) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (insts[mid].point_base <= gp) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Per point: winding numbers from the partial slots, the label decision of
// section 2.1.3 (s >= T, later surface wins) and the recheck flags.  In the
// plain FP64 form the slot masks mark points on the surface (enclosed) and
// nothing is flagged.
__global__ __launch_bounds__(256) void k_batch_finalize(BatchArgs a) {
    const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = gp < a.total_points;
    int ii = 0;
    int64_t p = 0;
    bool good = false, want = false;
    uint64_t enc = 0, flg = 0;
    if (live) {
        ii = find_inst(a.insts, a.n_inst, gp);
        const BatchInst &in = a.insts[ii];
        p = gp - in.point_base;
        good = finite3(in.x[p], in.y[p], in.z[p]);
        const int64_t block = p >> 6;
        const int ln = (int)(p & 63);
        int32_t lab = 0;
        unsigned n_band = 0, n_cond = 0;
        for (int k = 0; k < in.n_surf; ++k) {
            double S = 0.0;
            bool bit = false;
            for (int s = in.split_off[k]; s < in.split_off[k + 1]; ++s) {
                const int64_t slot = in.slot_base + block * in.splits_total + s;
                S += a.partial[slot * 64 + ln];
                bit |= ((a.slot_mask[slot] >> ln) & 1ull) != 0;
            }
            const double w = S * kInv2Pi;
            const bool inside = (a.fp64 && bit) || w >= a.threshold;
            const bool band = !a.fp64 && fabs(w - a.threshold) < a.band;
            const bool cond = !a.fp64 && bit;
            if (inside) { enc |= 1ull << k; lab = in.surf_label[k]; }
            if (band || cond) flg |= 1ull << k;
            n_band += band;
            n_cond += cond;
        }
        in.labels[p] = good ? lab : -1;
        want = good && flg != 0;
        if (good && (n_band || n_cond)) {
            unsigned long long *c = a.inst_counters + (int64_t)ii * kNumCounters;
            if (n_band) atomicAdd(&c[kCntBand], (unsigned long long)n_band);
            if (n_cond) atomicAdd(&c[kCntCond], (unsigned long long)n_cond);
        }
    }
    const uint64_t m = ballot(want);
    if (m == 0) return;
    const int leader = __builtin_ctzll(m);
    int64_t base = 0;
    if (lane_id() == leader)
        base = (int64_t)atomicAdd(&a.counters[kCntFlagged], (unsigned long long)__popcll(m));
    base = bcast_i64(base, leader);
    if (want) {
        FlagEntry e;
        e.idx = gp;
        e.enc = enc;
        e.flg = flg;
        a.flag_list[base + lanes_below(m)] = e;
    }
}

constexpr int kRecheckThreads = 256;

__global__ __launch_bounds__(kRecheckThreads) void k_batch_recheck(BatchArgs a) {
    __shared__ double red[kRecheckThreads];
    const int tid = threadIdx.x;
    int64_t count = (int64_t)a.counters[kCntFlagged];
    if (count > a.total_points) count = a.total_points;
    const float branch_cut = mixed::kPiF - 0.25f * a.kappa;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const FlagEntry e = a.flag_list[i];
        const int ii = find_inst(a.insts, a.n_inst, e.idx);
        const BatchInst &in = a.insts[ii];
        const int64_t p = e.idx - in.point_base;
        const float praw[3] = {in.x[p], in.y[p], in.z[p]};
        const double pd[3] = {praw[0], praw[1], praw[2]};
        uint64_t enc = e.enc;
        uint64_t f = e.flg;
        unsigned n_exact = 0, n_f64 = 0;
        while (f) {
            const int k = __builtin_ctzll(f);
            f &= f - 1;
            const SurfaceDev sd = in.surf[k];
            double part = 0.0;
            int on = 0;
            for (int64_t s = sd.strip_begin + tid; s < sd.strip_end; s += kRecheckThreads) {
                const int64_t r = in.strip_off[s];
                const int m = __float_as_int(in.rec32[r].v[6]);
                part += mixed::strip_sum(in.rec32, in.rec64, r, m, praw, pd, a.kappa, branch_cut,
                                         &on, &n_exact, &n_f64);
            }
            red[tid] = part;
            on = __syncthreads_or(on);
            for (int w = kRecheckThreads / 2; w > 0; w >>= 1) {
                if (tid < w) red[tid] += red[tid + w];
                __syncthreads();
            }
            const double wk = red[0] * kInv2Pi;
            __syncthreads();
            if (on || wk >= a.threshold) enc |= 1ull << k;
            else enc &= ~(1ull << k);
        }
        unsigned long long *c = a.inst_counters + (int64_t)ii * kNumCounters;
        if (n_exact) atomicAdd(&c[kCntExact], (unsigned long long)n_exact);
        if (n_f64) atomicAdd(&c[kCntRecheckF64], (unsigned long long)n_f64);
        if (tid == 0) {
            in.labels[p] = enc ? in.surf_label[63 - __builtin_clzll(enc)] : 0;
            atomicAdd(&c[kCntRecheck], (unsigned long long)__popcll(e.flg));
            atomicAdd(&c[kCntFlagged], 1ull);
        }
    }
}

}  // namespace

hipError_t launch_batch(const BatchArgs &a, int persistent_blocks, int recheck_blocks,
                        hipStream_t s) {
    if (a.n_items > 0) {
        if (a.fp64) k_batch_pairloop_f64<<<dim3(persistent_blocks), dim3(256), 0, s>>>(a);
        else k_batch_pairloop<<<dim3(persistent_blocks), dim3(256), 0, s>>>(a);
    }
    if (a.total_points > 0) {
        const int64_t g = (a.total_points + 255) / 256;
        k_batch_finalize<<<dim3((unsigned)g), dim3(256), 0, s>>>(a);
        if (!a.fp64)
            k_batch_recheck<<<dim3(recheck_blocks), dim3(kRecheckThreads), 0, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace sal
