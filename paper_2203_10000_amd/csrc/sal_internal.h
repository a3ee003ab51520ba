// Internal declarations shared by the host runtime (*.cpp) and the gfx950
// kernels (*.hip) of libsal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sal.h"

namespace sal {

// ---------------------------------------------------------------- records
// A surface is stored as triangle strips.  A strip with vertices
// v0, v1, ..., v_{m+1} holds the m triangles (v_i, v_{i+1}, v_{i+2}); the two
// last vertices of one triangle are the two first of the next, so the
// per-vertex terms (v - p, |v - p|) and the dot product of the shared edge
// are computed once per strip step instead of once per triangle.
//
// float32 stream, 32 bytes per record, read by every lane of a wavefront at
// the same address (scalar loads, broadcast through SGPRs):
//   head: { x0, y0, z0, x1, y1, z1, bits(m), 0 }
//   tri : { x, y, z,  32 nx, 32 ny, 32 nz,  |n|,  KN_SMALL |n| }
// where (x, y, z) is the strip's next vertex and n = (B - A) x (C - A) is the
// outward (unnormalised) normal of the original triangle (A, B, C), computed in
// double from the float32 vertices and rounded once.  The factor 32 is a power
// of two (exact) that folds the small-angle bound |N/D| < 1/32 into one
// comparison.
struct alignas(32) Rec32 {
    float v[8];
};

// float64 stream, same record order, 64 bytes per record:
//   head: { x0, y0, z0, x1, y1, z1, bits(m), 0 }
//   tri : { x, y, z,  nx, ny, nz,  32 eps |B - A| |C - A| (enlarged),  sigma }
// sigma = +1 when the strip order (v_i, v_{i+1}, v_{i+2}) is an even
// permutation of (A, B, C), -1 otherwise; it orients the exact predicate.
struct alignas(64) Rec64 {
    double v[8];
};

// |N - N_exact| <= ~10 eps |c| |B - A||C - A| for the double triple product
// N = (Z - p) . n; the FP64 records store 32 eps |B - A||C - A| (32 eps =
// 2^-48, margin included) so the guard is one product: |N| <= |c| v[6].
constexpr double kGuardEps = 32.0 * 1.1102230246251565e-16;
constexpr float kNScale = 32.0f;     // normal pre-scale in the float32 stream (a power of two)
constexpr float kKnSmall = 5.0f;     // small-angle path needs D > 5 |n| r_Z + ...
constexpr int kMaxSurfaces = 64;     // per-point masks are 64-bit

// Per-surface table in device memory.
// Triangles per tuner trial launch: float32 form, FP64 form, and the float32
// screening launches (every shape once, before the closest two are timed on
// the first prefix).
constexpr int kTuneEntries = 3;
constexpr int64_t kTuneTri[kTuneEntries] = {32768, 8192, 8192};

struct SurfaceDev {
    int64_t rec_begin, rec_end;      // [begin, end) in both record streams
    int64_t strip_begin, strip_end;  // [begin, end) in the strip table
    int64_t n_tri;
    int32_t label;
    int32_t pad;
    float lo[3], hi[3];              // bounding box of the vertices (+-inf: never culled)
    float ball[4];                   // centre and squared radius of a ball the surface does
                                     // not cross (radius shrunk for rounding)
    int32_t ball_w;                  // winding number inside that ball (0 or 1), -1: none
    int32_t pad2;
};

// A point with at least one (surface) winding number that the float32 pass
// cannot certify.
struct FlagEntry {
    int64_t idx;     // point index
    uint64_t enc;    // bit k: float32 pass found w_k >= T
    uint64_t flg;    // bit k: surface k must be recomputed in FP64
};

// Device counters (uint64) of one labeling call.
enum Counter {
    kCntFlagged = 0,   // entries appended to the flag list
    kCntBand = 1,      // (point, surface) pairs flagged by the band
    kCntCond = 2,      // pairs flagged by ill-conditioned triangles
    kCntExact = 3,     // exact-sign evaluations
    kCntRecheck = 4,   // pairs recomputed in FP64
    kCntRecheckF64 = 5,  // triangle terms of rechecked pairs evaluated in double
    kCntCulled = 6,      // pairs skipped: every point of the wavefront outside the box
    kNumCounters = 8
};

struct PairloopArgs {
    const Rec32 *__restrict__ rec32;
    const Rec64 *__restrict__ rec64;
    const SurfaceDev *__restrict__ surf;
    int n_surf;
    const float *__restrict__ x;
    const float *__restrict__ y;
    const float *__restrict__ z;
    int64_t n;
    const int64_t *__restrict__ n_dev;   // when set, the point count is read here (n is the
                                         // capacity the grid was sized for)
    float kappa;
    double threshold;
    double band;
    int32_t *__restrict__ labels;
    void *__restrict__ winding;   // [n_surf][n] float or double, or null
    int winding_type;
    int cull;                     // skip a surface for a wavefront whose points all lie
                                  // strictly outside its bounding box (w = 0 exactly)
                                  // or inside its ball (w = ball_w exactly)
    unsigned long long *__restrict__ masks;  // [n] enclosure bits per point, or null
    FlagEntry *__restrict__ flag_list;  // capacity n
    unsigned long long *__restrict__ counters;
};

// Pair-major recheck: the flagged (point, surface) pairs grouped by surface,
// each group padded to a multiple of 64 so that the 64 pairs of a wavefront
// share one surface and its records can be scalar loads.
struct RecheckPair {
    int32_t entry;   // flag-list index; -1 = padding
    int32_t surf;
};
struct RecheckOut {
    double sum;      // sum of atan2(N, D) over the surface (half the solid angle)
    int32_t on;      // the point lies on the surface
    uint32_t pad;
};
struct RecheckSeg {
    unsigned long long count[kMaxSurfaces];
    unsigned long long cursor[kMaxSurfaces];
    unsigned long long off[kMaxSurfaces];
    unsigned long long total;     // padded pair count
    unsigned long long overflow;  // more pairs than capacity: the per-point form runs instead
    unsigned long long splits;    // strip ranges per surface (more wavefronts for few pairs)
};

struct RecheckArgs {
    const Rec32 *__restrict__ rec32;
    const Rec64 *__restrict__ rec64;
    const SurfaceDev *__restrict__ surf;
    const int64_t *__restrict__ strip_off;  // record index of every strip head
    const float *__restrict__ x;
    const float *__restrict__ y;
    const float *__restrict__ z;
    int64_t n;
    double threshold;
    float kappa;
    int32_t *__restrict__ labels;
    void *__restrict__ winding;
    int winding_type;
    int cull;                     // skip a surface for a wavefront whose points all lie
                                  // strictly outside its bounding box (w = 0 exactly)
                                  // or inside its ball (w = ball_w exactly)
    unsigned long long *__restrict__ masks;  // [n] enclosure bits per point, or null
    const FlagEntry *__restrict__ flag_list;
    unsigned long long *__restrict__ counters;
    int n_surf;
    RecheckPair *__restrict__ pairs;      // [pair_cap]
    RecheckOut *__restrict__ pair_out;    // [pair_cap]
    unsigned long long *__restrict__ res; // [flag capacity]: enclosed bits per flagged point
    RecheckSeg *__restrict__ seg;
    int64_t pair_cap;
    int64_t target_waves;                  // wavefronts the pair-major form aims for
};

// Kernel launchers (pairloop.hip, recheck.hip).
hipError_t launch_pairloop_f32(const PairloopArgs &a, int points_per_lane, int block_waves,
                               hipStream_t s);
hipError_t launch_pairloop_f64(const PairloopArgs &a, int block_waves, hipStream_t s);
// The whole recheck: pair-major when the pairs fit, else one workgroup per
// flagged point; grid_blocks sizes the grid-stride kernels.
hipError_t launch_recheck_f64(const RecheckArgs &a, int grid_blocks, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);

// ------------------------------------------------------------ host helpers
sal_status set_error(sal_status s, const std::string &msg);

// Every device allocation of the library goes through here: hipMalloc, or a
// simulated out-of-memory when sal_debug_fail_allocation armed this call.
hipError_t dev_malloc(void **ptr, size_t bytes);
sal_status hip_error(hipError_t e, const char *what);

}  // namespace sal

#define SAL_HIP(expr)                                             \
    do {                                                          \
        hipError_t _e = (expr);                                   \
        if (_e != hipSuccess) return ::sal::hip_error(_e, #expr); \
    } while (0)
