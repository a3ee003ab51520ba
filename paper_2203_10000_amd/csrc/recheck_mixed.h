// Mixed-precision strip walk of the recheck: the winding number of a closed
// surface is an integer away from the surface (section 2.1.3 labels by it), so
// a (point, surface) pair only needs every triangle term correct to far less
// than 1/2 in total.  A term that float32 certifies (the small-angle test of
// the pair loop, or the full atan2 without its conditioning flags) is kept in
// float32; the others are recomputed in double with the exact-sign guard.  The
// float32 terms are the ones the pair loop accepts for unflagged pairs.
#pragma once

#include <hip/hip_runtime.h>

#include "sal_internal.h"
#include "vos_f64.h"

namespace sal {
namespace mixed {

constexpr float kPiF = 3.14159265358979323846f;
// atan(t) = u (1/32 - u^2 / (3 32^3) + u^4 / (5 32^5)) for u = 32 t,
// |t| <= 1/32: the pair loop's small-angle range, with one more term of the
// series (first omitted term below 1e-10 t).
constexpr float kA0 = 0.03125f;
constexpr float kA1 = -1.0172526042e-05f;   // -1 / (3 * 32768)
constexpr float kA2 = 5.9604644775e-09f;    //  1 / (5 * 33554432)
static_assert(kNScale == 32.0f, "series constants assume normals scaled by 32");

struct F64Term {
    double half;      // atan2(N, D)
    int on;           // the point lies on the closed triangle
    unsigned exact;   // exact-sign evaluations made
};

// One triangle (X, Y, Z) in double with the exact-sign guard; Z and the
// double normal come from its FP64 record.  Out of line and by value: it is
// rare, and inlined its registers would count against the float32 walk.
__device__ __noinline__ F64Term f64_triangle(float x0, float x1, float x2, float y0, float y1,
                                             float y2, const double *rec, float px, float py,
                                             float pz) {
    const double Xd[3] = {x0, x1, x2}, Yd[3] = {y0, y1, y2};
    const double pd[3] = {px, py, pz};
    const float pf[3] = {px, py, pz};
    StripF64 st;
    f64_strip_window(st, Xd, Yd, pd);
    F64Term r{0.0, 0, 0u};
    r.half = f64_strip_tri(st, rec, pd, pf, &r.on, &r.exact);
    return r;
}

// Sum of atan2(N, D) over the m triangles of the strip whose head is record r,
// for one lane's point (pf: float32 coordinates, pd: the same in double).
// *on is set when the point lies on one of the triangles; *n_f64 counts the
// triangles recomputed in double.
__device__ __forceinline__ double strip_sum(const Rec32 *__restrict__ rec32,
                                            const Rec64 *__restrict__ rec64, int64_t r, int m,
                                            const float *pf, const double *pd, float kap,
                                            float branch_cut, int *on, unsigned *n_exact,
                                            unsigned *n_f64) {
    const float *h = rec32[r].v;
    float X[3] = {h[0], h[1], h[2]}, Y[3] = {h[3], h[4], h[5]};
    float ax = X[0] - pf[0], ay = X[1] - pf[1], az = X[2] - pf[2];
    float bx = Y[0] - pf[0], by = Y[1] - pf[1], bz = Y[2] - pf[2];
    float ar = __builtin_amdgcn_sqrtf(fmaf(ax, ax, fmaf(ay, ay, az * az)));
    float br = __builtin_amdgcn_sqrtf(fmaf(bx, bx, fmaf(by, by, bz * bz)));
    float e01 = fmaf(ax, bx, fmaf(ay, by, az * bz));
    float rr01 = ar * br;
    float accf = 0.0f;
    double accd = 0.0;
    for (int t = 1; t <= m; ++t) {
        const float *q = rec32[r + t].v;
        const float cx = q[0] - pf[0], cy = q[1] - pf[1], cz = q[2] - pf[2];
        const float cr = __builtin_amdgcn_sqrtf(fmaf(cx, cx, fmaf(cy, cy, cz * cz)));
        const float e02 = fmaf(ax, cx, fmaf(ay, cy, az * cz));
        const float e12 = fmaf(bx, cx, fmaf(by, cy, bz * cz));
        const float nn = fmaf(cx, q[3], fmaf(cy, q[4], cz * q[5]));   // 32 N
        const float mm = rr01 * cr;
        const float dd = fmaf(e12, ar, fmaf(e02, br, fmaf(e01, cr, mm)));
        const float lim = fmaf(q[7], cr, fmaf(kap, mm, fabsf(nn)));
        if (__builtin_expect(dd > lim, 1)) {   // the common case as the fall-through path
            const float u = nn * __builtin_amdgcn_rcpf(dd);
            const float s = u * u;
            accf = fmaf(u, fmaf(fmaf(kA2, s, kA1), s, kA0), accf);
        } else {
            const float n1 = nn * (1.0f / kNScale);
            const float ang = atan2f(n1, dd);
            const float thr = fmaf(cr, kap * q[6], kap * mm);
            const bool ill = fmaxf(fabsf(n1), fabsf(dd)) <= thr;
            const bool cut = fabsf(ang) > branch_cut;
            if (ill || cut) {
                const F64Term d = f64_triangle(X[0], X[1], X[2], Y[0], Y[1], Y[2], rec64[r + t].v,
                                               pf[0], pf[1], pf[2]);
                accd += d.half;
                *on |= d.on;
                *n_exact += d.exact;
                *n_f64 += 1;
            } else {
                accf += ang;
            }
        }
        ax = bx; ay = by; az = bz; ar = br;
        bx = cx; by = cy; bz = cz; br = cr;
        e01 = e12;
        rr01 = ar * cr;
        X[0] = Y[0]; X[1] = Y[1]; X[2] = Y[2];
        Y[0] = q[0]; Y[1] = q[1]; Y[2] = q[2];
    }
    return accd + (double)accf;
}

}  // namespace mixed
}  // namespace sal
