// Double-precision strip walk of the plain FP64 form (k_pairloop_f64).
//
// Same Van Oosterom-Strackee terms as the float32 walk, all in double:
// for the triangle (X, Y, Z) of a strip step, with a = X - p, b = Y - p,
// c = Z - p, the half solid angle is atan2(N, D), N = c . n (n the outward
// normal (B - A) x (C - A) of the original triangle, from the record),
// D = |a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|.  The per-vertex length and
// the per-edge term |a||b| + a.b carry over to the next step, and three vertex
// slots rotate (the loop is unrolled by three), so nothing is copied.
//
// Where the float32 walk is issue-bound on plain ALU work, this one was bound
// by its library calls: a correctly rounded double sqrt and a double division
// each expand to about a dozen instructions with scaling and special-case
// fix-ups that these operands never need.  Here:
//  * |c| = sqrt(s) from the hardware reciprocal square root, one
//    Goldschmidt step and a residual correction.  s carries a seed of
//    1e-200 (the innermost FMA of the sum of squares adds it), so a point on
//    a vertex gets |c| = 1e-100 instead of 0 * inf; any nonzero sum is at
//    least ~1e-90 (a squared difference of two float32 values), which the
//    seed leaves unchanged, and far inside the normal range, so no scaling is
//    needed;
//  * N / D in the small-angle path (only taken when D > 512 |N| > 0) from
//    the hardware reciprocal, one Newton step and a residual correction.
// Both are within a few units in the last place of the correctly rounded
// results; they only enter magnitudes (|c| and the angle of a far triangle),
// never the sign of N, which the exact predicate certifies where double
// cannot.
#pragma once

#include <hip/hip_runtime.h>

#include "exact_dev.h"
#include "pairloop_f32.h"
#include "sal_internal.h"

namespace sal {
namespace f64 {

using f32::CRec64;

struct Vtx {
    double x, y, z, r;   // vertex - p and its length
};

struct Rec {
    double v[8];         // Z, n, 32 eps |B - A||C - A| (slightly enlarged), strip parity
};

// One 64-byte record from the constant address space: a single scalar load.
// Volatile pins the load where the source puts it (see the float32 walk).
__device__ __forceinline__ Rec load_rec(const CRec64 *p) {
    typedef double D8 __attribute__((ext_vector_type(8)));
    typedef __attribute__((address_space(4))) const volatile D8 VD8;
    const D8 w = *(const VD8 *)p;
    Rec r;
#pragma unroll
    for (int c = 0; c < 8; ++c) r.v[c] = w[c];
    return r;
}

// sqrt(s) for s >= 1e-200: y ~ 1/sqrt(s), g = s y, h = y / 2, one
// Goldschmidt step on g, then the residual correction g += (s - g^2) h.  The
// correction is ~2^-48 g, so h needs only the estimate's ~24 bits: the
// Goldschmidt update of h is left out (no change in the result beyond an
// occasional last-place unit).
__device__ __forceinline__ double sqrt_nn(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y;
    const double h = 0.5 * y;
    g = fma(g, fma(-g, h, 0.5), g);
    const double d = fma(-g, g, s);
    return fma(d, h, g);
}

// x^2 + y^2 + z^2 + 1e-200: the seed costs nothing (it replaces the product
// that starts the FMA chain) and keeps the sum a valid sqrt_nn argument.
__device__ __forceinline__ double sq_seeded(double x, double y, double z, double seed) {
    return fma(x, x, fma(y, y, fma(z, z, seed)));
}

// num / den for den > 0 finite (both normal): reciprocal, one Newton step,
// then the residual correction of the quotient.
__device__ __forceinline__ double div_pos(double num, double den) {
    double y = __builtin_amdgcn_rcp(den);
    y = fma(y, fma(-den, y, 1.0), y);
    const double q = num * y;
    return fma(fma(-den, q, num), y, q);
}

// Raw float32 coordinates of vertex v of the strip whose head is record h:
// vertices 0 and 1 are in the head, vertex v >= 2 is record h + v - 1.
__device__ __forceinline__ void strip_vertex(const Rec64 *h, int v, float *out) {
    const double *s = v < 2 ? h->v + 3 * v : h[v - 1].v;
    out[0] = (float)s[0];
    out[1] = (float)s[1];
    out[2] = (float)s[2];
}

struct ExactN {
    double n;    // N with its exact sign (magnitude kept); 0 when coplanar
    int flags;   // bit 0: the point is on the triangle's plane; bit 1: on the closed triangle
};

// Exact resolution of strip step t (triangle (vertex t-1, vertex t,
// vertex t+1)) whose N sign double cannot certify.  Out of line: it is rare,
// and it reads the vertices back from the records instead of keeping float
// copies of the window in registers.
__device__ __noinline__ ExactN exact_step(float px, float py, float pz, const Rec64 *head, int t,
                                          double n_val) {
    const float P[3] = {px, py, pz};
    float X[3], Y[3], Z[3];
    strip_vertex(head, t - 1, X);
    strip_vertex(head, t, Y);
    strip_vertex(head, t + 1, Z);
    const double sigma = head[t].v[7];
    const int o = exact_orient3d(P, X, Y, Z) * (sigma > 0.0 ? 1 : -1);
    ExactN r;
    if (o == 0) {
        r.n = 0.0;
        r.flags = 1 | (exact_in_triangle(P, X, Y, Z) ? 2 : 0);
        return r;
    }
    const double mag = n_val != 0.0 ? fabs(n_val) : 2.2250738585072014e-308;
    r.n = o > 0 ? mag : -mag;
    r.flags = 0;
    return r;
}

// The library atan2 for the near triangles (|N / D| >= 1/512: for a triangle
// with legs h, within about 11 h of the point).  Out of line: inlined, its polynomial constants were
// hoisted out of the loop into some forty registers, which spilled.
__device__ __noinline__ double atan2_ool(double y, double x) { return atan2(y, x); }

// One strip step: triangle (O, N, Z), Z and the normal in q; Z goes to the
// free slot F.  Returns atan2(N, D).
__device__ __forceinline__ double step(const Vtx &O, const Vtx &Nv, Vtx &F, double &kab,
                                       const Rec &q, double px, double py,
                                       double pz, float fx, float fy, float fz,
                                       const Rec64 *head, int t, int &on, unsigned &n_exact,
                                       double seed, double m_third, double fifth) {
    const double x2 = q.v[0] - px, y2 = q.v[1] - py, z2 = q.v[2] - pz;
    const double r2 = sqrt_nn(sq_seeded(x2, y2, z2, seed));
    const double e02 = fma(O.x, x2, fma(O.y, y2, O.z * z2));
    const double e12 = fma(Nv.x, x2, fma(Nv.y, y2, Nv.z * z2));
    double num = fma(x2, q.v[3], fma(y2, q.v[4], z2 * q.v[5]));
    // D = |c| (|a||b| + a.b) + (a.c)|b| + (b.c)|a|; kab = |a||b| + a.b carries
    // over from the previous step
    const double den = fma(r2, kab, fma(e02, Nv.r, e12 * O.r));
    double half;
    const double an = fabs(num), guard = r2 * q.v[6];   // v[6] = 32 eps |B - A||C - A|
    // The common case first, so that it is the fall-through path of the
    // divergent branches: the sign of N is certain and |N / D| < 1/512.
    if (__builtin_expect(an > guard && den > 512.0 * an, 1)) {
        // D > 0: atan(t) by its Taylor series to t^5 (the first omitted
        // term, t^7 / 7, is below 8e-18 t).  Wider ranges need more terms and
        // ran slower: 1/128 with terms to t^7 by 2 %, 1/16 with terms to t^13
        // by 12 %; the atan2 calls of the few extra near triangles cost less
        // than a longer polynomial on every far one.
        const double tt = div_pos(num, den), s = tt * tt;
        const double poly = fma(fifth, s, m_third);   // 1/5 s - 1/3
        half = fma(tt * s, poly, tt);
    } else if (an <= guard) {
        const ExactN x = exact_step(fx, fy, fz, head, t, num);
        num = x.n;
        if (x.flags & 2) on = 1;
        n_exact += 1;
        half = (x.flags & 1) ? 0.0 : atan2_ool(num, den);
    } else {
        half = atan2_ool(num, den);
    }
    kab = fma(Nv.r, r2, e12);
    F.x = x2;
    F.y = y2;
    F.z = z2;
    F.r = r2;
    return half;
}

// Sum of atan2(N, D) over the strips in records [rec_begin, rec_end) for
// one lane's point; *on set when the point lies on one of the triangles.
__device__ __forceinline__ double surface_sum(const CRec64 *rec, int64_t rec_begin, int64_t rec_end,
                                              double px, double py, double pz, float fx, float fy,
                                              float fz, int &on, unsigned &n_exact) {
    double S = 0.0;
    // the sum-of-squares seed, held in scalar registers (as a literal it was
    // copied into a vector register before every use)
    double seed = 1e-200;
    asm("" : "+s"(seed));
    // The series coefficients: -1/3 in scalar and 1/5 in vector registers, so
    // that their FMA takes both as operands (one scalar operand per
    // instruction).  With both as literals the compiler kept -1/3 in a vector
    // register and copied it into the FMA's accumulator every step: one
    // 64-bit move per pair, 1.5 % of the c2 launch (656 -> 646 ms, A/B).
    double m_third = -1.0 / 3.0, fifth = 1.0 / 5.0;
    asm("" : "+s"(m_third));
    asm("" : "+v"(fifth));
    for (int64_t r = rec_begin; r < rec_end;) {
        const Rec hd = load_rec(rec + r);
        const int m = (int)(__double_as_longlong(hd.v[6]) & 0x7fffffff);
        const Rec64 *head = (const Rec64 *)(rec + r);
        Vtx A, B, C;
        A.x = hd.v[0] - px; A.y = hd.v[1] - py; A.z = hd.v[2] - pz;
        B.x = hd.v[3] - px; B.y = hd.v[4] - py; B.z = hd.v[5] - pz;
        A.r = sqrt_nn(sq_seeded(A.x, A.y, A.z, seed));
        B.r = sqrt_nn(sq_seeded(B.x, B.y, B.z, seed));
        double kab = fma(A.r, B.r, fma(A.x, B.x, fma(A.y, B.y, A.z * B.z)));
        double acc = 0.0;
        // records prefetched one step ahead, as in the float32 walk
        const CRec64 *tr = rec + r + 1;
        const int last = m - 1;
        Rec c0 = load_rec(tr), c1, c2;
        int t = 0;
        for (; t + 2 < m; t += 3) {
            __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
            c1 = load_rec(tr + (t + 1));
            __builtin_amdgcn_sched_barrier(0);
            acc += step(A, B, C, kab, c0, px, py, pz, fx, fy, fz, head, t + 1, on,
                        n_exact, seed, m_third, fifth);
            __builtin_amdgcn_s_waitcnt(0xc07f);
            c2 = load_rec(tr + (t + 2));
            __builtin_amdgcn_sched_barrier(0);
            acc += step(B, C, A, kab, c1, px, py, pz, fx, fy, fz, head, t + 2, on,
                        n_exact, seed, m_third, fifth);
            __builtin_amdgcn_s_waitcnt(0xc07f);
            c0 = load_rec(tr + (t + 3 < last ? t + 3 : last));
            __builtin_amdgcn_sched_barrier(0);
            acc += step(C, A, B, kab, c2, px, py, pz, fx, fy, fz, head, t + 3, on,
                        n_exact, seed, m_third, fifth);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        if (t < m) {
            acc += step(A, B, C, kab, c0, px, py, pz, fx, fy, fz, head, t + 1, on,
                        n_exact, seed, m_third, fifth);
            if (t + 1 < m) {
                c1 = load_rec(tr + (t + 1));
                acc += step(B, C, A, kab, c1, px, py, pz, fx, fy, fz, head, t + 2, on,
                            n_exact, seed, m_third, fifth);
            }
        }
        S += acc;
        r += m + 1;
    }
    return S;
}

}  // namespace f64
}  // namespace sal
