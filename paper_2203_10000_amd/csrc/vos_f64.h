// Van Oosterom-Strackee solid angle in double precision along a triangle
// strip (the FP64 form and the FP64 recheck).
//
// For a point p and triangle (A, B, C) with a = A - p, b = B - p, c = C - p:
//   Omega / 2 = atan2(N, D),  N = a . (b x c),
//   D = |a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|
// (Van Oosterom & Strackee, IEEE Trans. Biomed. Eng. 30(2), 1983; the
// paper's section 2.1.3 labels a point by the solid angle of a closed surface
// over 4 pi).  D is symmetric in (a, b, c), so the strip order of the three
// vertices only matters for the sign of N, which is taken from the outward
// normal n = (B - A) x (C - A) stored per triangle: N = (Z - p) . n for any
// vertex Z of the triangle.
//
// When |N| is below its rounding-error bound the sign comes from the exact
// predicate; a point exactly on the triangle's plane and inside the closed
// triangle is "on the surface" (enclosed), otherwise it contributes 0.
#pragma once

#include "exact_dev.h"
#include "sal_internal.h"

namespace sal {

struct StripF64 {
    double dx0, dy0, dz0, r0;   // older vertex X: X - p, |X - p|
    double dx1, dy1, dz1, r1;   // newer vertex Y
    double e01, rr01;           // (X - p).(Y - p), |X - p||Y - p|
    float X[3], Y[3];           // raw coordinates (exact predicate inputs)
};

// Strip window with older vertex X and newer vertex Y (three doubles each).
__device__ __forceinline__ void f64_strip_window(StripF64 &s, const double *X, const double *Y,
                                                 const double *p) {
    s.dx0 = X[0] - p[0];
    s.dy0 = X[1] - p[1];
    s.dz0 = X[2] - p[2];
    s.dx1 = Y[0] - p[0];
    s.dy1 = Y[1] - p[1];
    s.dz1 = Y[2] - p[2];
    s.r0 = sqrt(s.dx0 * s.dx0 + s.dy0 * s.dy0 + s.dz0 * s.dz0);
    s.r1 = sqrt(s.dx1 * s.dx1 + s.dy1 * s.dy1 + s.dz1 * s.dz1);
    s.e01 = s.dx0 * s.dx1 + s.dy0 * s.dy1 + s.dz0 * s.dz1;
    s.rr01 = s.r0 * s.r1;
    s.X[0] = (float)X[0];
    s.X[1] = (float)X[1];
    s.X[2] = (float)X[2];
    s.Y[0] = (float)Y[0];
    s.Y[1] = (float)Y[1];
    s.Y[2] = (float)Y[2];
}

__device__ __forceinline__ void f64_strip_head(StripF64 &s, const double *h, const double *p) {
    f64_strip_window(s, h, h + 3, p);
}

// Result of the exact resolution: the corrected N, and flags (bit 0: the
// point is on the triangle's plane, bit 1: inside the closed triangle).
struct ExactN {
    double n;
    int flags;
};

// Out-of-line exact resolution of a triangle whose N sign is uncertain: the
// corrected N (exact sign, magnitude kept), or 0 with the coplanar flag.
// Coordinates come by value, so the caller's strip window stays in registers
// (a pointer argument would place it in scratch memory for every step).
__device__ __noinline__ ExactN f64_exact_n(float px, float py, float pz, float x0, float x1, float x2,
                                           float y0, float y1, float y2, float z0, float z1, float z2,
                                           double sigma, double n_val) {
    const float P[3] = {px, py, pz}, X[3] = {x0, x1, x2}, Y[3] = {y0, y1, y2}, Z[3] = {z0, z1, z2};
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

// One strip step: the triangle (X, Y, Z) with Z and its normal in record t.
// Returns atan2(N, D) (half the solid angle); advances the strip window.
__device__ __forceinline__ double f64_strip_tri(StripF64 &s, const double *t, const double *p,
                                                const float *praw, int *on,
                                                unsigned *n_exact) {
    const double dx2 = t[0] - p[0], dy2 = t[1] - p[1], dz2 = t[2] - p[2];
    const double r2 = sqrt(dx2 * dx2 + dy2 * dy2 + dz2 * dz2);
    const double e02 = s.dx0 * dx2 + s.dy0 * dy2 + s.dz0 * dz2;
    const double e12 = s.dx1 * dx2 + s.dy1 * dy2 + s.dz1 * dz2;
    double num = dx2 * t[3] + dy2 * t[4] + dz2 * t[5];
    const double den = s.rr01 * r2 + s.e01 * r2 + e02 * s.r1 + e12 * s.r0;
    double half = 0.0;
    // |N - N_exact| <= ~10 eps |Z - p| |B - A| |C - A|; the record holds
    // 32 eps |B - A||C - A| (margin included).
    if (fabs(num) <= r2 * t[6]) {
        const ExactN r = f64_exact_n(praw[0], praw[1], praw[2], s.X[0], s.X[1], s.X[2], s.Y[0], s.Y[1],
                                     s.Y[2], (float)t[0], (float)t[1], (float)t[2], t[7], num);
        num = r.n;
        if (r.flags & 2) *on = 1;
        *n_exact += 1;
        if (!(r.flags & 1)) half = atan2(num, den);
    } else if (den > 16.0 * fabs(num)) {
        // |N / D| < 1/16 with D > 0: atan2(N, D) = atan(t), t = N / D, by its
        // Taylor series to t^13 (the first omitted term is below 1e-18 t)
        const double t = num / den, q = t * t;
        double poly = 1.0 / 13.0;
        poly = fma(poly, q, -1.0 / 11.0);
        poly = fma(poly, q, 1.0 / 9.0);
        poly = fma(poly, q, -1.0 / 7.0);
        poly = fma(poly, q, 1.0 / 5.0);
        poly = fma(poly, q, -1.0 / 3.0);
        half = fma(t * q, poly, t);
    } else {
        half = atan2(num, den);
    }
    // slide the window: (X, Y) <- (Y, Z)
    s.dx0 = s.dx1; s.dy0 = s.dy1; s.dz0 = s.dz1; s.r0 = s.r1;
    s.dx1 = dx2; s.dy1 = dy2; s.dz1 = dz2; s.r1 = r2;
    s.e01 = e12;
    s.rr01 = s.r0 * r2;
    s.X[0] = s.Y[0]; s.X[1] = s.Y[1]; s.X[2] = s.Y[2];
    s.Y[0] = (float)t[0]; s.Y[1] = (float)t[1]; s.Y[2] = (float)t[2];
    return half;
}

}  // namespace sal
