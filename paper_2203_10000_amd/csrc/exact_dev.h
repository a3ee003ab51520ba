// Exact geometric signs for float32 inputs, device side.
//
// Method: Shewchuk, "Adaptive Precision Floating-Point Arithmetic and Fast
// Robust Geometric Predicates" (1997) -- error-free TwoSum / TwoProduct and
// expansion growth.  For float32 coordinates every product of two is exact in
// double (48 significant bits) and a product of three is exactly hi + lo with
// lo = fma(uv, w, -hi), so a determinant becomes a short list of doubles whose
// exact sum sign is read off a nonoverlapping expansion.
//
// These paths run only when a double evaluation cannot certify a sign, i.e.
// for points (numerically) on a triangle's plane; they are kept out of line so
// the hot loops keep their register budget.
#pragma once

#include <hip/hip_runtime.h>

namespace sal {

struct Expansion {
    double c[48];   // nonoverlapping, increasing magnitude
    int n;
};

__device__ __forceinline__ void exp_add(Expansion &e, double b) {
    // Adds b, keeping the components nonoverlapping (zero components dropped).
    double q = b;
    int w = 0;
    for (int i = 0; i < e.n; ++i) {
        const double h = e.c[i];
        const double s = q + h;
        const double hv = s - q;
        const double qv = s - hv;
        const double err = (q - qv) + (h - hv);
        q = s;
        if (err != 0.0) e.c[w++] = err;
    }
    if (q != 0.0) e.c[w++] = q;
    e.n = w;
}

__device__ __forceinline__ int exp_sign(const Expansion &e) {
    if (e.n == 0) return 0;
    return e.c[e.n - 1] > 0.0 ? 1 : -1;
}

// Adds s * det[u; v; w] (rows) as 6 exact triple products.
__device__ __forceinline__ void exp_add_det3(Expansion &e, double s, const float *u,
                                             const float *v, const float *w) {
    const int r0[6] = {0, 0, 1, 1, 2, 2};
    const int r1[6] = {1, 2, 2, 0, 0, 1};
    const int r2[6] = {2, 1, 0, 2, 1, 0};
    const double sg[6] = {1.0, -1.0, 1.0, -1.0, 1.0, -1.0};
    for (int m = 0; m < 6; ++m) {
        const double uv = (double)u[r0[m]] * (double)v[r1[m]];
        const double hi = uv * (double)w[r2[m]];
        const double lo = fma(uv, (double)w[r2[m]], -hi);
        const double f = s * sg[m];
        if (hi != 0.0) exp_add(e, f * hi);
        if (lo != 0.0) exp_add(e, f * lo);
    }
}

// Exact sign of det[a - p, b - p, c - p]
//   = det[a,b,c] - det[a,b,p] - det[a,p,c] - det[p,b,c]  (multilinearity).
__device__ __noinline__ int exact_orient3d(const float *p, const float *a, const float *b,
                                           const float *c) {
    Expansion e;
    e.n = 0;
    exp_add_det3(e, 1.0, a, b, c);
    exp_add_det3(e, -1.0, a, b, p);
    exp_add_det3(e, -1.0, a, p, c);
    exp_add_det3(e, -1.0, p, b, c);
    return exp_sign(e);
}

// Exact sign of the 2-D orientation of (a, b, c) on the plane without axis `drop`.
__device__ __forceinline__ int exact_orient2d(const float *a, const float *b, const float *c,
                                              int drop) {
    const int u = drop == 0 ? 1 : 0;
    const int v = drop == 2 ? 1 : 2;
    // (bu - au)(cv - av) - (bv - av)(cu - au) = bu cv - bv cu + au bv - av bu + av cu - au cv
    const double t[6] = {(double)b[u] * c[v], -(double)b[v] * c[u], (double)a[u] * b[v],
                         -(double)a[v] * b[u], (double)a[v] * c[u], -(double)a[u] * c[v]};
    Expansion e;
    e.n = 0;
    for (int i = 0; i < 6; ++i)
        if (t[i] != 0.0) exp_add(e, t[i]);
    return exp_sign(e);
}

// p (known coplanar with the triangle) lies in the closed triangle (a, b, c).
__device__ __noinline__ bool exact_in_triangle(const float *p, const float *a, const float *b,
                                               const float *c) {
    const double e1x = (double)b[0] - a[0], e1y = (double)b[1] - a[1], e1z = (double)b[2] - a[2];
    const double e2x = (double)c[0] - a[0], e2y = (double)c[1] - a[1], e2z = (double)c[2] - a[2];
    const double nx = fabs(e1y * e2z - e1z * e2y);
    const double ny = fabs(e1z * e2x - e1x * e2z);
    const double nz = fabs(e1x * e2y - e1y * e2x);
    const int drop = (nx >= ny && nx >= nz) ? 0 : (ny >= nz ? 1 : 2);
    const int st = exact_orient2d(a, b, c, drop);
    if (st == 0) return false;
    const int s0 = exact_orient2d(a, b, p, drop);
    const int s1 = exact_orient2d(b, c, p, drop);
    const int s2 = exact_orient2d(c, a, p, drop);
    return (s0 == 0 || s0 == st) && (s1 == 0 || s1 == st) && (s2 == 0 || s2 == st);
}

}  // namespace sal
