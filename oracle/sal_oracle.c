/*
 * FP64 CPU oracle for solid-angle labeling -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline timing use it; the GPU library never does, and the
 * two share no code.  Build: gcc -O2 -ffp-contract=off (no fast-math).
 *
 * Sources of the arithmetic:
 *  - Paper section 2.1.3 (Eq. 1): the labeling integral is the solid angle of
 *    the closed surface seen from the point, over 4 pi (the printed integrand
 *    lacks the |r - r_i|^-3 factor; the surrounding text defines s_i as the
 *    ratio of the subtended solid angle to the full angle).  The inside test is
 *    s_i >= T.
 *  - Per flat triangle, the solid angle is exact by the Van Oosterom-Strackee
 *    formula (IEEE Trans. Biomed. Eng. 30(2), 1983), which the paper takes from
 *    its labeling reference:
 *        tan(Omega / 2) = a.(b x c) / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|),
 *    a, b, c the vertices relative to the point, evaluated with atan2.
 *  - Section 2.1: nested compartments, the one first in the hierarchy wins
 *    where boundaries intersect; a bounding box is the outermost compartment.
 *  - The sign of a.(b x c) is made exact where the double value cannot certify
 *    it, with the expansion arithmetic of Shewchuk, "Adaptive Precision
 *    Floating-Point Arithmetic and Fast Robust Geometric Predicates" (1997):
 *    TwoSum, TwoProduct and Grow-Expansion.
 */
#define _GNU_SOURCE
#include "sal_oracle.h"

#include <float.h>
#include <math.h>
#include <pthread.h>
#include <sched.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ---------------------------------------------------------------- exact sums
 * Error-free transformations (Shewchuk 1997, section 2).  Every float32 value
 * is exact in double; a product of two of them is exact in double (48 bits);
 * a product of three is exactly hi + lo with lo from a fused multiply-add. */

static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *s = x;
    *e = (a - av) + (b - bv);
}

/* Grow-Expansion with zero elimination: adds b to the nonoverlapping
 * expansion h[0..*m) (increasing magnitude); the result stays nonoverlapping
 * and its exact sum is the old sum plus b. */
static void grow_expansion(double *h, int *m, double b)
{
    double q = b;
    int k = 0;
    for (int i = 0; i < *m; ++i) {
        double s, e;
        two_sum(q, h[i], &s, &e);
        q = s;
        if (e != 0.0)
            h[k++] = e;
    }
    if (q != 0.0)
        h[k++] = q;
    *m = k;
}

/* Exact sign of the sum of n doubles: the most significant component of a
 * nonoverlapping expansion carries the sign of its sum. */
static int exact_sum_sign(const double *x, int n)
{
    double h[64];
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (x[i] != 0.0)
            grow_expansion(h, &m, x[i]);
    if (m == 0)
        return 0;
    return h[m - 1] > 0.0 ? 1 : -1;
}

/* s * u * v * w exactly, as two doubles appended to out[*k]. */
static void push_triple(double *out, int *k, double s, double u, double v, double w)
{
    double uv = u * v;                /* exact: float32 x float32 */
    double hi = uv * w;
    double lo = fma(uv, w, -hi);      /* exact remainder */
    out[(*k)++] = s * hi;
    out[(*k)++] = s * lo;
}

/* det3 of rows u, v, w as 6 signed triple products (exact, 12 doubles). */
static void push_det3(double *out, int *k, double sign, const double *u,
                      const double *v, const double *w)
{
    push_triple(out, k, sign, u[0], v[1], w[2]);
    push_triple(out, k, -sign, u[0], v[2], w[1]);
    push_triple(out, k, sign, u[1], v[2], w[0]);
    push_triple(out, k, -sign, u[1], v[0], w[2]);
    push_triple(out, k, sign, u[2], v[0], w[1]);
    push_triple(out, k, -sign, u[2], v[1], w[0]);
}

int oracle_orient3d_sign(const float p[3], const float v0[3], const float v1[3],
                         const float v2[3])
{
    /* det[v0-p, v1-p, v2-p] is the 4x4 determinant with rows (v0,1), (v1,1),
     * (v2,1), (p,1); along the column of ones it is
     *   det3(v0,v1,v2) - det3(v0,v1,p) + det3(v0,v2,p) - det3(v1,v2,p),
     * a sum of 24 products of three float32 coordinates. */
    double a[3], b[3], c[3], d[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = v0[i];
        b[i] = v1[i];
        c[i] = v2[i];
        d[i] = p[i];
    }
    double terms[48];
    int k = 0;
    push_det3(terms, &k, 1.0, a, b, c);
    push_det3(terms, &k, -1.0, a, b, d);
    push_det3(terms, &k, 1.0, a, c, d);
    push_det3(terms, &k, -1.0, b, c, d);
    return exact_sum_sign(terms, k);
}

int oracle_orient2d_sign(const float a[3], const float b[3], const float c[3], int drop)
{
    int u = drop == 0 ? 1 : 0;
    int v = drop == 2 ? 1 : 2;
    /* (bu-au)(cv-av) - (bv-av)(cu-au), expanded into 6 exact products. */
    double au = a[u], av = a[v], bu = b[u], bv = b[v], cu = c[u], cv = c[v];
    double t[6] = {bu * cv, -bu * av, -au * cv, -bv * cu, bv * au, av * cu};
    return exact_sum_sign(t, 6);
}

/* Sign of det[v0-p, v1-p, v2-p]: the double value when its static error
 * bound certifies the sign, the exact expansion otherwise. */
int oracle_orient3d(const float p[3], const float v0[3], const float v1[3],
                             const float v2[3])
{
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = (double)v0[i] - (double)p[i];
        b[i] = (double)v1[i] - (double)p[i];
        c[i] = (double)v2[i] - (double)p[i];
    }
    double det = a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2])
               + a[2] * (b[0] * c[1] - b[1] * c[0]);
    double perm = fabs(a[0]) * (fabs(b[1] * c[2]) + fabs(b[2] * c[1]))
                + fabs(a[1]) * (fabs(b[2] * c[0]) + fabs(b[0] * c[2]))
                + fabs(a[2]) * (fabs(b[0] * c[1]) + fabs(b[1] * c[0]));
    if (det > 16.0 * DBL_EPSILON * perm)
        return 1;
    if (-det > 16.0 * DBL_EPSILON * perm)
        return -1;
    return oracle_orient3d_sign(p, v0, v1, v2);
}

/* p in the closed triangle, for p known to be coplanar with it. */
static int in_closed_triangle(const float p[3], const float v0[3], const float v1[3],
                              const float v2[3])
{
    double e1[3], e2[3], n[3];
    for (int i = 0; i < 3; ++i) {
        e1[i] = (double)v1[i] - (double)v0[i];
        e2[i] = (double)v2[i] - (double)v0[i];
    }
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    int drop = 0;
    if (fabs(n[1]) > fabs(n[drop]))
        drop = 1;
    if (fabs(n[2]) > fabs(n[drop]))
        drop = 2;
    int st = oracle_orient2d_sign(v0, v1, v2, drop);
    if (st == 0)
        return 0; /* degenerate triangle: no area to lie on */
    int s0 = oracle_orient2d_sign(v0, v1, p, drop);
    int s1 = oracle_orient2d_sign(v1, v2, p, drop);
    int s2 = oracle_orient2d_sign(v2, v0, p, drop);
    return (s0 == 0 || s0 == st) && (s1 == 0 || s1 == st) && (s2 == 0 || s2 == st);
}

/* ------------------------------------------------------ one triangle, VOS */

double oracle_tri_solid_angle(const float p[3], const float v0[3], const float v1[3],
                              const float v2[3], int *on_tri)
{
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = (double)v0[i] - (double)p[i];
        b[i] = (double)v1[i] - (double)p[i];
        c[i] = (double)v2[i] - (double)p[i];
    }
    double bxc0 = b[1] * c[2] - b[2] * c[1];
    double bxc1 = b[2] * c[0] - b[0] * c[2];
    double bxc2 = b[0] * c[1] - b[1] * c[0];
    double num = a[0] * bxc0 + a[1] * bxc1 + a[2] * bxc2;

    /* Static error bound of the triple product (rounded differences
     * included): well above Shewchuk's (7 + 56 eps) eps * permanent. */
    double perm = fabs(a[0]) * (fabs(b[1] * c[2]) + fabs(b[2] * c[1]))
                + fabs(a[1]) * (fabs(b[2] * c[0]) + fabs(b[0] * c[2]))
                + fabs(a[2]) * (fabs(b[0] * c[1]) + fabs(b[1] * c[0]));
    if (fabs(num) <= 16.0 * DBL_EPSILON * perm) {
        int s = oracle_orient3d_sign(p, v0, v1, v2);
        if (s == 0) {
            /* p is in the triangle's plane: either on the triangle (then on
             * the surface) or seen edge-on with zero solid angle. */
            if (on_tri)
                *on_tri = in_closed_triangle(p, v0, v1, v2);
            return 0.0;
        }
        if (num == 0.0 || (num > 0.0) != (s > 0))
            num = (double)s * (num == 0.0 ? DBL_MIN : fabs(num));
    }
    double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double ac = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
    double den = la * lb * lc + ab * lc + ac * lb + bc * la;
    return 2.0 * atan2(num, den);
}

/* Winding number of one surface at one point: Neumaier-compensated sum over
 * the triangles in index order, divided by 4 pi. */
static double winding_one(const float p[3], const float *verts, int64_t n_tri,
                          const int32_t *tris, int *on_surf)
{
    double s = 0.0, comp = 0.0;
    int on = 0;
    for (int64_t t = 0; t < n_tri; ++t) {
        const float *v0 = verts + 3 * (int64_t)tris[3 * t + 0];
        const float *v1 = verts + 3 * (int64_t)tris[3 * t + 1];
        const float *v2 = verts + 3 * (int64_t)tris[3 * t + 2];
        int on_tri = 0;
        double x = oracle_tri_solid_angle(p, v0, v1, v2, &on_tri);
        on |= on_tri;
        double u = s + x;
        if (fabs(s) >= fabs(x))
            comp += (s - u) + x;
        else
            comp += (x - u) + s;
        s = u;
    }
    *on_surf = on;
    return (s + comp) / (4.0 * M_PI);
}

/* ------------------------------------------------------------ thread pool */

typedef oracle_range_fn range_fn;

struct range_job {
    range_fn fn;
    void *ctx;
    int64_t begin, end;
};

static void *range_thread(void *arg)
{
    struct range_job *j = (struct range_job *)arg;
    j->fn(j->ctx, j->begin, j->end);
    return NULL;
}

static int resolve_threads(int n_threads)
{
    if (n_threads > 0)
        return n_threads;
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        int c = CPU_COUNT(&set);
        if (c > 0)
            return c;
    }
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

/* Splits [0, n) into one contiguous range per thread, [n i / nt, n (i+1) / nt)
 * (lengths differ by at most one); each index is computed by exactly one
 * thread, so results do not depend on the thread count. */
void oracle_parallel_for(int64_t n, int n_threads, range_fn fn, void *ctx)
{
    int nt = resolve_threads(n_threads);
    if (nt > 256)
        nt = 256;
    if (n < 2 * nt)
        nt = 1;
    if (nt == 1) {
        fn(ctx, 0, n);
        return;
    }
    pthread_t th[256];
    struct range_job jobs[256];
    for (int i = 0; i < nt; ++i) {
        jobs[i].fn = fn;
        jobs[i].ctx = ctx;
        jobs[i].begin = n * i / nt;
        jobs[i].end = n * (i + 1) / nt;
        pthread_create(&th[i], NULL, range_thread, &jobs[i]);
    }
    for (int i = 0; i < nt; ++i)
        pthread_join(th[i], NULL);
}

/* ---------------------------------------------------------- winding, labels */

struct winding_ctx {
    const float *px, *py, *pz, *verts;
    const int32_t *tris;
    int64_t n_tri;
    double *w;
    uint8_t *on;
};

static void winding_range(void *vctx, int64_t b, int64_t e)
{
    struct winding_ctx *c = (struct winding_ctx *)vctx;
    for (int64_t i = b; i < e; ++i) {
        float p[3] = {c->px[i], c->py[i], c->pz[i]};
        int on = 0;
        c->w[i] = winding_one(p, c->verts, c->n_tri, c->tris, &on);
        if (c->on)
            c->on[i] = (uint8_t)on;
    }
}

void oracle_winding(int64_t n, const float *px, const float *py, const float *pz,
                    int64_t n_vert, const float *verts, int64_t n_tri,
                    const int32_t *tris, int n_threads, double *w, uint8_t *on_surf)
{
    (void)n_vert;
    struct winding_ctx c = {px, py, pz, verts, tris, n_tri, w, on_surf};
    oracle_parallel_for(n, n_threads, winding_range, &c);
}

struct label_ctx {
    const float *px, *py, *pz, *verts;
    const int32_t *tris, *surf_label;
    const int64_t *vert_off, *tri_off;
    int n_surf;
    int64_t n;
    double threshold;
    int32_t *labels;
    double *w_out;
    uint64_t *mask_out;
};

static void label_range(void *vctx, int64_t b, int64_t e)
{
    struct label_ctx *c = (struct label_ctx *)vctx;
    for (int64_t i = b; i < e; ++i) {
        float p[3] = {c->px[i], c->py[i], c->pz[i]};
        int32_t label = 0; /* bounding box */
        uint64_t mask = 0;
        for (int s = 0; s < c->n_surf; ++s) {
            const float *v = c->verts + 3 * c->vert_off[s];
            const int32_t *t = c->tris + 3 * c->tri_off[s];
            int64_t nt = c->tri_off[s + 1] - c->tri_off[s];
            int on = 0;
            double w = winding_one(p, v, nt, t, &on);
            if (c->w_out)
                c->w_out[(int64_t)s * c->n + i] = w;
            /* later surfaces have higher priority: they overwrite */
            if (on || w >= c->threshold) {
                if (c->surf_label)
                    label = c->surf_label[s];
                mask |= (uint64_t)1 << s;
            }
        }
        if (c->labels)
            c->labels[i] = label;
        if (c->mask_out)
            c->mask_out[i] = mask;
    }
}

int64_t oracle_label(int64_t n, const float *px, const float *py, const float *pz,
                     int n_surf, const int64_t *vert_off, const int64_t *tri_off,
                     const float *verts, const int32_t *tris,
                     const int32_t *surf_label, double threshold, int n_threads,
                     int32_t *labels, double *w_out)
{
    struct label_ctx c = {px, py, pz, verts, tris, surf_label, vert_off, tri_off,
                          n_surf, n, threshold, labels, w_out, NULL};
    oracle_parallel_for(n, n_threads, label_range, &c);
    return n * (tri_off[n_surf] - tri_off[0]);
}

int64_t oracle_enclosure(int64_t n, const float *px, const float *py, const float *pz,
                         int n_surf, const int64_t *vert_off, const int64_t *tri_off,
                         const float *verts, const int32_t *tris, double threshold,
                         int n_threads, uint64_t *masks)
{
    struct label_ctx c = {px, py, pz, verts, tris, NULL, vert_off, tri_off,
                          n_surf, n, threshold, NULL, NULL, masks};
    if (n_surf > 64)
        return -1;
    oracle_parallel_for(n, n_threads, label_range, &c);
    return n * (tri_off[n_surf] - tri_off[0]);
}

/* ------------------------------------------------------------ radial test */

struct radial_ctx {
    const float *px, *py, *pz, *center, *verts;
    const int32_t *tris;
    int64_t n_tri;
    uint8_t *out;
};

static void radial_range(void *vctx, int64_t b, int64_t e)
{
    struct radial_ctx *c = (struct radial_ctx *)vctx;
    const float *ctr = c->center;
    for (int64_t i = b; i < e; ++i) {
        float p[3] = {c->px[i], c->py[i], c->pz[i]};
        if (p[0] == ctr[0] && p[1] == ctr[1] && p[2] == ctr[2]) {
            c->out[i] = 1;
            continue;
        }
        uint8_t res = 0;
        for (int64_t t = 0; t < c->n_tri; ++t) {
            const float *v0 = c->verts + 3 * (int64_t)c->tris[3 * t + 0];
            const float *v1 = c->verts + 3 * (int64_t)c->tris[3 * t + 1];
            const float *v2 = c->verts + 3 * (int64_t)c->tris[3 * t + 2];
            /* p - c = alpha (v0-c) + beta (v1-c) + gamma (v2-c); p is in the
             * closed cone when all three coefficients are >= 0, i.e. when the
             * three cone-side orientations are >= 0. */
            if (oracle_orient3d(ctr, v0, v1, p) < 0)
                continue;
            if (oracle_orient3d(ctr, v1, v2, p) < 0)
                continue;
            if (oracle_orient3d(ctr, v2, v0, p) < 0)
                continue;
            int s = oracle_orient3d(p, v0, v1, v2);
            res = s > 0 ? 1 : (s == 0 ? 2 : 0);
            break;
        }
        c->out[i] = res;
    }
}

void oracle_radial_inside(int64_t n, const float *px, const float *py, const float *pz,
                          const float center[3], const float *verts, int64_t n_tri,
                          const int32_t *tris, int n_threads, uint8_t *out)
{
    struct radial_ctx c = {px, py, pz, center, verts, tris, n_tri, out};
    oracle_parallel_for(n, n_threads, radial_range, &c);
}
