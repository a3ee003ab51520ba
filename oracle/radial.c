/*
 * Exact radial inside test with a direction index -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's checking legs use this
 * file; the GPU library never does, and the two share no code.
 * Build: gcc -O2 -ffp-contract=off (no fast-math), together with sal_oracle.c.
 *
 * What it decides.  Paper section 2.1.3 calls a point inside a closed surface
 * when the surface's solid angle seen from the point, over 4 pi, reaches the
 * threshold T in (0, 1).  For a closed surface that does not cross itself that
 * ratio is 1 inside and 0 outside, so the test is a point-in-polyhedron test.
 * Every synthetic compartment surface is star-shaped about a known centre c:
 * the cones (c, v0, v1, v2) of its triangles are all positively oriented and
 * cover the directions around c exactly once.  The ray from c through a point
 * p then meets the surface once, on the triangle whose cone holds p, and p is
 *   - inside when it lies strictly on c's side of that triangle's plane,
 *   - on the surface when it lies in that plane (section 2.1.3 counts such a
 *     point as enclosed, like the winding oracle),
 *   - outside otherwise.
 * All three decisions are exact orientation predicates on the float32
 * coordinates (oracle_orient3d); no solid angle is evaluated.  It is a second
 * inside test, independent of the Van Oosterom-Strackee sum, and cheap enough
 * to check every label of a full-size workload.
 *
 * When a point lies on the boundary plane of two or more cones, every cone that
 * holds it gives the same answer: the ray then meets the surface on the shared
 * edge or vertex, which lies in each of those triangles' planes.
 *
 * Finding the cone.  The directions around c are indexed by a cube map: a
 * direction d belongs to the cube face of the axis a with the largest |d_a|
 * (ties: the lower axis) and the sign of d_a, and maps to the point
 * (d_b / |d_a|, d_e / |d_a|) of [-1, 1]^2 on that face, (b, e) the two other
 * axes in cyclic order.  This central projection maps the cone of a triangle
 * to a flat triangle, so a cone is listed in every cell of a G x G grid on each
 * face that its projected bounding box (padded) meets.  A cone whose vertex
 * directions span 30 degrees or more is kept in a separate list instead: a
 * cone narrower than that which holds a direction of a face's pyramid (within
 * 54.8 degrees of the face's axis) has every vertex within 85 degrees of that
 * axis, so its projection onto the face is the flat triangle the grid uses.
 * A query tests the cones of its cell, then the wide list, and if neither
 * holds the point it tests every cone (counted in the index's fallback
 * counter): the index only saves work, it never decides an answer.
 *
 * Preconditions checked when an index is built: every cone is positively
 * oriented (exact), and the winding number of the surface at c, from the
 * oracle's solid-angle sum, is 1 (all cones positive and the sum 4 pi mean the
 * cones cover every direction once).
 */
#define _GNU_SOURCE
#include "sal_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define WIDE_COS 0.87 /* cones with two vertex directions >= ~29.5 deg apart are wide */
#define GRID_PAD 1e-7 /* padding of a projected box, in face coordinates */

struct oracle_radial {
    float c[3];
    float lo[3], hi[3]; /* box of the vertices */
    float *v;           /* [n_vert][3] */
    int32_t *t;         /* [n_tri][3] */
    int64_t n_vert, n_tri;
    int g;              /* cells per face side */
    int64_t *cell_start; /* [6 g g + 1] */
    int32_t *cell_cone;
    int32_t *wide;
    int64_t n_wide;
    int64_t fallbacks;  /* queries that needed the scan over every cone */
    int64_t undecided;  /* queries no cone holds (only if the preconditions fail) */
};

static int cell_of(double x, int g)
{
    double f = floor((x + 1.0) * 0.5 * (double)g);
    if (f < 0.0)
        return 0;
    if (f > (double)(g - 1))
        return g - 1;
    return (int)f;
}

/* Face and face coordinates of a nonzero direction q. */
static int face_coords(const double q[3], double *u, double *w)
{
    int a = 0;
    if (fabs(q[1]) > fabs(q[a]))
        a = 1;
    if (fabs(q[2]) > fabs(q[a]))
        a = 2;
    int b = (a + 1) % 3, e = (a + 2) % 3;
    double t = fabs(q[a]);
    *u = q[b] / t;
    *w = q[e] / t;
    return 2 * a + (q[a] > 0.0 ? 0 : 1);
}

static const float *vert(const struct oracle_radial *r, int64_t tri, int k)
{
    return r->v + 3 * (int64_t)r->t[3 * tri + k];
}

static int cone_is_wide(const double d[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) {
            double dot = d[i][0] * d[j][0] + d[i][1] * d[j][1] + d[i][2] * d[j][2];
            double ni = sqrt(d[i][0] * d[i][0] + d[i][1] * d[i][1] + d[i][2] * d[i][2]);
            double nj = sqrt(d[j][0] * d[j][0] + d[j][1] * d[j][1] + d[j][2] * d[j][2]);
            if (dot < WIDE_COS * ni * nj)
                return 1;
        }
    return 0;
}

/* Calls visit(ctx, cell) for every grid cell the narrow cone `tri` is listed in. */
static void cone_cells(const struct oracle_radial *r, const double d[3][3],
                       void (*visit)(void *, int64_t), void *ctx)
{
    int g = r->g;
    for (int f = 0; f < 6; ++f) {
        int a = f >> 1, b = (a + 1) % 3, e = (a + 2) % 3;
        double s = (f & 1) ? -1.0 : 1.0;
        double umin = 1e300, umax = -1e300, wmin = 1e300, wmax = -1e300;
        int ok = 1;
        for (int i = 0; i < 3 && ok; ++i) {
            double t = s * d[i][a];
            if (!(t > 0.0)) {
                ok = 0;
                break;
            }
            double u = d[i][b] / t, w = d[i][e] / t;
            umin = fmin(umin, u);
            umax = fmax(umax, u);
            wmin = fmin(wmin, w);
            wmax = fmax(wmax, w);
        }
        if (!ok)
            continue;
        umin -= GRID_PAD;
        wmin -= GRID_PAD;
        umax += GRID_PAD;
        wmax += GRID_PAD;
        if (umax < -1.0 || umin > 1.0 || wmax < -1.0 || wmin > 1.0)
            continue;
        int iu0 = cell_of(umin, g), iu1 = cell_of(umax, g);
        int iw0 = cell_of(wmin, g), iw1 = cell_of(wmax, g);
        for (int iu = iu0; iu <= iu1; ++iu)
            for (int iw = iw0; iw <= iw1; ++iw)
                visit(ctx, ((int64_t)f * g + iu) * g + iw);
    }
}

static void count_cell(void *ctx, int64_t cell)
{
    ((int64_t *)ctx)[cell + 1] += 1;
}

struct fill_ctx {
    int64_t *pos;
    int32_t *out;
    int32_t tri;
};

static void fill_cell(void *vctx, int64_t cell)
{
    struct fill_ctx *c = (struct fill_ctx *)vctx;
    c->out[c->pos[cell]++] = c->tri;
}

static void cone_dirs(const struct oracle_radial *r, int64_t tri, double d[3][3])
{
    for (int k = 0; k < 3; ++k) {
        const float *v = vert(r, tri, k);
        for (int i = 0; i < 3; ++i)
            d[k][i] = (double)v[i] - (double)r->c[i];
    }
}

void oracle_radial_free(struct oracle_radial *r)
{
    if (!r)
        return;
    free(r->v);
    free(r->t);
    free(r->cell_start);
    free(r->cell_cone);
    free(r->wide);
    free(r);
}

struct oracle_radial *oracle_radial_new(const float center[3], int64_t n_vert,
                                        const float *verts, int64_t n_tri,
                                        const int32_t *tris, int *status)
{
    *status = 3;
    if (n_vert < 4 || n_tri < 4 || n_tri > INT32_MAX)
        return NULL;
    struct oracle_radial *r = (struct oracle_radial *)calloc(1, sizeof(*r));
    if (!r)
        return NULL;
    memcpy(r->c, center, sizeof(r->c));
    r->n_vert = n_vert;
    r->n_tri = n_tri;
    r->v = (float *)malloc(sizeof(float) * 3 * n_vert);
    r->t = (int32_t *)malloc(sizeof(int32_t) * 3 * n_tri);
    if (!r->v || !r->t) {
        oracle_radial_free(r);
        return NULL;
    }
    memcpy(r->v, verts, sizeof(float) * 3 * n_vert);
    memcpy(r->t, tris, sizeof(int32_t) * 3 * n_tri);
    for (int64_t i = 0; i < 3 * n_tri; ++i)
        if (r->t[i] < 0 || r->t[i] >= n_vert) {
            oracle_radial_free(r);
            return NULL;
        }
    for (int i = 0; i < 3; ++i) {
        r->lo[i] = r->hi[i] = r->v[i];
        for (int64_t k = 1; k < n_vert; ++k) {
            float x = r->v[3 * k + i];
            r->lo[i] = x < r->lo[i] ? x : r->lo[i];
            r->hi[i] = x > r->hi[i] ? x : r->hi[i];
        }
    }

    /* every cone positively oriented, exactly */
    for (int64_t t = 0; t < n_tri; ++t)
        if (oracle_orient3d(r->c, vert(r, t, 0), vert(r, t, 1), vert(r, t, 2)) <= 0) {
            *status = 1;
            oracle_radial_free(r);
            return NULL;
        }
    /* the cones cover the directions once: winding number 1 at the centre */
    double wc = 0.0;
    float cx = r->c[0], cy = r->c[1], cz = r->c[2];
    oracle_winding(1, &cx, &cy, &cz, n_vert, r->v, n_tri, r->t, 1, &wc, NULL);
    if (!(fabs(wc - 1.0) < 0.25)) {
        *status = 2;
        oracle_radial_free(r);
        return NULL;
    }

    double gs = ceil(sqrt((double)n_tri / 6.0));
    r->g = gs < 1.0 ? 1 : (int)gs;
    int64_t n_cells = 6 * (int64_t)r->g * r->g;
    r->cell_start = (int64_t *)calloc(n_cells + 1, sizeof(int64_t));
    r->wide = (int32_t *)malloc(sizeof(int32_t) * n_tri);
    if (!r->cell_start || !r->wide) {
        oracle_radial_free(r);
        return NULL;
    }
    for (int64_t t = 0; t < n_tri; ++t) {
        double d[3][3];
        cone_dirs(r, t, d);
        if (cone_is_wide(d))
            r->wide[r->n_wide++] = (int32_t)t;
        else
            cone_cells(r, d, count_cell, r->cell_start);
    }
    for (int64_t c = 0; c < n_cells; ++c)
        r->cell_start[c + 1] += r->cell_start[c];
    r->cell_cone = (int32_t *)malloc(sizeof(int32_t) * (r->cell_start[n_cells] + 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * n_cells);
    if (!r->cell_cone || !pos) {
        free(pos);
        oracle_radial_free(r);
        return NULL;
    }
    memcpy(pos, r->cell_start, sizeof(int64_t) * n_cells);
    for (int64_t t = 0; t < n_tri; ++t) {
        double d[3][3];
        cone_dirs(r, t, d);
        if (cone_is_wide(d))
            continue;
        struct fill_ctx fc = {pos, r->cell_cone, (int32_t)t};
        cone_cells(r, d, fill_cell, &fc);
    }
    free(pos);
    *status = 0;
    return r;
}

/* 1 when p lies in the closed cone of triangle t. */
static int in_cone(const struct oracle_radial *r, int64_t t, const float p[3])
{
    const float *v0 = vert(r, t, 0), *v1 = vert(r, t, 1), *v2 = vert(r, t, 2);
    /* p - c = alpha (v0 - c) + beta (v1 - c) + gamma (v2 - c) with the cone
     * positively oriented: gamma >= 0 iff det[v0 - c, v1 - c, p - c] >= 0, and
     * likewise for alpha and beta. */
    return oracle_orient3d(r->c, v0, v1, p) >= 0 && oracle_orient3d(r->c, v1, v2, p) >= 0
        && oracle_orient3d(r->c, v2, v0, p) >= 0;
}

static uint8_t side_of(const struct oracle_radial *r, int64_t t, const float p[3])
{
    int s = oracle_orient3d(p, vert(r, t, 0), vert(r, t, 1), vert(r, t, 2));
    return s > 0 ? 1 : (s == 0 ? 2 : 0);
}

/* 0 outside, 1 inside, 2 on the surface, 3 no cone holds p. */
static uint8_t radial_one(struct oracle_radial *r, const float p[3])
{
    for (int i = 0; i < 3; ++i)
        if (p[i] < r->lo[i] || p[i] > r->hi[i])
            return 0; /* outside the vertices' box, hence outside the surface */
    double q[3] = {(double)p[0] - r->c[0], (double)p[1] - r->c[1], (double)p[2] - r->c[2]};
    if (q[0] == 0.0 && q[1] == 0.0 && q[2] == 0.0)
        return 1; /* the centre lies strictly inside every cone's face */
    double u, w;
    int f = face_coords(q, &u, &w);
    int64_t cell = ((int64_t)f * r->g + cell_of(u, r->g)) * r->g + cell_of(w, r->g);
    for (int64_t k = r->cell_start[cell]; k < r->cell_start[cell + 1]; ++k)
        if (in_cone(r, r->cell_cone[k], p))
            return side_of(r, r->cell_cone[k], p);
    for (int64_t k = 0; k < r->n_wide; ++k)
        if (in_cone(r, r->wide[k], p))
            return side_of(r, r->wide[k], p);
    __atomic_fetch_add(&r->fallbacks, 1, __ATOMIC_RELAXED);
    for (int64_t t = 0; t < r->n_tri; ++t)
        if (in_cone(r, t, p))
            return side_of(r, t, p);
    __atomic_fetch_add(&r->undecided, 1, __ATOMIC_RELAXED);
    return 3;
}

void oracle_radial_stats(const struct oracle_radial *r, int64_t out[6])
{
    out[0] = r->n_tri;
    out[1] = r->g;
    out[2] = r->cell_start[6 * (int64_t)r->g * r->g];
    out[3] = r->n_wide;
    out[4] = __atomic_load_n(&r->fallbacks, __ATOMIC_RELAXED);
    out[5] = __atomic_load_n(&r->undecided, __ATOMIC_RELAXED);
}

/* ----------------------------------------------------------- point sets */

struct query_ctx {
    struct oracle_radial *r;
    const float *px, *py, *pz;
    uint8_t *out;
};

static void query_range(void *vctx, int64_t b, int64_t e)
{
    struct query_ctx *c = (struct query_ctx *)vctx;
    for (int64_t i = b; i < e; ++i) {
        float p[3] = {c->px[i], c->py[i], c->pz[i]};
        c->out[i] = radial_one(c->r, p);
    }
}

void oracle_radial_query(struct oracle_radial *r, int64_t n, const float *px,
                         const float *py, const float *pz, int n_threads, uint8_t *out)
{
    struct query_ctx c = {r, px, py, pz, out};
    oracle_parallel_for(n, n_threads, query_range, &c);
}

/* Enclosure mask and label of one point (section 2.1: the later surface in
 * the list wins; label 0 when none encloses it).  *undecided counts the
 * surfaces for which no cone held the point. */
static int32_t label_one(struct oracle_radial *const *rs, const int32_t *surf_label, int n_surf,
                         const float p[3], uint64_t *mask, int64_t *undecided)
{
    int32_t label = 0;
    uint64_t m = 0;
    for (int s = 0; s < n_surf; ++s) {
        uint8_t res = radial_one(rs[s], p);
        if (res == 3)
            ++*undecided;
        if (res == 1 || res == 2) {
            label = surf_label[s];
            m |= (uint64_t)1 << (s & 63);
        }
    }
    *mask = m;
    return label;
}

struct label_ctx {
    struct oracle_radial *const *rs;
    const int32_t *surf_label;
    int n_surf;
    const float *px, *py, *pz;
    int32_t *labels;
    uint64_t *masks;
    int64_t undecided;
};

static void label_range(void *vctx, int64_t b, int64_t e)
{
    struct label_ctx *c = (struct label_ctx *)vctx;
    int64_t und = 0;
    for (int64_t i = b; i < e; ++i) {
        float p[3] = {c->px[i], c->py[i], c->pz[i]};
        uint64_t m;
        int32_t l = label_one(c->rs, c->surf_label, c->n_surf, p, &m, &und);
        if (c->labels)
            c->labels[i] = l;
        if (c->masks)
            c->masks[i] = m;
    }
    __atomic_fetch_add(&c->undecided, und, __ATOMIC_RELAXED);
}

int64_t oracle_radial_label(int64_t n, const float *px, const float *py, const float *pz,
                            int n_surf, struct oracle_radial *const *rs,
                            const int32_t *surf_label, int n_threads, int32_t *labels,
                            uint64_t *masks)
{
    if (masks && n_surf > 64)
        return -1;
    struct label_ctx c = {rs, surf_label, n_surf, px, py, pz, labels, masks, 0};
    oracle_parallel_for(n, n_threads, label_range, &c);
    return c.undecided;
}

/* ------------------------------------------- lattice and leaf-key checks
 * Kuhn lattice conventions (section 2.1.1, six tetrahedra per cube): cell
 * (i, j, k) of level l spans origin + h 2^-l [(i, j, k), (i, j, k) + 1]; the
 * permutation q (lexicographic over the axis orders) splits it into
 * 1 >= u[p0] >= u[p1] >= u[p2] >= 0, whose vertices are x0 = cell corner,
 * x1 = x0 + e_p0, x2 = x1 + e_p1, x3 = x0 + (1, 1, 1), and whose centroid has
 * local coordinates u[p0] = 3/4, u[p1] = 1/2, u[p2] = 1/4.  Keys are
 * level << 60 | q << 57 | i << 38 | j << 19 | k; level-0 points are numbered
 * ((k ny + j) nx + i) 6 + q.  Coordinates are formed in double as
 * origin + scale * t (product and sum rounded separately), then rounded once
 * to float32. */

static const int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static void centroid_f32(const double origin[3], double h, int level, int q, const int64_t cell[3],
                         float out[3])
{
    double c[3];
    c[PERM[q][0]] = 0.75;
    c[PERM[q][1]] = 0.5;
    c[PERM[q][2]] = 0.25;
    double hl = ldexp(h, -level);
    for (int a = 0; a < 3; ++a) {
        double t = (double)cell[a] + c[a];
        double prod = hl * t;
        out[a] = (float)(origin[a] + prod);
    }
}

/* The four vertices (lattice units times 2^level, integers) of a leaf. */
static void vertices_int(int q, const int64_t cell[3], int64_t x[4][3])
{
    for (int a = 0; a < 3; ++a)
        x[0][a] = cell[a];
    memcpy(x[1], x[0], sizeof(x[0]));
    x[1][PERM[q][0]] += 1;
    memcpy(x[2], x[1], sizeof(x[0]));
    x[2][PERM[q][1]] += 1;
    for (int a = 0; a < 3; ++a)
        x[3][a] = cell[a] + 1;
}

static void node_f32(const double origin[3], double h, int level, const int64_t x[3], float out[3])
{
    for (int a = 0; a < 3; ++a) {
        double u = ldexp((double)x[a], -level); /* exact */
        double prod = h * u;
        out[a] = (float)(origin[a] + prod);
    }
}

struct check_ctx {
    /* geometry */
    double origin[3], h;
    int64_t cells[3];
    int64_t first;
    const uint64_t *keys;
    int rule; /* 0: centroid label; 1: four-node label */
    /* surfaces */
    struct oracle_radial *const *rs;
    const int32_t *surf_label;
    int n_surf;
    /* results */
    const int32_t *got;
    int64_t mismatches, undecided;
    int64_t *bad;
    int64_t bad_cap, n_bad;
};

static void record(struct check_ctx *c, int64_t idx)
{
    int64_t slot = __atomic_fetch_add(&c->n_bad, 1, __ATOMIC_RELAXED);
    if (slot < c->bad_cap)
        c->bad[slot] = idx;
}

/* Label of the leaf (level, q, cell) under the chosen element rule. */
static int32_t leaf_label(struct check_ctx *c, int level, int q, const int64_t cell[3], int64_t *und)
{
    uint64_t m;
    if (c->rule == 0) {
        float p[3];
        centroid_f32(c->origin, c->h, level, q, cell, p);
        return label_one(c->rs, c->surf_label, c->n_surf, p, &m, und);
    }
    /* four-node rule: a leaf belongs to surface s when all four of its
     * vertices are enclosed by s; the later such surface wins */
    int64_t x[4][3];
    vertices_int(q, cell, x);
    uint64_t all = ~(uint64_t)0;
    for (int k = 0; k < 4; ++k) {
        float p[3];
        node_f32(c->origin, c->h, level, x[k], p);
        label_one(c->rs, c->surf_label, c->n_surf, p, &m, und);
        all &= m;
    }
    int32_t label = 0;
    for (int s = 0; s < c->n_surf; ++s)
        if ((all >> s) & 1)
            label = c->surf_label[s];
    return label;
}

static void lattice_range(void *vctx, int64_t b, int64_t e)
{
    struct check_ctx *c = (struct check_ctx *)vctx;
    int64_t mism = 0, und = 0;
    for (int64_t i = b; i < e; ++i) {
        int64_t t = c->first + i;
        int q = (int)(t % 6);
        int64_t cl = t / 6;
        int64_t cell[3] = {cl % c->cells[0], (cl / c->cells[0]) % c->cells[1],
                           cl / (c->cells[0] * c->cells[1])};
        int32_t want = leaf_label(c, 0, q, cell, &und);
        if (want != c->got[i]) {
            ++mism;
            record(c, t);
        }
    }
    __atomic_fetch_add(&c->mismatches, mism, __ATOMIC_RELAXED);
    __atomic_fetch_add(&c->undecided, und, __ATOMIC_RELAXED);
}

static void keys_range(void *vctx, int64_t b, int64_t e)
{
    struct check_ctx *c = (struct check_ctx *)vctx;
    const uint64_t m19 = (1u << 19) - 1;
    int64_t mism = 0, und = 0;
    for (int64_t i = b; i < e; ++i) {
        uint64_t key = c->keys[i];
        int level = (int)(key >> 60);
        int q = (int)((key >> 57) & 7);
        int64_t cell[3] = {(int64_t)((key >> 38) & m19), (int64_t)((key >> 19) & m19),
                           (int64_t)(key & m19)};
        int32_t want = q < 6 ? leaf_label(c, level, q, cell, &und) : INT32_MIN;
        if (want != c->got[i]) {
            ++mism;
            record(c, i);
        }
    }
    __atomic_fetch_add(&c->mismatches, mism, __ATOMIC_RELAXED);
    __atomic_fetch_add(&c->undecided, und, __ATOMIC_RELAXED);
}

int64_t oracle_radial_check_lattice(const double origin[3], double h, const int64_t cells[3],
                                    int64_t first, int64_t n, const int32_t *got, int n_surf,
                                    struct oracle_radial *const *rs, const int32_t *surf_label,
                                    int n_threads, int64_t *undecided, int64_t *bad,
                                    int64_t bad_cap)
{
    struct check_ctx c;
    memset(&c, 0, sizeof(c));
    memcpy(c.origin, origin, sizeof(c.origin));
    memcpy(c.cells, cells, sizeof(c.cells));
    c.h = h;
    c.first = first;
    c.rs = rs;
    c.surf_label = surf_label;
    c.n_surf = n_surf;
    c.got = got;
    c.bad = bad;
    c.bad_cap = bad_cap;
    oracle_parallel_for(n, n_threads, lattice_range, &c);
    *undecided = c.undecided;
    return c.mismatches;
}

int64_t oracle_radial_check_keys(const double origin[3], double h, int64_t n,
                                 const uint64_t *keys, const int32_t *got, int rule, int n_surf,
                                 struct oracle_radial *const *rs, const int32_t *surf_label,
                                 int n_threads, int64_t *undecided, int64_t *bad, int64_t bad_cap)
{
    struct check_ctx c;
    memset(&c, 0, sizeof(c));
    if (rule == 1 && n_surf > 64)
        return -1;
    memcpy(c.origin, origin, sizeof(c.origin));
    c.h = h;
    c.keys = keys;
    c.rule = rule;
    c.rs = rs;
    c.surf_label = surf_label;
    c.n_surf = n_surf;
    c.got = got;
    c.bad = bad;
    c.bad_cap = bad_cap;
    oracle_parallel_for(n, n_threads, keys_range, &c);
    *undecided = c.undecided;
    return c.mismatches;
}

/* Centroids (rule 0) or the four vertices (rule 1, [n][4] points) of leaves
 * given by key, as the checks above form them; for pinning those formulas. */
void oracle_leaf_points(const double origin[3], double h, int64_t n, const uint64_t *keys,
                        int rule, float *xyz)
{
    const uint64_t m19 = (1u << 19) - 1;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t key = keys[i];
        int level = (int)(key >> 60);
        int q = (int)((key >> 57) & 7) % 6;
        int64_t cell[3] = {(int64_t)((key >> 38) & m19), (int64_t)((key >> 19) & m19),
                           (int64_t)(key & m19)};
        if (rule == 0) {
            centroid_f32(origin, h, level, q, cell, xyz + 3 * i);
        } else {
            int64_t x[4][3];
            vertices_int(q, cell, x);
            for (int k = 0; k < 4; ++k)
                node_f32(origin, h, level, x[k], xyz + 3 * (4 * i + k));
        }
    }
}
