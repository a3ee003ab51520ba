/*
 * FP64 CPU oracle for solid-angle labeling.  TEST INFRASTRUCTURE ONLY: it is
 * called by the tests, by the smoke check and by the CPU-baseline timing of
 * the benchmark, never by the library it checks.  It shares no code with it.
 *
 * What it computes (paper section 2.1.3, Eq. 1, with the |r - r_i|^-3 kernel
 * that the printed equation omits): for a point p and a closed, outward
 * oriented triangulated surface S, the winding number
 *     w(p) = Omega_S(p) / (4 pi),
 * where Omega_S is the solid angle of S seen from p, summed exactly per flat
 * triangle with the Van Oosterom-Strackee formula.  A point is enclosed by S
 * when w >= T, or when it lies on S.  The compartment label is that of the
 * highest-priority enclosing surface (section 2.1: later in the list = higher
 * priority), else 0 (the bounding box).
 *
 * All inputs are float32 and promoted exactly to double.
 */
#ifndef SAL_ORACLE_H
#define SAL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Exact sign (-1, 0, +1) of det[v0 - p, v1 - p, v2 - p]. */
int oracle_orient3d_sign(const float p[3], const float v0[3], const float v1[3],
                         const float v2[3]);

/* The same sign as oracle_orient3d_sign, decided by the double value when a
 * static error bound certifies it and by the exact expansion otherwise. */
int oracle_orient3d(const float p[3], const float v0[3], const float v1[3],
                    const float v2[3]);

/* Runs fn(ctx, begin, end) over [0, n) split into one contiguous range per
 * host thread (n_threads <= 0: every core this process may use). */
typedef void (*oracle_range_fn)(void *ctx, int64_t begin, int64_t end);
void oracle_parallel_for(int64_t n, int n_threads, oracle_range_fn fn, void *ctx);

/* Exact sign of (b - a) x (c - a) projected on the plane that drops axis
 * `drop` (0 = x, 1 = y, 2 = z). */
int oracle_orient2d_sign(const float a[3], const float b[3], const float c[3],
                         int drop);

/* Solid angle (steradians) of triangle (v0, v1, v2) seen from p.  Sets
 * *on_tri = 1 (and returns 0) when p lies in the closed triangle. */
double oracle_tri_solid_angle(const float p[3], const float v0[3], const float v1[3],
                              const float v2[3], int *on_tri);

/* Winding numbers of one surface at n points.
 *   px, py, pz : float32 [n]           query points
 *   verts      : float32 [n_vert][3]   surface vertices
 *   tris       : int32 [n_tri][3]      counter-clockwise seen from outside
 *   w          : double [n] out        Omega / (4 pi), compensated sum
 *   on_surf    : uint8 [n] out or NULL 1 when p lies on the surface
 * Uses n_threads host threads over point blocks (<= 0: all online cores). */
void oracle_winding(int64_t n, const float *px, const float *py, const float *pz,
                    int64_t n_vert, const float *verts, int64_t n_tri,
                    const int32_t *tris, int n_threads, double *w, uint8_t *on_surf);

/* Labels for n points against n_surf surfaces listed outermost first.
 *   vert_off[s], tri_off[s] : offsets of surface s into verts / tris
 *   (the tris of surface s index its own vertex block)
 *   surf_label[s]           : compartment id of surface s
 *   labels                  : int32 [n] out
 *   w_out                   : double [n_surf][n] out, or NULL
 * Returns the number of (point, surface) pairs evaluated. */
int64_t oracle_label(int64_t n, const float *px, const float *py, const float *pz,
                     int n_surf, const int64_t *vert_off, const int64_t *tri_off,
                     const float *verts, const int32_t *tris,
                     const int32_t *surf_label, double threshold, int n_threads,
                     int32_t *labels, double *w_out);

/* Enclosure bits for n points: bit s of masks[i] is set when point i is
 * enclosed by surface s (w >= threshold, or on the surface), the same test
 * oracle_label applies.  At most 64 surfaces (else returns -1).  Returns
 * the number of (point, surface) pairs evaluated. */
int64_t oracle_enclosure(int64_t n, const float *px, const float *py, const float *pz,
                         int n_surf, const int64_t *vert_off, const int64_t *tri_off,
                         const float *verts, const int32_t *tris, double threshold,
                         int n_threads, uint64_t *masks);

/* Independent inside test for a surface that is star-shaped about `center`:
 * find the face whose cone (center, v0, v1, v2) holds p, then take the exact
 * side of p against that face.  Returns 1 inside, 0 outside, 2 on the surface.
 * Exact predicates only; O(n_tri) per point. */
void oracle_radial_inside(int64_t n, const float *px, const float *py, const float *pz,
                          const float center[3], const float *verts, int64_t n_tri,
                          const int32_t *tris, int n_threads, uint8_t *out);

/* ---------------------------------------------------------------------------
 * Exact radial inside test with a direction index (radial.c).  For a surface
 * star-shaped about `center` (every cone (center, v0, v1, v2) positively
 * oriented, winding number 1 at the centre): the triangle whose cone holds p
 * decides, by the exact side of p against its plane.  Query results: 0
 * outside, 1 inside, 2 on the surface, 3 no cone holds p (never, when the
 * preconditions hold).  O(1) expected per query.
 */
typedef struct oracle_radial oracle_radial;

/* Builds the index (the arrays are copied).  *status: 0 ok, 1 a cone is not
 * positively oriented, 2 the winding number at the centre is not 1, 3 bad
 * arguments or out of memory; NULL unless 0. */
oracle_radial *oracle_radial_new(const float center[3], int64_t n_vert, const float *verts,
                                 int64_t n_tri, const int32_t *tris, int *status);
void oracle_radial_free(oracle_radial *r);

/* out[6] = {triangles, grid cells per face side, grid entries, wide cones,
 * queries that fell back to scanning every cone, undecided queries}. */
void oracle_radial_stats(const oracle_radial *r, int64_t out[6]);

void oracle_radial_query(oracle_radial *r, int64_t n, const float *px, const float *py,
                         const float *pz, int n_threads, uint8_t *out);

/* Labels (the later enclosing or touching surface wins, else 0) and/or
 * enclosure masks (bit s: enclosed by surface s; at most 64 surfaces) of n
 * points; either output may be NULL.  Returns the number of undecided
 * (point, surface) queries, -1 on bad arguments. */
int64_t oracle_radial_label(int64_t n, const float *px, const float *py, const float *pz,
                            int n_surf, oracle_radial *const *rs, const int32_t *surf_label,
                            int n_threads, int32_t *labels, uint64_t *masks);

/* Checks the labels `got` [n] of the level-0 lattice points first .. first+n-1
 * (numbered ((k ny + j) nx + i) 6 + q; centroids formed here) against the
 * radial labels.  Returns the number of mismatches; the first bad_cap
 * mismatching point numbers go to bad (in no particular order).
 * *undecided counts undecided queries. */
int64_t oracle_radial_check_lattice(const double origin[3], double h, const int64_t cells[3],
                                    int64_t first, int64_t n, const int32_t *got, int n_surf,
                                    oracle_radial *const *rs, const int32_t *surf_label,
                                    int n_threads, int64_t *undecided, int64_t *bad,
                                    int64_t bad_cap);

/* The same for leaves given by key: rule 0 labels a leaf by its centroid,
 * rule 1 by its four vertices (the leaf belongs to a surface that encloses all
 * four; the later such surface wins).  bad receives positions into keys. */
int64_t oracle_radial_check_keys(const double origin[3], double h, int64_t n,
                                 const uint64_t *keys, const int32_t *got, int rule, int n_surf,
                                 oracle_radial *const *rs, const int32_t *surf_label,
                                 int n_threads, int64_t *undecided, int64_t *bad,
                                 int64_t bad_cap);

/* The points those checks form: centroids [n][3] (rule 0) or the four
 * vertices [n][4][3] (rule 1) of the leaves. */
void oracle_leaf_points(const double origin[3], double h, int64_t n, const uint64_t *keys,
                        int rule, float *xyz);

#ifdef __cplusplus
}
#endif
#endif
