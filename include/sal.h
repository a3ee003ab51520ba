/*
 * sal.h -- solid-angle labeling of tetrahedral lattices on AMD Instinct MI355X
 * (gfx950).  C ABI; every entry point is noexcept and reports through
 * sal_status.
 *
 * The method (paper "Multi-compartment human head modeling: generating
 * adaptive tetrahedral mesh with GPU acceleration", section 2.1):
 *   - a regular hexahedral lattice fills the domain; each hexahedron is split
 *     into tetrahedra (section 2.1.1; this library uses the six-tetrahedron
 *     Kuhn split of Fig. 1c);
 *   - a point is labeled with the solid-angle method (section 2.1.3, Eq. 1):
 *     s = Omega_S(p) / (4 pi) is the winding number of the closed surface S at
 *     p; p is enclosed by S when s >= T;
 *   - compartments are nested and, where boundaries intersect, the surface
 *     first in the hierarchy wins; a bounding box is the outermost compartment
 *     (section 2.1);
 *   - elements on a label boundary are refined 1 -> 8 (section 2.1.2, Fig. 2)
 *     and only the new elements are labeled again, recursively (section
 *     2.1.3 item 2, Fig. 3).
 *
 * Conventions shared by all calls
 *   - Coordinates are float32 millimetres; they are promoted exactly to double
 *     wherever double precision is used.
 *   - Surfaces are closed, consistently oriented triangle meshes whose
 *     triangles are counter-clockwise seen from outside (outward normals), so
 *     the winding number is +1 inside.  They are given outermost first: a
 *     later surface has higher priority ("first in the hierarchy") and wins
 *     where several enclose a point.  Label 0 is the bounding box.
 *   - A point lying exactly on a surface counts as enclosed by it.
 *   - Device pointers are HIP device (or managed) memory owned by the caller;
 *     they must stay valid until the work enqueued on the context's stream
 *     has finished.  Host pointers are read during the call only.
 *   - Work is enqueued on the context's stream and the call returns without
 *     waiting, unless a stats pointer is given (then the call synchronises
 *     the stream to fill it) or the entry point says otherwise.
 *   - On any error nothing further is enqueued; outputs are unspecified.
 *     sal_last_error_message() returns a thread-local description of the
 *     last error on the calling thread.
 *   - Nothing in this library runs on the CPU except argument checking,
 *     surface preprocessing (validation, triangle strips) and launch logic.
 */
#ifndef SAL_H
#define SAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SAL_ABI_VERSION 1

typedef enum sal_status {
    SAL_OK = 0,
    SAL_ERR_INVALID_ARG = 1,   /* NULL pointer, bad size, bad option, NaN input */
    SAL_ERR_NOT_CLOSED = 2,    /* a surface is not a closed 2-manifold */
    SAL_ERR_ORIENTATION = 3,   /* a surface encloses negative volume (inward faces) */
    SAL_ERR_OUT_OF_MEMORY = 4, /* device or host allocation failed */
    SAL_ERR_DEVICE = 5,        /* HIP runtime error, or no usable device */
    SAL_ERR_CAPACITY = 6,      /* a size limit of this library was exceeded */
    SAL_ERR_INTERNAL = 7
} sal_status;

/* Static description of a status code. */
const char *sal_status_string(sal_status s);
/* Description of the last failure on this thread (empty if none). */
const char *sal_last_error_message(void);
/* SAL_ABI_VERSION of the loaded library. */
int sal_abi_version(void);

/* Fault injection for tests of the error paths: with n > 0 the n-th device
 * allocation the library makes from now on (in any thread) fails once, as if
 * the device were out of memory (the call that makes it returns
 * SAL_ERR_OUT_OF_MEMORY, or SAL_ERR_DEVICE where a HIP error is reported as
 * such); n <= 0 disarms it.  Nothing else changes: no kernel sees it. */
void sal_debug_fail_allocation(int64_t n);

typedef struct sal_context sal_context;
typedef struct sal_surface_set sal_surface_set;
typedef struct sal_tet_mesh sal_tet_mesh;

/* ------------------------------------------------------------------ context
 * Binds a device and a stream.  hip_stream is a hipStream_t (NULL = the
 * default stream).  The context owns its scratch memory; it is not
 * thread-safe (use one context per host thread). */
sal_status sal_context_create(int device, void *hip_stream, sal_context **out);
sal_status sal_context_set_stream(sal_context *ctx, void *hip_stream);
void sal_context_destroy(sal_context *ctx); /* NULL-safe; waits for the stream */

/* ------------------------------------------------------------- surface set
 * The closed segmentation surfaces of section 2.1 in hierarchy order
 * (outermost first).  Creation validates every surface, builds triangle
 * strips and copies the geometry to the device (float32 strip records plus a
 * float64 copy for the recheck and plain-FP64 forms).  The set owns its
 * device memory and does not reference the descriptors after the call.
 *
 * Errors: SAL_ERR_INVALID_ARG (NULL, n_surfaces outside 1..64, an index out
 * of range, a repeated vertex in a triangle, a zero-area triangle, a
 * non-finite coordinate, label <= 0), SAL_ERR_NOT_CLOSED (some directed edge
 * appears twice or lacks its reverse), SAL_ERR_ORIENTATION (negative enclosed
 * volume and SAL_SURF_AUTO_ORIENT not set). */
typedef struct sal_surface_desc {
    int64_t n_vertices;
    const float *xyz;      /* host [n_vertices][3] */
    int64_t n_triangles;
    const int32_t *tri;    /* host [n_triangles][3], counter-clockwise from outside */
    int32_t label;         /* compartment id, > 0 */
} sal_surface_desc;

#define SAL_SURF_AUTO_ORIENT 1u /* reverse surfaces that enclose negative volume */

sal_status sal_surface_set_create(sal_context *ctx, const sal_surface_desc *surfaces,
                                  int32_t n_surfaces, uint32_t flags,
                                  sal_surface_set **out);
void sal_surface_set_destroy(sal_surface_set *set); /* NULL-safe */

typedef struct sal_surface_set_info {
    int32_t n_surfaces;
    int64_t n_triangles;   /* total over all surfaces */
    int64_t n_strips;      /* triangle strips built at creation */
    int64_t device_bytes;  /* device memory held by the set */
} sal_surface_set_info;
sal_status sal_surface_set_get_info(const sal_surface_set *set, sal_surface_set_info *info);

/* The validation and strip building of sal_surface_set_create (section
 * 2.1.3: closed, consistently oriented segmentation boundaries) on the host
 * alone, with no context and no device: the same checks and error statuses,
 * and with SAL_OK `info` (if not NULL) gets what the set would hold
 * (device_bytes: the bytes its creation would allocate).  Nothing is kept. */
sal_status sal_surface_set_check(const sal_surface_desc *surfaces, int32_t n_surfaces,
                                 uint32_t flags, sal_surface_set_info *info);

/* ----------------------------------------------------------------- labeling
 * Precision forms of the pair loop:
 *   SAL_PREC_FP64          every (point, triangle) solid angle in double, with
 *                          an exact sign of the triple product where double
 *                          cannot certify it ("plain FP64");
 *   SAL_PREC_FP32_RECHECK  solid angles in float32, summed per strip and
 *                          accumulated in double; a (point, surface) pair is
 *                          recomputed in the FP64 form when |w - T| <
 *                          recheck_band or when any of its triangles is
 *                          ill-conditioned in float32 (see kappa).  Labels are
 *                          those of the FP64 form. */
enum { SAL_PREC_FP64 = 0, SAL_PREC_FP32_RECHECK = 1 };
enum { SAL_WINDING_NONE = 0, SAL_WINDING_F32 = 1, SAL_WINDING_F64 = 2 };
/* Element rule of sal_refine_relabel (section 2.1.3):
 *   SAL_RULE_CENTROID    a tetrahedron takes the label of its centroid;
 *   SAL_RULE_FOUR_NODES  the solid-angle test is applied to the mesh nodes and
 *                        a tetrahedron takes the label of the highest-priority
 *                        surface enclosing all four of its nodes (else 0); a
 *                        split labels the six edge midpoints of the parent. */
enum { SAL_RULE_CENTROID = 0, SAL_RULE_FOUR_NODES = 1 };

typedef struct sal_label_options {
    int32_t precision;        /* SAL_PREC_* (default SAL_PREC_FP32_RECHECK) */
    int32_t winding_type;     /* SAL_WINDING_* for the optional winding output */
    double threshold;         /* T of section 2.1.3, in (0, 1); default 0.5 */
    double recheck_band;      /* default 1e-3 */
    double kappa;             /* float32 conditioning threshold; 0 = 2^-5 */
    int32_t points_per_lane;  /* 0 = tuned; else 1, 2 or 4 */
    int32_t block_waves;      /* 0 = tuned; else 1, 2, 4 or 8 wavefronts per block.
                                 Tuned: the first call for a (device, precision,
                                 log2 triangles, log2 points) times every candidate
                                 on up to 2^19 of the points against the leading
                                 strips of the set (about 32768 triangles, 8192 in
                                 the FP64 form), synchronising the stream, and
                                 caches the fastest for the process, and in the
                                 file named by SAL_TUNE_CACHE if set; SAL_TUNE=0
                                 disables tuning (1 point, 4 waves). */
    int32_t use_graph;        /* sal_label_batch: 1 = capture the launch sequence in a
                                 hipGraph and replay it while the same instances (same
                                 surface sets, pointers, sizes, options) come back;
                                 sal_refine_relabel: 1 = run the rounds as launches of
                                 one captured round graph (see there; centroid
                                 rule only: with the four-node rule it is
                                 rejected with SAL_ERR_INVALID_ARG);
                                 sal_label_points ignores it */
    int32_t element_rule;     /* SAL_RULE_* for sal_refine_relabel; fixed by a mesh's
                                 first labeling (a later call with another rule
                                 fails with SAL_ERR_INVALID_ARG) */
    int32_t cull_bounds;      /* 1: a wavefront whose points all lie strictly
                                 outside the bounding box of a surface's vertices
                                 (outside its convex hull: w = 0 exactly), or all
                                 inside a ball that the surface does not cross
                                 (w = that of the ball's centre, 0 or 1, found by
                                 the plain FP64 form on the set's first culling
                                 call),
                                 skips that surface; the labels are the same.
                                 Default 0.  sal_label_batch ignores it */
    int32_t reserved;
} sal_label_options;

/* Fills the defaults listed above. */
void sal_label_options_default(sal_label_options *opt);

typedef struct sal_label_stats {
    int64_t n_points;
    int64_t n_pairs;           /* n_points x total triangles (nominal) */
    int64_t n_recheck_points;  /* points with at least one FP64-rechecked surface */
    int64_t n_recheck_pairs;   /* (point, surface) pairs rechecked in FP64 */
    int64_t n_band_flags;      /* pairs flagged by |w - T| < recheck_band */
    int64_t n_cond_flags;      /* pairs flagged by an ill-conditioned triangle */
    int64_t n_exact_fallbacks; /* triangle evaluations that needed the exact sign */
    int64_t n_recheck_f64_terms; /* triangle terms of rechecked pairs evaluated in
                                    double (the others are certified float32) */
    float ms_pairloop;         /* device time of the pair loop */
    float ms_recheck;          /* device time of the FP64 recheck */
    float ms_total;            /* device time from the pair loop's start to the
                                  last kernel (launch-shape tuning excluded) */
    int32_t points_per_lane;   /* launch shape used (chosen by the tuner when 0 was asked) */
    int32_t block_waves;
    int64_t n_pairs_culled;    /* pairs of n_pairs skipped by cull_bounds (w = 0 exactly) */
} sal_label_stats;

/* Labels n_points points (section 2.1.3: s = Omega / 4 pi, enclosed when
 * s >= T or on the surface; section 2.1: the highest-priority enclosing
 * surface gives the label, else 0).
 *   x, y, z  device float32 [n_points] (SoA)
 *   labels   device int32 [n_points] out; -1 for a point with a non-finite
 *            coordinate
 *   winding  device [n_surfaces][n_points] of float (SAL_WINDING_F32) or
 *            double (SAL_WINDING_F64), or NULL; receives w per surface
 *   opt      NULL = defaults
 *   stats    NULL, or filled after synchronising the stream
 * n_points == 0 is valid and enqueues nothing. */
sal_status sal_label_points(sal_context *ctx, const sal_surface_set *set, int64_t n_points,
                            const float *x, const float *y, const float *z,
                            const sal_label_options *opt, int32_t *labels, void *winding,
                            sal_label_stats *stats);

/* sal_label_points for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (labels; winding numbers
 * to the float32 form's tolerance, bit for bit with the same launch shape)
 * as sal_label_points, but the call allocates nothing: its scratch (counters,
 * flag list, recheck buffers, about 38 MB) is one static device array per
 * GPU, held until the process ends, and its counters are cleared by a fill
 * kernel on every call.  Limits and differences:
 *   n_points  at most 1048576 per call (SAL_ERR_CAPACITY beyond; label larger
 *             sets in chunks);
 *   opt       cull_bounds must be 0 (SAL_ERR_INVALID_ARG); a launch shape left
 *             at 0 is not tuned but set to 1 point per lane and 4 wavefronts
 *             per workgroup (no trial launches, no synchronisation);
 *   stats     NULL for a call that must not synchronise (filled, as in
 *             sal_label_points, after synchronising the stream).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap in time on one GPU (other streams, other
 * contexts, other threads) race and must be serialised by the caller. */
sal_status sal_label_points_noalloc(sal_context *ctx, const sal_surface_set *set,
                                    int64_t n_points, const float *x, const float *y,
                                    const float *z, const sal_label_options *opt,
                                    int32_t *labels, void *winding, sal_label_stats *stats);

/* ----------------------------------------------------------- tetrahedral mesh
 * A Kuhn lattice (section 2.1.1) with nested red refinement (section 2.1.2).
 *
 * Geometry, in lattice units u = (x - origin) / h:
 *   level-0 cell (i, j, k) is the cube [i, i+1] x [j, j+1] x [k, k+1]; it
 *   holds six tetrahedra, one per permutation pi of the axes, q = index of pi
 *   in the lexicographic list (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y),
 *   (z,y,x):  {u : 1 >= f[pi0] >= f[pi1] >= f[pi2] >= 0}, f = u - cell;
 *   level l uses cells of edge h 2^-l; the 8 children of a tetrahedron are
 *   the level-(l+1) tetrahedra inside it (red refinement).
 * Centroid, computed in double and rounded once to float32:
 *   x_a = origin_a + (h 2^-l) (cell_a + c_a), c[pi0] = 3/4, c[pi1] = 1/2,
 *   c[pi2] = 1/4.
 * Key (uint64): l << 60 | q << 57 | i << 38 | j << 19 | k (i, j, k < 2^19).
 * Level-0 leaves are numbered ((k ny + j) nx + i) 6 + q.
 *
 * Creation allocates the level-0 leaves (unlabeled).  Limits: cells in
 * 1..2^19 >> 3 per axis (so three refinement levels fit in 19 bits), at most
 * 3 refinement levels. */
sal_status sal_tet_mesh_create_lattice(sal_context *ctx, const double origin[3], double h,
                                       const int32_t cells[3], sal_tet_mesh **out);
void sal_tet_mesh_destroy(sal_tet_mesh *mesh); /* NULL-safe */

typedef struct sal_refine_stats {
    int64_t n_leaves;     /* leaves after this round */
    int64_t n_boundary;   /* leaves split this round (0 for round 0) */
    int64_t n_labeled;    /* points labeled this round */
    int64_t n_pairs;      /* n_labeled x total triangles */
    int64_t n_recheck_pairs;
    /* device times; ms_label and ms_recheck leave out launch-shape tuning,
       ms_total (the whole round) includes it.  A round run as a replay of
       the captured round graph reports ms_total only. */
    float ms_mark, ms_compact, ms_split, ms_label, ms_recheck, ms_total;
    int32_t graph;        /* 0: host-driven round; 1: launch of the round graph
                             captured in this call; 2: launch of a round graph
                             kept from an earlier call */
    int32_t reserved;
} sal_refine_stats;

/* Section 2.1.3: labels every unlabeled leaf (round 0: the whole lattice),
 * then `rounds` times: marks each leaf sharing a 2-D part of a face with a
 * leaf of another label (faces on the domain boundary ignored), splits the
 * marked leaves 1 -> 8 and labels only the children.
 *   per_round  NULL, or [rounds + 1] filled after synchronising
 * Without opt->use_graph the host drives each round and synchronises the
 * stream once per round to size the new level.  With opt->use_graph, once
 * the lattice is labeled, the steps of one round (marking, compaction, split,
 * labeling of the children with the FP64 recheck, commit of their labels)
 * are captured once as a hipGraph that reads every size from device memory;
 * the graph is launched `rounds` times back to back, with one synchronisation
 * at the end, and kept on the mesh for later calls until a buffer it uses is
 * reallocated.  Every level and the scratch are reserved up front for twice
 * the current leaf count of new children per round, at least 2^20
 * (device memory of about 60 bytes per reserved child; the environment
 * variable SAL_REFINE_GRAPH_BUDGET overrides the count); a round that would not fit is
 * stopped on the device before it changes the mesh, and that round and the
 * rest run host-driven (growing the buffers).  A launch shape left at 0 is
 * resolved before capture.  The leaves, their order and labels are the same
 * in both modes.  Errors: SAL_ERR_CAPACITY when a leaf would exceed
 * refinement level 3. */
sal_status sal_refine_relabel(sal_context *ctx, sal_tet_mesh *mesh, const sal_surface_set *set,
                              int32_t rounds, const sal_label_options *opt,
                              sal_refine_stats *per_round);

/* Section 2.1.3 item 2 and Fig. 3: the recursion repeated until the
 * boundary between compartments no longer changes.  Labels every unlabeled
 * leaf (as sal_refine_relabel's round 0), then repeats steps: mark each leaf
 * sharing a 2-D part of a face with a leaf of another label, split the
 * marked leaves that are coarser than `finest_level` 1 -> 8 and label only
 * the children (or, under the four-node rule, only the new nodes).  The
 * recursion has converged with the first step that finds no such leaf: then
 * every leaf on a label boundary is at `finest_level` and another step would
 * change nothing.  It ends there, or after `max_steps` steps that split.
 *   finest_level  0..3 (refinement levels above the lattice)
 *   per_step      NULL, or [max_steps + 1]: entry 0 the lattice labeling,
 *                 entry s the s-th step that split (filled after
 *                 synchronising); the final step that splits nothing is
 *                 not recorded
 *   n_steps       NULL, or receives the number of steps that split
 *   converged     NULL, or receives 1 when the recursion converged, 0 when
 *                 max_steps steps all split
 * The rounds are host-driven (opt->use_graph must be 0).  The element rule
 * and the leaves' storage are those of sal_refine_relabel; a mesh may mix
 * calls of both. */
sal_status sal_refine_relabel_converge(sal_context *ctx, sal_tet_mesh *mesh,
                                       const sal_surface_set *set, int32_t finest_level,
                                       int32_t max_steps, const sal_label_options *opt,
                                       sal_refine_stats *per_step, int32_t *n_steps,
                                       int32_t *converged);

/* Number of leaves and the deepest level present. */
sal_status sal_tet_mesh_size(const sal_tet_mesh *mesh, int64_t *n_leaves, int32_t *max_level);

/* Copies the leaves, ordered by level then by position within the level,
 * into caller device buffers [n_leaves] (each may be NULL):
 *   keys (uint64), labels (int32; -2 for a leaf not labeled yet),
 *   cx, cy, cz (float32 centroids). */
sal_status sal_tet_mesh_export(sal_context *ctx, const sal_tet_mesh *mesh, uint64_t *keys,
                               int32_t *labels, float *cx, float *cy, float *cz);

/* Checkpoint / resume: rebuilds the leaves of a refined mesh from the keys
 * and labels sal_tet_mesh_export wrote (in any order), so that refinement can
 * continue in another process or after the original mesh is gone.  The mesh
 * must come fresh from sal_tet_mesh_create_lattice with the same origin, h
 * and cells.
 *   keys, labels  device [n_leaves] (caller-owned; copied, not kept)
 * The leaves must be exactly a nested red refinement of the lattice: every
 * key inside the lattice and at most 3 levels deep, no key twice, every
 * refined tetrahedron with all 8 children present (as leaves or refined), no
 * tetrahedron both a leaf and refined, every lattice tetrahedron covered;
 * labels >= 0.  Otherwise SAL_ERR_INVALID_ARG and the mesh is unchanged.
 * The imported mesh is labeled under the centroid rule (the four-node rule's
 * node table is not part of a checkpoint).  The layout of the levels may
 * differ from the exporting mesh's; the leaves, their labels and every later
 * refinement are the same. */
sal_status sal_tet_mesh_import(sal_context *ctx, sal_tet_mesh *mesh, int64_t n_leaves,
                               const uint64_t *keys, const int32_t *labels);

/* ---------------------------------------------- conforming transition mesh */
typedef struct sal_conform_info {
    int64_t n_tets;           /* tetrahedra of the conforming mesh */
    int64_t n_nodes;          /* distinct nodes */
    int64_t n_leaves;         /* leaves after the closure */
    int64_t n_by_pieces[4];   /* leaves cut into 1, 2, 3 and 4 tetrahedra */
    int32_t closure_rounds;   /* rounds of 1 -> 8 closure splits */
    int32_t reserved;
} sal_conform_info;

/* Section 2.1.2 (Fig. 2c-e): removes the hanging nodes that refinement left
 * between leaves of different levels.  An edge of a leaf is hanging when its
 * midpoint is a vertex of another leaf.  A leaf whose hanging edges are one
 * edge, two edges of one face or the three edges of one face is cut into 2, 3
 * or 4 tetrahedra (the quadrilateral of the two-edge case along its diagonal
 * through the smallest node key, so that both sides of the face agree).  A
 * leaf with any other pattern, or with a node at a quarter point of an edge
 * (a neighbour two levels finer), is split 1 -> 8, its children keeping its
 * label, and the patterns are found again until none is left (closure).  The
 * result is stored on the mesh: tetrahedra over numbered nodes, each with the
 * label of the leaf it comes from.  Nodes are the points of the level-3 grid
 * (spacing h / 8), numbered in ascending key order, key = (i << 42) |
 * (j << 21) | k with (i, j, k) the level-3 grid coordinates.  Tetrahedra are
 * positively oriented; their order is that of their leaves as
 * sal_tet_mesh_export lists them.  After this call the mesh cannot be refined
 * again (SAL_ERR_INVALID_ARG), nor made conforming twice.
 *   info  NULL, or filled after synchronising
 * Errors: SAL_ERR_CAPACITY above 2^31 tetrahedron corners; SAL_ERR_OUT_OF_MEMORY.
 * After such an error the mesh is not conforming, but its leaf set may already
 * hold closure splits (children with their parent's label); calling this
 * function again resumes the closure from there. */
sal_status sal_tet_mesh_conform(sal_context *ctx, sal_tet_mesh *mesh, sal_conform_info *info);

/* Copies the conforming mesh into caller device buffers (each may be NULL):
 *   tets [n_tets][4] int32 node ids, labels [n_tets] int32,
 *   xyz [n_nodes][3] float32 node coordinates (origin + key coordinate x h/8,
 *   rounded once from double), node_keys [n_nodes] int64.
 * Errors: SAL_ERR_INVALID_ARG before sal_tet_mesh_conform. */
sal_status sal_tet_mesh_export_conforming(sal_context *ctx, const sal_tet_mesh *mesh, int32_t *tets,
                                          int32_t *labels, float *xyz, int64_t *node_keys);

/* ------------------------------------------------------- Taubin smoothing */
typedef struct sal_smooth_params {
    double lambda;            /* forward step, 0 < lambda < 1 (default 0.4) */
    double mu;                /* backward step, 0 < mu < 1 (default 0.4) */
    double xi_surface;        /* stopping ratio of the surface phase (0.1) */
    double xi_volume;         /* stopping ratio of the volume phase (0.9) */
    int32_t max_iter_surface; /* iteration caps (100 each); 0 skips a phase */
    int32_t max_iter_volume;
} sal_smooth_params;

void sal_smooth_params_default(sal_smooth_params *p); /* the values of section 2.6.1 */

typedef struct sal_smooth_info {
    int64_t n_edges;          /* edges of the conforming mesh */
    int64_t n_surface_edges;  /* edges whose tetrahedra carry two or more labels */
    int64_t n_surface_nodes;  /* nodes moved by the surface phase */
    int64_t n_volume_nodes;   /* nodes moved by the volume phase */
    int32_t iters_surface, iters_volume;
    double ratio_surface;     /* stopping ratio of each phase's last iteration */
    double ratio_volume;
    float ms_build;           /* edge graph and node classes (first call only) */
    float ms_surface, ms_volume;
    int32_t reserved;
    int64_t n_entries_surface; /* neighbour entries one half step reads */
    int64_t n_entries_volume;  /* (interface rows read whole in the surface phase) */
} sal_smooth_info;

/* Section 2.2.1: Taubin smoothing of the conforming mesh's nodes, in place.
 * One iteration is a forward and a backward half step over the nodes a
 * phase moves,
 *   x_i <- x_i + lambda (m_i - x_i),   then   x_i <- x_i - mu (m_i - x_i),
 * m_i the mean position over node i and its neighbours (each half step reads
 * the positions of the previous one).  The surface phase moves the nodes on
 * an interface (an edge joining tetrahedra of two or more labels) along
 * interface edges only; the volume phase then moves every other node along
 * all edges.  Nodes on a face of the lattice box never move.  A phase stops
 * after the first iteration k with ||x(k+1/2) - x(k)|| / ||x(0)|| <= xi
 * (norms over the nodes it moves, x(0) their positions at the phase start)
 * or after its iteration cap; a phase with no node to move runs no
 * iteration.  Positions are kept in float32 and each half
 * step is computed in double.  The edge graph is built on the first call and
 * kept on the mesh; later calls smooth the current positions again.
 *   params  NULL for the defaults;  info  NULL, or filled
 * Errors: SAL_ERR_INVALID_ARG before sal_tet_mesh_conform or for parameters
 * outside (0, 1); SAL_ERR_CAPACITY above 2^28 nodes, 357M tetrahedra or
 * labels outside [-1, 254]. */
sal_status sal_tet_mesh_smooth(sal_context *ctx, sal_tet_mesh *mesh, const sal_smooth_params *params,
                               sal_smooth_info *info);

/* -------------------------------------------------------------- inflation */
typedef struct sal_inflate_info {
    int64_t n_candidates;     /* interface nodes off the lattice box */
    int64_t n_moved;          /* of those, nodes with an edge crossing a triangle */
    int64_t n_edges_tested;   /* their incident edges (directed) */
    int64_t n_triangle_tests; /* segment-triangle tests made */
    int64_t n_triangles;      /* triangles of the surface set */
    int64_t n_bin_items;      /* (bin, triangle) entries of the lattice binning */
    float ms_prepare;         /* triangles, binning, edge graph if not built yet */
    float ms_inflate;         /* the move */
} sal_inflate_info;

/* Section 2.2.2: moves every interface node of the conforming mesh (an edge
 * of the node joins tetrahedra of two or more labels; nodes on the lattice
 * box excepted) toward the surfaces.  Each incident edge x_i -> x_j is
 * tested against the triangles of `set` (segment-triangle crossing, bounds
 * included, in double); over the edges, the crossing nearest to x_i along its
 * edge, at distance d, wins (equal distances: the neighbour with the smaller
 * node key), and x_i <- x_i + zeta d (x_j - x_i) / |x_j - x_i|.  Nodes whose
 * edges cross no triangle stay; all moves read the positions from before the
 * call.  Positions are kept in float32.  The surface set is the one the mesh
 * was labeled with, or any other on the same device.
 *   zeta  in [0, 1) (section 2.6.1 uses 0.05);  info  NULL, or filled
 * Errors: SAL_ERR_INVALID_ARG before sal_tet_mesh_conform or for zeta
 * outside [0, 1); SAL_ERR_CAPACITY as for sal_tet_mesh_smooth. */
sal_status sal_tet_mesh_inflate(sal_context *ctx, sal_tet_mesh *mesh, const sal_surface_set *set,
                                double zeta, sal_inflate_info *info);

/* ------------------------------------------------------------ batched form
 * Many independent labeling problems in one persistent launch: the work is
 * cut into (instance, point block, surface, triangle range) items ordered by
 * cost, pulled by resident workgroups from a device counter; partial winding
 * sums are reduced per (point, surface) in a fixed order; one FP64 recheck
 * pass serves all instances.  With precision SAL_PREC_FP64 the items run the
 * plain FP64 walk (exact sign where double cannot certify it, points on a
 * surface enclosed) and there is no recheck.  Labels equal those of
 * sal_label_points on each instance.  Each instance's arrays follow the rules of sal_label_points.
 *   per_instance  NULL, or [n_inst] stats filled after synchronising */
typedef struct sal_instance {
    const sal_surface_set *surfaces;
    int64_t n_points;
    const float *x, *y, *z; /* device float32 [n_points] */
    int32_t *labels;        /* device int32 [n_points] out */
} sal_instance;

sal_status sal_label_batch(sal_context *ctx, const sal_instance *inst, int32_t n_inst,
                           const sal_label_options *opt, sal_label_stats *per_instance);

#ifdef __cplusplus
}
#endif
#endif /* SAL_H */
