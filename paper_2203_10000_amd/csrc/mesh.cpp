// Tetrahedral mesh: Kuhn lattice creation, recursive refine-and-relabel
// rounds (paper section 2.1.3 item 2), export of the leaves.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mesh_internal.h"
#include "post_internal.h"
#include "runtime.h"

namespace sal {

// Children tables from the parent rule: the level-(l+1) tetrahedron (code,
// q') in sub-cell `code` lies in the parent q when sorting U_a = 4 d_a + w_a
// (w = 3, 2, 1 along q''s permutation) in decreasing order gives q's
// permutation.
static ChildTables make_child_tables() {
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    ChildTables T;
    std::memset(&T, -1, sizeof(T));
    int count[6] = {0, 0, 0, 0, 0, 0};
    for (int code = 0; code < 8; ++code) {
        for (int cq = 0; cq < 6; ++cq) {
            int w[3], U[3];
            w[perm[cq][0]] = 3;
            w[perm[cq][1]] = 2;
            w[perm[cq][2]] = 1;
            for (int a = 0; a < 3; ++a) U[a] = 4 * ((code >> a) & 1) + w[a];
            int pq = -1;
            for (int q = 0; q < 6; ++q)
                if (U[perm[q][0]] > U[perm[q][1]] && U[perm[q][1]] > U[perm[q][2]]) pq = q;
            const int r = count[pq]++;
            T.list[pq][r][0] = (int8_t)code;
            T.list[pq][r][1] = (int8_t)cq;
            T.rank[pq][code][cq] = (int8_t)r;
        }
    }
    return T;
}

}  // namespace sal

struct sal_tet_mesh {
    int device = 0;
    sal::LatticeGeom g{};
    sal::ChildTables T{};
    int64_t n[sal::kMaxLevels + 1] = {};
    int64_t cap[sal::kMaxLevels + 1] = {};
    uint64_t *key[sal::kMaxLevels + 1] = {};
    int32_t *label[sal::kMaxLevels + 1] = {};
    int32_t *child[sal::kMaxLevels + 1] = {};
    uint8_t *flag[sal::kMaxLevels + 1] = {};
    int max_level = 0;
    bool labeled0 = false;
    // conforming mesh (sal_tet_mesh_conform); no refinement after it
    bool conformed = false;
    int64_t conf_tets = 0, conf_nodes = 0;
    int32_t *conf_ids = nullptr;     // [conf_tets][4] node ids
    int32_t *conf_labels = nullptr;  // [conf_tets]
    int64_t *conf_keys = nullptr;    // [conf_nodes] node keys, ascending
    float *conf_xyz = nullptr;       // [conf_nodes][3]
    sal::SmoothCache *smooth = nullptr;   // edge graph for smoothing
    int64_t n_leaves = 0;
    // scratch
    float *cen[3] = {};
    int64_t cen_cap = 0;
    int32_t *list = nullptr;
    int64_t list_cap = 0;
    int64_t *blocks = nullptr;
    int64_t blocks_cap = 0;
    int64_t *totals = nullptr;   // kMaxLevels + 1 counts
    hipEvent_t ev[16] = {};
    // captured refine round
    int32_t *lab_scratch = nullptr;
    int64_t lab_cap = 0;
    sal::RoundState *rs = nullptr;
    hipGraphExec_t round_graph = nullptr;
    uint64_t round_key = 0;
    std::vector<uint64_t> round_fields;   // the fields hashed into round_key
    // four-node rule: level-0 node grid masks, per-leaf vertex masks of
    // levels >= 1, masks of the labeled midpoints
    int rule = -1;   // element rule fixed by the first labeling
    unsigned long long *node0 = nullptr;
    unsigned long long *vmask[sal::kMaxLevels + 1] = {};
    unsigned long long *mid_masks = nullptr;
    int64_t mid_cap = 0;
    // midpoints of a split level and the node table (each node labeled once)
    float *mid_xyz[3] = {};
    int64_t mid_xyz_cap = 0;
    uint64_t *mid_key = nullptr;
    int64_t mid_key_cap = 0;
    int64_t *mid_slot = nullptr;
    int64_t mid_slot_cap = 0;
    int32_t *new_list = nullptr;
    int64_t new_list_cap = 0;
    unsigned long long *new_masks = nullptr;
    int64_t new_masks_cap = 0;
    unsigned long long *n_new = nullptr;
    unsigned long long *tkeys = nullptr, *tmasks = nullptr;
    int64_t tcap = 0, tused = 0;   // tused: upper bound of the entries
};

namespace sal {
namespace {

sal::LevelPtrs ptrs(const sal_tet_mesh *m) {
    LevelPtrs L{};   // n_dev stays null: host-driven sizes
    for (int l = 0; l <= kMaxLevels; ++l) {
        L.key[l] = m->key[l];
        L.label[l] = m->label[l];
        L.child[l] = m->child[l];
        L.flag[l] = m->flag[l];
        L.n[l] = m->n[l];
    }
    return L;
}

template <typename T>
sal_status grow(T **p, int64_t old_n, int64_t new_cap, hipStream_t s) {
    T *q = nullptr;
    SAL_HIP(dev_malloc((void **)&q, (size_t)new_cap * sizeof(T)));
    if (*p && old_n > 0)
        SAL_HIP(hipMemcpyAsync(q, *p, (size_t)old_n * sizeof(T), hipMemcpyDeviceToDevice, s));
    if (*p) {
        SAL_HIP(hipStreamSynchronize(s));
        SAL_HIP(hipFree(*p));
    }
    *p = q;
    return SAL_OK;
}

sal_status ensure_level(sal_tet_mesh *m, int l, int64_t need, hipStream_t s) {
    if (need <= m->cap[l]) return SAL_OK;
    int64_t cap = m->cap[l] + m->cap[l] / 2;
    if (cap < need) cap = need;
    sal_status st;
    if (l > 0 && (st = grow(&m->key[l], m->n[l], cap, s)) != SAL_OK) return st;
    if ((st = grow(&m->label[l], m->n[l], cap, s)) != SAL_OK) return st;
    if ((st = grow(&m->child[l], m->n[l], cap, s)) != SAL_OK) return st;
    if ((st = grow(&m->flag[l], m->n[l], cap, s)) != SAL_OK) return st;
    if (l > 0 && m->rule == SAL_RULE_FOUR_NODES &&
        (st = grow(&m->vmask[l], 4 * m->n[l], 4 * cap, s)) != SAL_OK)
        return st;
    m->cap[l] = cap;
    return SAL_OK;
}

template <typename T>
sal_status ensure_buf(T **p, int64_t *cap, int64_t need, hipStream_t s) {
    if (need <= *cap) return SAL_OK;
    const int64_t c = need + need / 4 + 1024;
    sal_status st = grow(p, 0, c, s);
    if (st == SAL_OK) *cap = c;
    return st;
}

sal_status ensure_centroids(sal_tet_mesh *m, int64_t need, hipStream_t s) {
    if (need <= m->cen_cap) return SAL_OK;
    const int64_t c = need + need / 4 + 1024;
    for (int a = 0; a < 3; ++a) {
        int64_t dummy = 0;
        sal_status st = grow(&m->cen[a], 0, c, s);
        (void)dummy;
        if (st != SAL_OK) return st;
    }
    m->cen_cap = c;
    return SAL_OK;
}

sal_status compact(sal_tet_mesh *m, const CompactSrc &src, int64_t n, int32_t *out, int64_t *total,
                   hipStream_t s) {
    sal_status st = ensure_buf(&m->blocks, &m->blocks_cap, compact_blocks(n) + 1, s);
    if (st != SAL_OK) return st;
    SAL_HIP(launch_compact(src, n, m->blocks, total, out, s));
    return SAL_OK;
}

// Labels n points whose centroids sit in the scratch into `labels`; records
// ev_start after any launch-shape tuning and ev_mid after the pair loop
// (before the recheck).
sal_status label_scratch(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set, int64_t n,
                         const sal_label_options &opt, int32_t *labels, hipEvent_t ev_start,
                         hipEvent_t ev_mid, unsigned long long *masks = nullptr) {
    if (n <= 0) return SAL_OK;
    if (opt.precision == SAL_PREC_FP32_RECHECK) {
        sal_status st = ensure_flag_capacity(ctx, n);
        if (st != SAL_OK) return st;
    }
    SAL_HIP(launch_fill_u64(ctx->counters + kCntFlagged, 0ull, 1, ctx->stream));
    return enqueue_label(ctx, set, n, m->cen[0], m->cen[1], m->cen[2], opt, labels, nullptr,
                         ev_start, ev_mid, nullptr, masks);
}

// As label_scratch, for a point count held on the device (capacity n_cap).
sal_status label_scratch_dev(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set,
                             int64_t n_cap, const unsigned long long *n_dev,
                             const sal_label_options &opt_in, int32_t *labels, hipEvent_t ev_start,
                             hipEvent_t ev_mid, unsigned long long *masks) {
    if (n_cap <= 0) return SAL_OK;
    if (opt_in.precision == SAL_PREC_FP32_RECHECK) {
        sal_status st = ensure_flag_capacity(ctx, n_cap);
        if (st != SAL_OK) return st;
    }
    SAL_HIP(launch_fill_u64(ctx->counters + kCntFlagged, 0ull, 1, ctx->stream));
    sal_label_options opt = opt_in;
    sal_status st = tune_launch(ctx, set, n_cap, m->cen[0], m->cen[1], m->cen[2], labels, &opt);
    if (st != SAL_OK) return st;
    SAL_HIP(hipEventRecord(ev_start, ctx->stream));
    return enqueue_label_on(ctx, set, n_cap, (const int64_t *)n_dev, m->cen[0], m->cen[1],
                            m->cen[2], opt, labels, nullptr, ev_mid, ctx->stream, masks);
}

// Room in the node table for `more` entries (kept at most half full; a
// larger table is filled by re-inserting the old entries).
sal_status ensure_node_table(sal_tet_mesh *m, int64_t more, hipStream_t s) {
    const int64_t need = 2 * (m->tused + more);
    if (need <= m->tcap) return SAL_OK;
    int64_t cap = 1 << 16;
    while (cap < need) cap <<= 1;
    unsigned long long *k = nullptr, *v = nullptr;
    SAL_HIP(dev_malloc((void **)&k, (size_t)cap * sizeof(unsigned long long)));
    const hipError_t ev = dev_malloc((void **)&v, (size_t)cap * sizeof(unsigned long long));
    if (ev != hipSuccess) {
        (void)hipFree(k);
        return hip_error(ev, "hipMalloc(node table)");
    }
    SAL_HIP(launch_fill_u64(k, ~0ull, cap, s));
    if (m->tkeys) {
        SAL_HIP(launch_node_rehash(m->tkeys, m->tmasks, m->tcap, k, v, cap, s));
        SAL_HIP(hipStreamSynchronize(s));
        SAL_HIP(hipFree(m->tkeys));
        SAL_HIP(hipFree(m->tmasks));
    }
    m->tkeys = k;
    m->tmasks = v;
    m->tcap = cap;
    return SAL_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0f;
    return ms;
}

// One host-driven round (section 2.1.3 item 2): mark, compact, then for each
// level, deepest first, split the marked leaves and label their children.
// Marked leaves at level `finest` or deeper are left as they are (the
// converging recursion); without a limit a marked level-3 leaf is an error.
// Synchronises once to size the new level (and once per level for timing).
sal_status eager_round(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set,
                       const sal_label_options &opt, sal_refine_stats *out,
                       int finest = kMaxLevels + 1, int64_t *n_split_out = nullptr) {
    hipStream_t s = ctx->stream;
    sal_status st;
    const int top = m->max_level;
    int64_t total_entries = 0;
    for (int l = 0; l <= top; ++l) total_entries += m->n[l];
    if ((st = ensure_buf(&m->list, &m->list_cap, total_entries, s)) != SAL_OK) return st;
    SAL_HIP(launch_fill_u64(ctx->counters, 0ull, kNumCounters, s));
    SAL_HIP(hipEventRecord(m->ev[2], s));
    for (int l = 0; l <= top; ++l) SAL_HIP(launch_fill_u8(m->flag[l], 0, m->n[l], s));
    LevelPtrs L = ptrs(m);
    for (int l = 0; l <= top; ++l) SAL_HIP(launch_mark(L, m->g, m->T, l, s));
    SAL_HIP(hipEventRecord(m->ev[3], s));
    int64_t off[kMaxLevels + 2] = {0};
    for (int l = 0; l <= top; ++l) {
        off[l + 1] = off[l] + m->n[l];
        CompactSrc src{m->flag[l], nullptr};
        if ((st = compact(m, src, m->n[l], m->list + off[l], m->totals + l, s)) != SAL_OK) return st;
    }
    SAL_HIP(hipEventRecord(m->ev[4], s));
    int64_t count[kMaxLevels + 1] = {0};
    SAL_HIP(hipMemcpyAsync(count, m->totals, sizeof(int64_t) * (top + 1), hipMemcpyDeviceToHost, s));
    SAL_HIP(hipStreamSynchronize(s));
    for (int l = finest; l <= top; ++l) count[l] = 0;
    if (top == kMaxLevels && count[top] > 0)
        return set_error(SAL_ERR_CAPACITY, "refinement beyond level 3");
    int64_t n_split = 0, n_label = 0;
    float ms_split = 0.0f, ms_label = 0.0f, ms_recheck = 0.0f;
    // Every buffer the round needs is allocated before the first split, so a
    // round that runs out of device memory fails with the mesh unchanged
    // (the in-loop ensure calls below then find the room already there).
    {
        const bool nodes = m->rule == SAL_RULE_FOUR_NODES;
        int64_t pts_max = 0, pts_sum = 0;
        for (int l = top; l >= 0; --l) {
            if (count[l] == 0) continue;
            const int64_t n_pts = nodes ? 6 * count[l] : 8 * count[l];
            pts_max = std::max(pts_max, n_pts);
            pts_sum += n_pts;
            if ((st = ensure_level(m, l + 1, m->n[l + 1] + 8 * count[l], s)) != SAL_OK) return st;
        }
        if (pts_max > 0) {
            if ((st = ensure_centroids(m, pts_max, s)) != SAL_OK) return st;
            if (opt.precision == SAL_PREC_FP32_RECHECK &&
                (st = ensure_flag_capacity(ctx, pts_max)) != SAL_OK)
                return st;
            if (nodes) {
                int64_t c3 = m->mid_xyz_cap;
                for (int a = 0; a < 3; ++a) {
                    c3 = m->mid_xyz_cap;
                    if ((st = ensure_buf(&m->mid_xyz[a], &c3, pts_max, s)) != SAL_OK) return st;
                }
                m->mid_xyz_cap = c3;
                if ((st = ensure_buf(&m->lab_scratch, &m->lab_cap, pts_max, s)) != SAL_OK ||
                    (st = ensure_buf(&m->mid_masks, &m->mid_cap, pts_max, s)) != SAL_OK ||
                    (st = ensure_buf(&m->mid_key, &m->mid_key_cap, pts_max, s)) != SAL_OK ||
                    (st = ensure_buf(&m->mid_slot, &m->mid_slot_cap, pts_max, s)) != SAL_OK ||
                    (st = ensure_buf(&m->new_list, &m->new_list_cap, pts_max, s)) != SAL_OK ||
                    (st = ensure_buf(&m->new_masks, &m->new_masks_cap, pts_max, s)) != SAL_OK ||
                    (st = ensure_node_table(m, pts_sum, s)) != SAL_OK)
                    return st;
                if (!m->n_new && dev_malloc((void **)&m->n_new, sizeof(unsigned long long)) != hipSuccess)
                    return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(node counter)");
            }
        }
    }
    // deepest level first: its children array never moves under a pending
    // split of a coarser level
    for (int l = top; l >= 0; --l) {
        if (count[l] == 0) continue;
        const int64_t kids = 8 * count[l];
        const bool nodes = m->rule == SAL_RULE_FOUR_NODES;
        const int64_t n_pts = nodes ? 6 * count[l] : kids;   // midpoints or centroids
        if ((st = ensure_level(m, l + 1, m->n[l + 1] + kids, s)) != SAL_OK) return st;
        if ((st = ensure_centroids(m, n_pts, s)) != SAL_OK) return st;
        if (nodes) {
            int64_t c3 = m->mid_xyz_cap;
            for (int a = 0; a < 3; ++a) {
                c3 = m->mid_xyz_cap;
                if ((st = ensure_buf(&m->mid_xyz[a], &c3, n_pts, s)) != SAL_OK) return st;
            }
            m->mid_xyz_cap = c3;
            if ((st = ensure_buf(&m->lab_scratch, &m->lab_cap, n_pts, s)) != SAL_OK ||
                (st = ensure_buf(&m->mid_masks, &m->mid_cap, n_pts, s)) != SAL_OK ||
                (st = ensure_buf(&m->mid_key, &m->mid_key_cap, n_pts, s)) != SAL_OK ||
                (st = ensure_buf(&m->mid_slot, &m->mid_slot_cap, n_pts, s)) != SAL_OK ||
                (st = ensure_buf(&m->new_list, &m->new_list_cap, n_pts, s)) != SAL_OK ||
                (st = ensure_buf(&m->new_masks, &m->new_masks_cap, n_pts, s)) != SAL_OK ||
                (st = ensure_node_table(m, n_pts, s)) != SAL_OK)
                return st;
            if (!m->n_new && dev_malloc((void **)&m->n_new, sizeof(unsigned long long)) != hipSuccess)
                return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(node counter)");
        }
        const int64_t base_block = m->n[l + 1] / 8;
        LevelPtrs L2 = ptrs(m);
        SAL_HIP(hipEventRecord(m->ev[5], s));
        SAL_HIP(launch_split(L2, m->g, m->T, l, m->list + off[l], count[l], base_block,
                             nodes ? nullptr : m->cen[0], nodes ? nullptr : m->cen[1],
                             nodes ? nullptr : m->cen[2], s));
        if (nodes) {
            // midpoints -> node table -> only the nodes not labeled before
            SAL_HIP(launch_midpoints(L2, m->g, l, m->list + off[l], count[l], m->mid_xyz[0],
                                     m->mid_xyz[1], m->mid_xyz[2], m->mid_key, s));
            SAL_HIP(launch_fill_u64(m->n_new, 0ull, 1, s));
            SAL_HIP(launch_node_insert(m->mid_key, n_pts, m->tkeys, m->tcap, m->mid_slot,
                                       m->new_list, m->n_new, s));
            SAL_HIP(launch_node_gather(m->new_list, m->n_new, n_pts, m->mid_xyz[0], m->mid_xyz[1],
                                       m->mid_xyz[2], m->cen[0], m->cen[1], m->cen[2], s));
            m->tused += n_pts;
        }
        SAL_HIP(hipEventRecord(m->ev[6], s));
        m->n[l + 1] += kids;
        m->n_leaves += 7 * count[l];
        if (nodes) {
            if ((st = label_scratch_dev(ctx, m, set, n_pts, m->n_new, opt, m->lab_scratch,
                                        m->ev[10], m->ev[9], m->new_masks)) != SAL_OK)
                return st;
            SAL_HIP(launch_node_store(m->new_list, m->n_new, n_pts, m->mid_slot, m->new_masks,
                                      m->tmasks, s));
            SAL_HIP(launch_node_fetch(m->mid_slot, n_pts, m->tmasks, m->mid_masks, s));
            SAL_HIP(launch_child_masks(L2, m->g, l, m->list + off[l], count[l], base_block,
                                       m->node0, m->vmask[l], m->mid_masks, m->vmask[l + 1],
                                       set->surf, s));
        } else if ((st = label_scratch(ctx, m, set, kids, opt, m->label[l + 1] + 8 * base_block,
                                       m->ev[10], m->ev[9])) != SAL_OK) {
            return st;
        }
        SAL_HIP(hipEventRecord(m->ev[7], s));
        SAL_HIP(hipEventSynchronize(m->ev[7]));
        ms_split += elapsed(m->ev[5], m->ev[6]);
        ms_label += elapsed(m->ev[10], m->ev[9]);
        ms_recheck += elapsed(m->ev[9], m->ev[7]);
        if (l + 1 > m->max_level) m->max_level = l + 1;
        n_split += count[l];
        if (nodes) {
            unsigned long long fresh = 0;
            SAL_HIP(hipMemcpy(&fresh, m->n_new, sizeof(fresh), hipMemcpyDeviceToHost));
            n_label += (int64_t)fresh;
        } else {
            n_label += n_pts;
        }
    }
    if (n_split_out) *n_split_out = n_split;
    SAL_HIP(hipEventRecord(m->ev[8], s));
    if (out) {
        unsigned long long cnt[kNumCounters];
        SAL_HIP(hipEventSynchronize(m->ev[8]));
        SAL_HIP(hipMemcpy(cnt, ctx->counters, sizeof(cnt), hipMemcpyDeviceToHost));
        out->n_leaves = m->n_leaves;
        out->n_boundary = n_split;
        out->n_labeled = n_label;
        out->n_pairs = n_label * set->n_tri;
        out->n_recheck_pairs = (int64_t)cnt[kCntRecheck];
        out->ms_mark = elapsed(m->ev[2], m->ev[3]);
        out->ms_compact = elapsed(m->ev[3], m->ev[4]);
        out->ms_split = ms_split;
        out->ms_label = ms_label;
        out->ms_recheck = ms_recheck;
        out->ms_total = elapsed(m->ev[2], m->ev[8]);
        out->graph = 0;
    }
    return SAL_OK;
}

// ----------------------------------------------------- captured round graph
uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

int64_t *rs_n(sal::RoundState *rs) {
    return (int64_t *)((char *)rs + offsetof(sal::RoundState, n));
}

int64_t *rs_n_kids(sal::RoundState *rs) {
    return (int64_t *)((char *)rs + offsetof(sal::RoundState, n_kids));
}

// Grows `cap` to 1.5 budget when fewer than `budget` entries are free, so that
// a graph captured against these buffers survives the following rounds.
sal_status reserve_level(sal_tet_mesh *m, int l, int64_t budget, hipStream_t s) {
    if (m->cap[l] - m->n[l] >= budget) return SAL_OK;
    return ensure_level(m, l, m->n[l] + budget + budget / 2, s);
}

// Enqueues the steps of one refine round on q, every size read on the
// device.  Levels without storage take no part (their split count must be 0,
// else the plan step stops the round).
sal_status enqueue_round(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set,
                         const sal_label_options &opt, int64_t kid_cap, hipStream_t q) {
    RoundState *rs = m->rs;
    int64_t *n_dev = rs_n(rs);
    LevelPtrs L = ptrs(m);
    L.n_dev = n_dev;
    int64_t off[kMaxLevels + 2] = {0};
    for (int l = 0; l <= kMaxLevels; ++l) off[l + 1] = off[l] + m->cap[l];
    SAL_HIP(launch_round_begin(rs, ctx->counters, q));
    for (int l = 0; l <= kMaxLevels; ++l)
        if (m->cap[l] > 0) SAL_HIP(launch_clear_flags_dev(m->flag[l], n_dev + l, q));
    for (int l = 0; l <= kMaxLevels; ++l)
        if (m->cap[l] > 0) SAL_HIP(launch_mark(L, m->g, m->T, l, q));
    for (int l = 0; l <= kMaxLevels; ++l) {
        if (m->cap[l] > 0) {
            CompactSrc src{m->flag[l], nullptr};
            SAL_HIP(launch_compact_dev(src, n_dev + l, m->cap[l], m->blocks, m->totals + l,
                                       m->list + off[l], q));
        } else {
            SAL_HIP(launch_fill_u64((unsigned long long *)(m->totals + l), 0ull, 1, q));
        }
    }
    SAL_HIP(launch_plan(rs, m->totals, q));
    for (int l = kMaxLevels - 1; l >= 0; --l)
        if (m->cap[l] > 0 && m->cap[l + 1] > 0)
            SAL_HIP(launch_split_dev(L, m->g, m->T, l, m->list + off[l], m->totals, rs, m->cen[0],
                                     m->cen[1], m->cen[2], q));
    sal_status st = enqueue_label_on(ctx, set, kid_cap, rs_n_kids(rs), m->cen[0], m->cen[1],
                                     m->cen[2], opt, m->lab_scratch, nullptr, nullptr, q);
    if (st != SAL_OK) return st;
    for (int l = kMaxLevels - 1; l >= 0; --l)
        if (m->cap[l] > 0 && m->cap[l + 1] > 0)
            SAL_HIP(launch_commit(rs, m->totals, l, m->lab_scratch, m->label[l + 1], q));
    SAL_HIP(launch_round_end(rs, ctx->counters, q));
    return SAL_OK;
}

// Runs up to `rounds` rounds as launches of the captured round graph; *done
// = rounds that completed (the rest stopped for capacity).
sal_status graph_rounds(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set,
                        sal_label_options opt, int rounds, sal_refine_stats *out, int *done) {
    hipStream_t s = ctx->stream;
    sal_status st;
    *done = 0;
    int64_t budget = std::max<int64_t>((int64_t)1 << 20, 2 * m->n_leaves);
    if (const char *e = std::getenv("SAL_REFINE_GRAPH_BUDGET")) {
        const long long v = std::atoll(e);
        if (v > 0) budget = (int64_t)v;
    }
    // every level, so that later calls find the same buffers and replay
    for (int l = 1; l <= kMaxLevels; ++l)
        if ((st = reserve_level(m, l, budget, s)) != SAL_OK) return st;
    if (m->cen_cap < budget && (st = ensure_centroids(m, budget + budget / 2, s)) != SAL_OK) return st;
    if (m->lab_cap < budget &&
        (st = ensure_buf(&m->lab_scratch, &m->lab_cap, budget + budget / 2, s)) != SAL_OK)
        return st;
    if (opt.precision == SAL_PREC_FP32_RECHECK && ctx->flag_cap < budget &&
        (st = ensure_flag_capacity(ctx, budget + budget / 2)) != SAL_OK)
        return st;
    int64_t kid_cap = std::min(m->cen_cap, m->lab_cap);
    if (opt.precision == SAL_PREC_FP32_RECHECK) kid_cap = std::min(kid_cap, ctx->flag_cap);
    int64_t list_need = 0, blocks_need = 1;
    for (int l = 0; l <= kMaxLevels; ++l) {
        list_need += m->cap[l];
        blocks_need = std::max<int64_t>(blocks_need, compact_blocks(m->cap[l]) + 1);
    }
    if ((st = ensure_buf(&m->list, &m->list_cap, list_need, s)) != SAL_OK) return st;
    if ((st = ensure_buf(&m->blocks, &m->blocks_cap, blocks_need, s)) != SAL_OK) return st;
    if (!m->rs && dev_malloc((void **)&m->rs, sizeof(RoundState)) != hipSuccess)
        return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(round state)");

    // The launch shape is fixed in the graph: resolve it now (tuning
    // synchronises), on lattice centroids written into the scratch.
    if (opt.points_per_lane == 0 || opt.block_waves == 0) {
        const int64_t nt = std::min<int64_t>(std::min<int64_t>(m->n[0], kid_cap), (int64_t)1 << 19);
        SAL_HIP(launch_lattice_centroids(m->g, nt, m->cen[0], m->cen[1], m->cen[2], s));
        // the trials read only the nt centroids written here
        if ((st = tune_launch(ctx, set, nt, m->cen[0], m->cen[1], m->cen[2], m->lab_scratch,
                              &opt)) != SAL_OK)
            return st;
    }

    // Everything the captured round reads or is shaped by: compared in full
    // (a hash of it is the quick first test) before a replay.
    std::vector<uint64_t> f;
    auto add = [&](uint64_t v) { f.push_back(v); };
    auto addp = [&](const void *p) { f.push_back((uint64_t)(uintptr_t)p); };
    auto addd = [&](double d) {
        uint64_t u;
        std::memcpy(&u, &d, sizeof u);
        f.push_back(u);
    };
    add(set->uid);
    addp(ctx);
    addp(ctx->flag_list);
    addp(ctx->rc_pairs);
    addp(ctx->rc_out);
    addp(ctx->rc_res);
    addp(ctx->rc_seg);
    add((uint64_t)ctx->flag_cap);
    add((uint64_t)ctx->rc_pair_cap);
    addp(ctx->counters);
    add((uint64_t)opt.precision);
    addd(opt.threshold);
    addd(opt.recheck_band);
    addd(opt.kappa);
    add((uint64_t)opt.points_per_lane);
    add((uint64_t)opt.block_waves);
    add((uint64_t)opt.cull_bounds);
    for (int l = 0; l <= kMaxLevels; ++l) {
        addp(m->key[l]);
        addp(m->label[l]);
        addp(m->child[l]);
        addp(m->flag[l]);
        add((uint64_t)m->cap[l]);
    }
    for (auto *c : m->cen) addp(c);
    addp(m->lab_scratch);
    addp(m->list);
    addp(m->blocks);
    addp(m->totals);
    addp(m->rs);
    add((uint64_t)kid_cap);
    uint64_t key = 0x5a1d5a1dull;
    for (const uint64_t v : f) key = mix(key, v);
    if (key == 0) key = 1;   // 0 marks "no graph"
    const bool capture = !m->round_graph || m->round_key != key || m->round_fields != f;
    if (capture) {
        if (m->round_graph) {
            SAL_HIP(hipGraphExecDestroy(m->round_graph));
            m->round_graph = nullptr;
        }
        m->round_key = 0;
        SAL_HIP(hipStreamSynchronize(s));
        hipGraph_t g = nullptr;
        SAL_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        sal_status cst = enqueue_round(ctx, m, set, opt, kid_cap, ctx->capture_stream);
        hipError_t ee = hipStreamEndCapture(ctx->capture_stream, &g);
        if (cst != SAL_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cst;
        }
        if (ee != hipSuccess) return hip_error(ee, "hipStreamEndCapture");
        ee = hipGraphInstantiate(&m->round_graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ee != hipSuccess) return hip_error(ee, "hipGraphInstantiate");
        m->round_key = key;
        m->round_fields = f;
    }

    RoundState h{};
    for (int l = 0; l <= kMaxLevels; ++l) {
        h.n[l] = m->n[l];
        h.cap[l] = m->cap[l];
    }
    h.kid_cap = kid_cap;
    h.n_leaves = m->n_leaves;
    SAL_HIP(hipStreamSynchronize(s));
    SAL_HIP(hipMemcpy(m->rs, &h, sizeof h, hipMemcpyHostToDevice));
    SAL_HIP(hipEventRecord(m->ev[11], s));
    for (int r = 0; r < rounds; ++r) {
        SAL_HIP(hipGraphLaunch(m->round_graph, s));
        SAL_HIP(hipEventRecord(m->ev[12 + r], s));
    }
    SAL_HIP(hipStreamSynchronize(s));
    SAL_HIP(hipMemcpy(&h, m->rs, sizeof h, hipMemcpyDeviceToHost));
    for (int l = 0; l <= kMaxLevels; ++l) {
        m->n[l] = h.n[l];
        if (h.n[l] > 0 && l > m->max_level) m->max_level = l;
    }
    m->n_leaves = h.n_leaves;
    *done = h.round;
    if (out) {
        for (int r = 0; r < h.round; ++r) {
            sal_refine_stats &o = out[r];
            o.n_leaves = h.stat[r].n_leaves;
            o.n_boundary = h.stat[r].n_boundary;
            o.n_labeled = h.stat[r].n_labeled;
            o.n_pairs = h.stat[r].n_labeled * set->n_tri;
            o.n_recheck_pairs = h.stat[r].n_recheck_pairs;
            o.ms_total = elapsed(m->ev[11 + r], m->ev[12 + r]);
            o.graph = capture ? 1 : 2;
        }
    }
    if (h.status == 2) return set_error(SAL_ERR_CAPACITY, "refinement beyond level 3");
    return SAL_OK;
}

}  // namespace
}  // namespace sal

using namespace sal;

namespace sal {

// The conforming mesh for the post-processing passes; null before
// sal_tet_mesh_conform.
bool conform_view(sal_tet_mesh *m, ConformView *v) {
    if (!m || !m->conformed) return false;
    v->g = m->g;
    v->n_tets = m->conf_tets;
    v->n_nodes = m->conf_nodes;
    v->ids = m->conf_ids;
    v->labels = m->conf_labels;
    v->keys = m->conf_keys;
    v->xyz = m->conf_xyz;
    v->cache = &m->smooth;
    return true;
}
int mesh_device(const sal_tet_mesh *m) { return m->device; }

namespace {

// Device scratch freed when the call ends.
struct DevScratch {
    std::vector<void *> bufs;
    ~DevScratch() { clear(); }
    void clear() {
        for (void *p : bufs) (void)hipFree(p);
        bufs.clear();
    }
    template <typename T>
    sal_status get(T **p, int64_t n) {
        void *q = nullptr;
        const size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
        if (dev_malloc(&q, bytes) != hipSuccess) return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(conform)");
        bufs.push_back(q);
        *p = (T *)q;
        return SAL_OK;
    }
};

// A device buffer reused across the rounds of one call, reallocated (with a
// quarter to spare) only when a round needs more than it holds.
template <typename T>
struct GrowBuf {
    T *p = nullptr;
    int64_t cap = 0;
    ~GrowBuf() {
        if (p) (void)hipFree(p);
    }
    sal_status need(int64_t n) {
        if (n <= cap) return SAL_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        const int64_t c = n + n / 4 + 1024;
        if (dev_malloc((void **)&p, (size_t)c * sizeof(T)) != hipSuccess)
            return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(conform)");
        cap = c;
        return SAL_OK;
    }
};

}  // namespace
}  // namespace sal

extern "C" {

void sal_tet_mesh_destroy(sal_tet_mesh *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    for (int l = 0; l <= kMaxLevels; ++l) {
        if (m->key[l]) (void)hipFree(m->key[l]);
        if (m->label[l]) (void)hipFree(m->label[l]);
        if (m->child[l]) (void)hipFree(m->child[l]);
        if (m->flag[l]) (void)hipFree(m->flag[l]);
    }
    for (auto &c : m->cen)
        if (c) (void)hipFree(c);
    if (m->list) (void)hipFree(m->list);
    if (m->blocks) (void)hipFree(m->blocks);
    if (m->totals) (void)hipFree(m->totals);
    if (m->lab_scratch) (void)hipFree(m->lab_scratch);
    sal::smooth_cache_free(m->smooth);
    void *conf[] = {m->conf_ids, m->conf_labels, m->conf_keys, m->conf_xyz};
    for (void *p : conf)
        if (p) (void)hipFree(p);
    if (m->node0) (void)hipFree(m->node0);
    for (auto *v : m->vmask)
        if (v) (void)hipFree(v);
    if (m->mid_masks) (void)hipFree(m->mid_masks);
    for (auto *p : m->mid_xyz)
        if (p) (void)hipFree(p);
    void *more[] = {m->mid_key, m->mid_slot, m->new_list, m->new_masks, m->n_new, m->tkeys,
                    m->tmasks};
    for (void *p : more)
        if (p) (void)hipFree(p);
    if (m->rs) (void)hipFree(m->rs);
    if (m->round_graph) (void)hipGraphExecDestroy(m->round_graph);
    for (auto &e : m->ev)
        if (e) (void)hipEventDestroy(e);
    delete m;
}

sal_status sal_tet_mesh_create_lattice(sal_context *ctx, const double origin[3], double h,
                                       const int32_t cells[3], sal_tet_mesh **out) {
    try {
        if (out) *out = nullptr;
        if (!ctx || !origin || !cells || !out) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
        if (!(std::isfinite(h) && h > 0.0)) return set_error(SAL_ERR_INVALID_ARG, "h must be > 0");
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(origin[a])) return set_error(SAL_ERR_INVALID_ARG, "non-finite origin");
            if (cells[a] < 1 || cells[a] > (1 << 16))
                return set_error(SAL_ERR_INVALID_ARG, "cells must be in 1..65536 per axis");
        }
        const int64_t n0 = 6ll * cells[0] * cells[1] * cells[2];
        if (n0 > 0x7fffffffll)
            return set_error(SAL_ERR_CAPACITY, "more than 2^31 lattice tetrahedra");
        SAL_HIP(hipSetDevice(ctx->device));
        auto *m = new sal_tet_mesh();
        m->device = ctx->device;
        for (int a = 0; a < 3; ++a) {
            m->g.origin[a] = origin[a];
            m->g.cells[a] = cells[a];
        }
        m->g.h = h;
        m->T = make_child_tables();
        sal_status st = SAL_OK;
        auto fail = [&](sal_status s) { sal_tet_mesh_destroy(m); return s; };
        for (auto &e : m->ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(set_error(SAL_ERR_DEVICE, "hipEventCreate"));
        if ((st = ensure_level(m, 0, n0, ctx->stream)) != SAL_OK) return fail(st);
        m->n[0] = n0;
        if (dev_malloc((void **)&m->totals, (kMaxLevels + 1) * sizeof(int64_t)) != hipSuccess)
            return fail(set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(totals)"));
        if (hipError_t e = launch_fill_i32(m->child[0], -1, n0, ctx->stream); e != hipSuccess)
            return fail(hip_error(e, "fill child"));
        if (hipError_t e = launch_fill_i32(m->label[0], -2, n0, ctx->stream); e != hipSuccess)
            return fail(hip_error(e, "fill label"));
        m->n_leaves = n0;
        *out = m;
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_tet_mesh_create_lattice");
    }
}

sal_status sal_tet_mesh_size(const sal_tet_mesh *m, int64_t *n_leaves, int32_t *max_level) {
    if (!m) return set_error(SAL_ERR_INVALID_ARG, "mesh is NULL");
    if (n_leaves) *n_leaves = m->n_leaves;
    if (max_level) *max_level = m->max_level;
    return SAL_OK;
}

namespace {

// Arguments shared by the refinement entry points; fills the resolved
// options.  Nothing is enqueued.
sal_status check_refine_args(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set,
                             const sal_label_options *opt_in, sal_label_options *opt) {
    if (!ctx || !m || !set) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
    if (set->device != ctx->device || m->device != ctx->device)
        return set_error(SAL_ERR_INVALID_ARG, "objects live on different devices");
    sal_status st = resolve_options(opt_in, opt);
    if (st != SAL_OK) return st;
    opt->winding_type = SAL_WINDING_NONE;
    if (m->conformed)
        return set_error(SAL_ERR_INVALID_ARG, "the mesh was made conforming; it cannot be refined");
    if (m->labeled0 && m->rule != opt->element_rule)
        return set_error(SAL_ERR_INVALID_ARG, "the mesh was labeled with another element rule");
    if (opt->use_graph && opt->element_rule == SAL_RULE_FOUR_NODES)
        return set_error(SAL_ERR_INVALID_ARG,
                         "use_graph applies to the centroid rule; the four-node rule runs host-driven");
    return SAL_OK;
}

// Section 2.1.3 item 1: labels the whole lattice if it is not labeled yet
// (the centroids, or under the four-node rule every lattice node and then
// each tetrahedron from its four nodes).  r0 (if set) gets the round's stats.
sal_status label_lattice(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set,
                         const sal_label_options &opt, sal_refine_stats *r0) {
    hipStream_t s = ctx->stream;
    sal_status st;
    SAL_HIP(launch_fill_u64(ctx->counters, 0ull, kNumCounters, s));
    SAL_HIP(hipEventRecord(m->ev[0], s));
    int64_t labeled0 = 0;
    if (!m->labeled0 && opt.element_rule == SAL_RULE_FOUR_NODES) {
        m->rule = SAL_RULE_FOUR_NODES;
        const int64_t n_nodes = (int64_t)(m->g.cells[0] + 1) * (m->g.cells[1] + 1) *
                                (int64_t)(m->g.cells[2] + 1);
        if ((st = ensure_centroids(m, n_nodes, s)) != SAL_OK) return st;
        if ((st = ensure_buf(&m->lab_scratch, &m->lab_cap, n_nodes, s)) != SAL_OK) return st;
        if (!m->node0 && dev_malloc((void **)&m->node0, (size_t)n_nodes * sizeof(uint64_t)) !=
                             hipSuccess)
            return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(node masks)");
        SAL_HIP(launch_lattice_nodes(m->g, n_nodes, m->cen[0], m->cen[1], m->cen[2], s));
        if ((st = label_scratch(ctx, m, set, n_nodes, opt, m->lab_scratch, m->ev[10], m->ev[9],
                                m->node0)) != SAL_OK)
            return st;
        SAL_HIP(launch_elem_from_nodes0(m->g, m->n[0], m->node0, set->surf, m->label[0], s));
        m->labeled0 = true;
        labeled0 = n_nodes;
    } else if (!m->labeled0) {
        m->rule = SAL_RULE_CENTROID;
        if ((st = ensure_centroids(m, m->n[0], s)) != SAL_OK) return st;
        SAL_HIP(launch_lattice_centroids(m->g, m->n[0], m->cen[0], m->cen[1], m->cen[2], s));
        if ((st = label_scratch(ctx, m, set, m->n[0], opt, m->label[0], m->ev[10], m->ev[9])) !=
            SAL_OK)
            return st;
        m->labeled0 = true;
        labeled0 = m->n[0];
    } else {
        SAL_HIP(hipEventRecord(m->ev[10], s));
        SAL_HIP(hipEventRecord(m->ev[9], s));
    }
    SAL_HIP(hipEventRecord(m->ev[1], s));
    if (r0) {
        unsigned long long cnt[kNumCounters];
        SAL_HIP(hipEventSynchronize(m->ev[1]));
        SAL_HIP(hipMemcpy(cnt, ctx->counters, sizeof(cnt), hipMemcpyDeviceToHost));
        r0->n_leaves = m->n_leaves;
        r0->n_labeled = labeled0;
        r0->n_pairs = labeled0 * set->n_tri;
        r0->n_recheck_pairs = (int64_t)cnt[kCntRecheck];
        r0->ms_label = elapsed(m->ev[10], m->ev[9]);
        r0->ms_recheck = elapsed(m->ev[9], m->ev[1]);
        r0->ms_total = elapsed(m->ev[0], m->ev[1]);
    }
    return SAL_OK;
}

}  // namespace

sal_status sal_refine_relabel(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set,
                              int32_t rounds, const sal_label_options *opt_in,
                              sal_refine_stats *per_round) {
    try {
        sal_label_options opt;
        sal_status st = check_refine_args(ctx, m, set, opt_in, &opt);
        if (st != SAL_OK) return st;
        if (rounds < 0) return set_error(SAL_ERR_INVALID_ARG, "rounds < 0");
        if (m->max_level + rounds > kMaxLevels)
            return set_error(SAL_ERR_CAPACITY, "at most 3 refinement levels");
        SAL_HIP(hipSetDevice(ctx->device));
        if (opt.cull_bounds && (st = ensure_surface_balls(ctx, set)) != SAL_OK) return st;
        if (per_round) std::memset(per_round, 0, sizeof(sal_refine_stats) * (size_t)(rounds + 1));
        if ((st = label_lattice(ctx, m, set, opt, per_round)) != SAL_OK) return st;
        int first = 1;
        if (opt.use_graph && rounds > 0) {
            int done = 0;
            st = graph_rounds(ctx, m, set, opt, rounds, per_round ? per_round + 1 : nullptr, &done);
            if (st != SAL_OK) return st;
            first = 1 + done;
        }
        for (int r = first; r <= rounds; ++r)
            if ((st = eager_round(ctx, m, set, opt, per_round ? per_round + r : nullptr)) != SAL_OK)
                return st;
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_refine_relabel");
    }
}

sal_status sal_refine_relabel_converge(sal_context *ctx, sal_tet_mesh *m,
                                       const sal_surface_set *set, int32_t finest_level,
                                       int32_t max_steps, const sal_label_options *opt_in,
                                       sal_refine_stats *per_step, int32_t *n_steps,
                                       int32_t *converged) {
    try {
        sal_label_options opt;
        sal_status st = check_refine_args(ctx, m, set, opt_in, &opt);
        if (st != SAL_OK) return st;
        if (finest_level < 0 || finest_level > kMaxLevels)
            return set_error(SAL_ERR_INVALID_ARG, "finest_level outside 0..3");
        if (max_steps < 0) return set_error(SAL_ERR_INVALID_ARG, "max_steps < 0");
        if (opt.use_graph)
            return set_error(SAL_ERR_INVALID_ARG, "the converging recursion runs host-driven");
        SAL_HIP(hipSetDevice(ctx->device));
        if (opt.cull_bounds && (st = ensure_surface_balls(ctx, set)) != SAL_OK) return st;
        if (per_step) std::memset(per_step, 0, sizeof(sal_refine_stats) * (size_t)(max_steps + 1));
        if (n_steps) *n_steps = 0;
        if (converged) *converged = 0;
        if ((st = label_lattice(ctx, m, set, opt, per_step)) != SAL_OK) return st;
        for (int step = 1; step <= max_steps; ++step) {
            sal_refine_stats one{};
            int64_t split = 0;
            if ((st = eager_round(ctx, m, set, opt, per_step ? &one : nullptr, finest_level,
                                  &split)) != SAL_OK)
                return st;
            if (split == 0) {
                if (converged) *converged = 1;
                return SAL_OK;
            }
            if (per_step) per_step[step] = one;
            if (n_steps) *n_steps = step;
        }
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_refine_relabel_converge");
    }
}

sal_status sal_tet_mesh_conform(sal_context *ctx, sal_tet_mesh *m, sal_conform_info *info) {
    // Frees the conforming-mesh arrays unless the call completes, so a call
    // that fails part way leaves none behind for a later call to overwrite.
    struct DropUnlessDone {
        sal_tet_mesh *m;
        bool done = false;
        ~DropUnlessDone() {
            if (done) return;
            int32_t **i32[] = {&m->conf_ids, &m->conf_labels};
            for (int32_t **p : i32)
                if (*p) (void)hipFree(*p), *p = nullptr;
            if (m->conf_keys) (void)hipFree(m->conf_keys), m->conf_keys = nullptr;
            if (m->conf_xyz) (void)hipFree(m->conf_xyz), m->conf_xyz = nullptr;
        }
    };
    try {
        if (!ctx || !m) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
        if (m->device != ctx->device) return set_error(SAL_ERR_INVALID_ARG, "mesh lives on another device");
        if (m->conformed) return set_error(SAL_ERR_INVALID_ARG, "the mesh is already conforming");
        DropUnlessDone guard{m};
        SAL_HIP(hipSetDevice(ctx->device));
        hipStream_t s = ctx->stream;
        sal_status st;
        DevScratch keep;                 // lives to the end of the call
        unsigned long long *counters = nullptr;   // [0] keys added, [1] overflow
        if ((st = keep.get(&counters, 2)) != SAL_OK) return st;
        // closure state: flags per entry (hanging bits, quarter point, red)
        // and the set of all vertices, built once and grown with the splits
        int64_t entries = 0;
        for (int l = 0; l <= m->max_level; ++l) entries += m->n[l];
        int64_t cap = 1 << 16, used = 0;
        while (cap < 2 * entries) cap <<= 1;
        DevScratch set_mem;
        unsigned long long *set = nullptr;
        // (re)builds the set from every entry and the full patterns
        auto rebuild = [&]() -> sal_status {
            for (;;) {
                set_mem.clear();
                sal_status e;
                if ((e = set_mem.get(&set, cap)) != SAL_OK) return e;
                SAL_HIP(launch_fill_u64(set, ~0ull, cap, s));
                SAL_HIP(launch_fill_u64(counters, 0ull, 2, s));
                LevelPtrs L = ptrs(m);
                for (int l = 0; l <= m->max_level; ++l)
                    SAL_HIP(launch_insert_range(L, m->g, l, 0, m->n[l], set, cap, nullptr, 0,
                                                nullptr, counters, counters + 1, s));
                unsigned long long c[2] = {0, 0};
                SAL_HIP(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, s));
                SAL_HIP(hipStreamSynchronize(s));
                used = (int64_t)c[0];
                if (c[1] == 0 && 2 * used <= cap) break;
                cap <<= 2;
            }
            LevelPtrs L = ptrs(m);
            for (int l = 0; l <= m->max_level; ++l)
                SAL_HIP(launch_pattern_full(L, m->g, l, 0, m->n[l], set, cap, s));
            return SAL_OK;
        };
        if ((st = rebuild()) != SAL_OK) return st;
        int rounds = 0;
        GrowBuf<int32_t> red_buf;              // red leaves of a round
        GrowBuf<unsigned long long> fresh_buf; // vertices new in a round
        GrowBuf<uint32_t> cells_buf;           // level-0 cells those vertices touch, one bit each
        const int64_t cell_words =
            ((int64_t)m->g.cells[0] * m->g.cells[1] * m->g.cells[2] + 31) / 32;
        for (;;) {
            int64_t off[kMaxLevels + 2] = {0};
            for (int l = 0; l <= m->max_level; ++l) off[l + 1] = off[l] + m->n[l];
            if ((st = red_buf.need(off[m->max_level + 1])) != SAL_OK) return st;
            int32_t *red_list = red_buf.p;
            int64_t red[kMaxLevels + 1] = {0}, total_red = 0;
            for (int l = 0; l <= m->max_level; ++l) {
                CompactSrc src{m->flag[l], nullptr, 0x80};
                if ((st = compact(m, src, m->n[l], red_list + off[l], m->totals + l, s)) != SAL_OK)
                    return st;
            }
            SAL_HIP(hipMemcpyAsync(red, m->totals, sizeof(int64_t) * (m->max_level + 1),
                                   hipMemcpyDeviceToHost, s));
            SAL_HIP(hipStreamSynchronize(s));
            for (int l = 0; l <= m->max_level; ++l) total_red += red[l];
            if (total_red == 0) break;
            if (m->max_level == kMaxLevels && red[kMaxLevels] > 0)
                return set_error(SAL_ERR_INTERNAL, "closure beyond level 3");
            // red splits, deepest level first (its arrays never move under a
            // pending split of a coarser level); children keep the label
            int64_t old_n[kMaxLevels + 1] = {0};
            for (int l = 0; l <= kMaxLevels; ++l) old_n[l] = m->n[l];
            for (int l = m->max_level; l >= 0; --l) {
                if (red[l] == 0) continue;
                const int64_t kids = 8 * red[l];
                if ((st = ensure_level(m, l + 1, m->n[l + 1] + kids, s)) != SAL_OK) return st;
                const int64_t base_block = m->n[l + 1] / 8;
                LevelPtrs L2 = ptrs(m);
                L2.inherit = 1;
                SAL_HIP(launch_split(L2, m->g, m->T, l, red_list + off[l], red[l], base_block, nullptr,
                                     nullptr, nullptr, s));
                m->n[l + 1] += kids;
                if (l + 1 > m->max_level) m->max_level = l + 1;
                m->n_leaves += 7 * red[l];
            }
            ++rounds;
            // the new vertices are edge midpoints of the split leaves (6 each)
            int64_t fcap = 1024;
            while (fcap < 12 * total_red) fcap <<= 1;
            if ((st = fresh_buf.need(fcap)) != SAL_OK) return st;
            unsigned long long *fresh = fresh_buf.p;
            if ((st = cells_buf.need(cell_words)) != SAL_OK) return st;
            uint32_t *cells_new = cells_buf.p;
            SAL_HIP(launch_fill_u64(fresh, ~0ull, fcap, s));
            SAL_HIP(launch_fill_i32((int32_t *)cells_new, 0, cell_words, s));
            SAL_HIP(launch_fill_u64(counters, 0ull, 2, s));
            LevelPtrs L = ptrs(m);
            for (int l = 0; l <= m->max_level; ++l)
                SAL_HIP(launch_insert_range(L, m->g, l, old_n[l], m->n[l] - old_n[l], set, cap, fresh,
                                            fcap, cells_new, counters, counters + 1, s));
            unsigned long long c[2] = {0, 0};
            SAL_HIP(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, s));
            SAL_HIP(hipStreamSynchronize(s));
            used += (int64_t)c[0];
            if (c[1] != 0 || 2 * used > cap) {
                // a table filled up: a larger set and full patterns
                while (cap < 4 * used) cap <<= 1;
                if (c[1] != 0) cap <<= 1;
                if ((st = rebuild()) != SAL_OK) return st;
                SAL_HIP(hipStreamSynchronize(s));
                continue;
            }
            // old entries: patterns plus what the new vertices hit; new
            // children: full patterns
            for (int l = 0; l <= m->max_level; ++l) {
                SAL_HIP(launch_pattern_fresh(L, m->g, l, old_n[l], fresh, fcap, cells_new, s));
                SAL_HIP(launch_pattern_full(L, m->g, l, old_n[l], m->n[l] - old_n[l], set, cap, s));
            }
            SAL_HIP(hipStreamSynchronize(s));
        }

        // the leaves in index order per level
        int64_t count[kMaxLevels + 1] = {0}, off[kMaxLevels + 2] = {0}, n_all = 0;
        for (int l = 0; l <= m->max_level; ++l) off[l + 1] = off[l] + m->n[l];
        if ((st = ensure_buf(&m->list, &m->list_cap, off[m->max_level + 1], s)) != SAL_OK) return st;
        for (int l = 0; l <= m->max_level; ++l) {
            CompactSrc src{nullptr, m->child[l]};
            if ((st = compact(m, src, m->n[l], m->list + off[l], m->totals + l, s)) != SAL_OK) return st;
        }
        SAL_HIP(hipMemcpyAsync(count, m->totals, sizeof(int64_t) * (m->max_level + 1),
                               hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        for (int l = 0; l <= m->max_level; ++l) n_all += count[l];
        if (n_all != m->n_leaves) return set_error(SAL_ERR_INTERNAL, "leaf count mismatch");

        // the tetrahedra of each leaf, at the exclusive sum of the counts
        int32_t *counts = nullptr;
        int64_t *offsets = nullptr;
        if ((st = keep.get(&counts, n_all)) != SAL_OK || (st = keep.get(&offsets, n_all)) != SAL_OK)
            return st;
        unsigned long long *hist = nullptr;   // leaves by number of pieces
        if ((st = keep.get(&hist, 4)) != SAL_OK) return st;
        SAL_HIP(launch_fill_u64(hist, 0ull, 4, s));
        {
            LevelPtrs L = ptrs(m);
            int64_t coff = 0;
            for (int l = 0; l <= m->max_level; coff += count[l], ++l)
                SAL_HIP(launch_tet_counts(L, l, m->list + off[l], count[l], counts + coff, hist, s));
        }
        size_t tmp_bytes = 0;
        SAL_HIP(exclusive_sum_i32(counts, offsets, n_all, nullptr, &tmp_bytes, s));
        char *tmp = nullptr;
        if ((st = keep.get(&tmp, (int64_t)tmp_bytes)) != SAL_OK) return st;
        SAL_HIP(exclusive_sum_i32(counts, offsets, n_all, tmp, &tmp_bytes, s));
        int64_t last_off = 0;
        int32_t last_cnt = 0;
        SAL_HIP(hipMemcpyAsync(&last_off, offsets + n_all - 1, sizeof(last_off), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipMemcpyAsync(&last_cnt, counts + n_all - 1, sizeof(last_cnt), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        const int64_t n_tets = last_off + last_cnt;
        const int64_t n_corner = 4 * n_tets;
        if (n_corner > INT32_MAX) return set_error(SAL_ERR_CAPACITY, "conforming mesh above 2^31 corners");
        int64_t *tkeys = nullptr, *sorted = nullptr, *pos = nullptr, *nodes = nullptr;
        int32_t *head = nullptr;
        if ((st = keep.get(&tkeys, n_corner)) != SAL_OK || (st = keep.get(&sorted, n_corner)) != SAL_OK ||
            (st = keep.get(&pos, n_corner)) != SAL_OK || (st = keep.get(&head, n_corner)) != SAL_OK ||
            (st = keep.get(&nodes, n_corner)) != SAL_OK)
            return st;
        if (dev_malloc((void **)&m->conf_labels, (size_t)std::max<int64_t>(n_tets, 1) * sizeof(int32_t)) !=
                hipSuccess ||
            dev_malloc((void **)&m->conf_ids, (size_t)std::max<int64_t>(n_corner, 1) * sizeof(int32_t)) !=
                hipSuccess)
            return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(conforming mesh)");
        LevelPtrs L = ptrs(m);
        int64_t boff = 0;
        for (int l = 0; l <= m->max_level; boff += count[l], ++l)
            SAL_HIP(launch_emit(L, m->g, l, m->list + off[l], count[l], offsets + boff, tkeys,
                                m->conf_labels, s));
        // nodes: the distinct corner keys in ascending order; ids by search
        size_t sort_bytes = 0, uniq_bytes = 0;
        SAL_HIP(sort_keys_i64(tkeys, sorted, n_corner, nullptr, &sort_bytes, s));
        SAL_HIP(launch_unique(sorted, n_corner, head, pos, nodes, nullptr, &uniq_bytes, s));
        tmp_bytes = std::max(sort_bytes, uniq_bytes);
        if ((st = keep.get(&tmp, (int64_t)tmp_bytes)) != SAL_OK) return st;
        SAL_HIP(sort_keys_i64(tkeys, sorted, n_corner, tmp, &tmp_bytes, s));
        SAL_HIP(launch_unique(sorted, n_corner, head, pos, nodes, tmp, &tmp_bytes, s));
        int64_t last_pos = 0;
        int32_t last_head = 0;
        SAL_HIP(hipMemcpyAsync(&last_pos, pos + n_corner - 1, sizeof(last_pos), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipMemcpyAsync(&last_head, head + n_corner - 1, sizeof(last_head), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        const int64_t n_nodes = last_pos + last_head;
        if (dev_malloc((void **)&m->conf_keys, (size_t)std::max<int64_t>(n_nodes, 1) * sizeof(int64_t)) !=
                hipSuccess ||
            dev_malloc((void **)&m->conf_xyz, (size_t)std::max<int64_t>(3 * n_nodes, 1) * sizeof(float)) !=
                hipSuccess)
            return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(conforming nodes)");
        SAL_HIP(hipMemcpyAsync(m->conf_keys, nodes, (size_t)n_nodes * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
        SAL_HIP(launch_node_ids(tkeys, n_corner, m->conf_keys, n_nodes, m->conf_ids, s));
        SAL_HIP(launch_node_xyz(m->g, m->conf_keys, n_nodes, m->conf_xyz, s));
        unsigned long long hh[4] = {0, 0, 0, 0};
        SAL_HIP(hipMemcpyAsync(hh, hist, sizeof(hh), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        m->conf_tets = n_tets;
        m->conf_nodes = n_nodes;
        m->conformed = true;
        guard.done = true;
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->n_tets = n_tets;
            info->n_nodes = n_nodes;
            info->n_leaves = n_all;
            for (int k = 0; k < 4; ++k) info->n_by_pieces[k] = (int64_t)hh[k];
            info->closure_rounds = rounds;
        }
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_tet_mesh_conform");
    }
}

sal_status sal_tet_mesh_export_conforming(sal_context *ctx, const sal_tet_mesh *m, int32_t *tets,
                                          int32_t *labels, float *xyz, int64_t *node_keys) {
    if (!ctx || !m) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
    if (!m->conformed) return set_error(SAL_ERR_INVALID_ARG, "call sal_tet_mesh_conform first");
    SAL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    if (tets)
        SAL_HIP(hipMemcpyAsync(tets, m->conf_ids, (size_t)m->conf_tets * 4 * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, s));
    if (labels)
        SAL_HIP(hipMemcpyAsync(labels, m->conf_labels, (size_t)m->conf_tets * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, s));
    if (xyz)
        SAL_HIP(hipMemcpyAsync(xyz, m->conf_xyz, (size_t)m->conf_nodes * 3 * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    if (node_keys)
        SAL_HIP(hipMemcpyAsync(node_keys, m->conf_keys, (size_t)m->conf_nodes * sizeof(int64_t),
                               hipMemcpyDeviceToDevice, s));
    return SAL_OK;
}

namespace {

struct KeyParts {
    int l, q;
    int64_t c[3];
};

KeyParts decode_key(uint64_t k) {
    KeyParts p;
    p.l = (int)(k >> 60);
    p.q = (int)((k >> 57) & 7u);
    p.c[0] = (int64_t)((k >> 38) & 0x7ffffu);
    p.c[1] = (int64_t)((k >> 19) & 0x7ffffu);
    p.c[2] = (int64_t)(k & 0x7ffffu);
    return p;
}

uint64_t encode_key(int l, int q, const int64_t c[3]) {
    return ((uint64_t)l << 60) | ((uint64_t)q << 57) | ((uint64_t)c[0] << 38) |
           ((uint64_t)c[1] << 19) | (uint64_t)c[2];
}

// The parent of a level-l (l >= 1) tetrahedron and the child's rank in the
// parent's block (the order the splits use).
uint64_t parent_of(const sal::ChildTables &T, const KeyParts &p, int *rank) {
    const int code = (int)(p.c[0] & 1) | (int)((p.c[1] & 1) << 1) | (int)((p.c[2] & 1) << 2);
    const int64_t pc[3] = {p.c[0] >> 1, p.c[1] >> 1, p.c[2] >> 1};
    for (int pq = 0; pq < 6; ++pq)
        if (T.rank[pq][code][p.q] >= 0) {
            *rank = T.rank[pq][code][p.q];
            return encode_key(p.l - 1, pq, pc);
        }
    *rank = -1;
    return ~0ull;
}

bool sorted_has(const std::vector<uint64_t> &v, uint64_t k) {
    return std::binary_search(v.begin(), v.end(), k);
}

}  // namespace

sal_status sal_tet_mesh_import(sal_context *ctx, sal_tet_mesh *m, int64_t n, const uint64_t *keys,
                               const int32_t *labels) {
    try {
        if (!ctx || !m) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
        if (m->device != ctx->device) return set_error(SAL_ERR_INVALID_ARG, "mesh lives on another device");
        if (m->labeled0 || m->max_level != 0 || m->conformed)
            return set_error(SAL_ERR_INVALID_ARG, "import needs a mesh fresh from sal_tet_mesh_create_lattice");
        if (n <= 0 || !keys || !labels) return set_error(SAL_ERR_INVALID_ARG, "no leaves to import");
        SAL_HIP(hipSetDevice(ctx->device));
        hipStream_t s = ctx->stream;
        std::vector<uint64_t> hk((size_t)n);
        std::vector<int32_t> hl((size_t)n);
        SAL_HIP(hipMemcpyAsync(hk.data(), keys, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipMemcpyAsync(hl.data(), labels, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        const int64_t n0 = m->n[0];
        // leaves per level, sorted by key (label alongside)
        std::vector<std::pair<uint64_t, int32_t>> leaf[kMaxLevels + 1];
        for (int64_t i = 0; i < n; ++i) {
            const KeyParts p = decode_key(hk[(size_t)i]);
            if (p.l > kMaxLevels || p.q > 5)
                return set_error(SAL_ERR_INVALID_ARG, "a key has no valid level or permutation");
            for (int a = 0; a < 3; ++a)
                if (p.c[a] >= ((int64_t)m->g.cells[a] << p.l))
                    return set_error(SAL_ERR_INVALID_ARG, "a key lies outside the lattice");
            if (hl[(size_t)i] < 0) return set_error(SAL_ERR_INVALID_ARG, "a leaf has no label");
            leaf[p.l].push_back({hk[(size_t)i], hl[(size_t)i]});
        }
        std::vector<uint64_t> leaf_keys[kMaxLevels + 1], inner[kMaxLevels + 1];
        for (int l = 0; l <= kMaxLevels; ++l) {
            std::sort(leaf[l].begin(), leaf[l].end());
            leaf_keys[l].resize(leaf[l].size());
            for (size_t i = 0; i < leaf[l].size(); ++i) leaf_keys[l][i] = leaf[l][i].first;
            if (std::adjacent_find(leaf_keys[l].begin(), leaf_keys[l].end()) != leaf_keys[l].end())
                return set_error(SAL_ERR_INVALID_ARG, "a key is listed twice");
        }
        // inner tetrahedra: the parents of every entry one level down; each
        // must have all 8 children and must not be a leaf itself
        int deepest = 0;
        for (int l = kMaxLevels; l >= 1; --l) {
            std::vector<uint64_t> entries(leaf_keys[l]);
            entries.insert(entries.end(), inner[l].begin(), inner[l].end());
            if (!entries.empty()) deepest = std::max(deepest, l);
            std::vector<uint64_t> par;
            par.reserve(entries.size());
            for (uint64_t k : entries) {
                int r;
                par.push_back(parent_of(m->T, decode_key(k), &r));
            }
            std::sort(par.begin(), par.end());
            for (size_t i = 0; i < par.size();) {
                size_t j = i;
                while (j < par.size() && par[j] == par[i]) ++j;
                if (j - i != 8)
                    return set_error(SAL_ERR_INVALID_ARG, "a refined tetrahedron lacks some of its 8 children");
                inner[l - 1].push_back(par[i]);
                i = j;
            }
            for (uint64_t k : inner[l - 1])
                if (sorted_has(leaf_keys[l - 1], k))
                    return set_error(SAL_ERR_INVALID_ARG, "a tetrahedron is both a leaf and refined");
        }
        if ((int64_t)(leaf_keys[0].size() + inner[0].size()) != n0)
            return set_error(SAL_ERR_INVALID_ARG, "the leaves do not cover the lattice");
        // layout: level 0 by index; each refined entry's children form one
        // block of 8 on the next level, blocks in the order of their parents
        std::vector<uint64_t> key_l[kMaxLevels + 1];
        std::vector<int32_t> lab_l[kMaxLevels + 1], child_l[kMaxLevels + 1];
        lab_l[0].assign((size_t)n0, -2);
        child_l[0].assign((size_t)n0, -1);
        for (const auto &e : leaf[0]) {
            const KeyParts p = decode_key(e.first);
            const int64_t idx = ((p.c[2] * m->g.cells[1] + p.c[1]) * m->g.cells[0] + p.c[0]) * 6 + p.q;
            lab_l[0][(size_t)idx] = e.second;
        }
        auto key_at = [&](int l, int64_t i) -> uint64_t {
            if (l > 0) return key_l[l][(size_t)i];
            const int q = (int)(i % 6);
            int64_t cell = i / 6;
            const int64_t c[3] = {cell % m->g.cells[0], (cell / m->g.cells[0]) % m->g.cells[1],
                                  cell / ((int64_t)m->g.cells[0] * m->g.cells[1])};
            return encode_key(0, q, c);
        };
        for (int l = 0; l < deepest; ++l) {
            const int64_t nl = l == 0 ? n0 : (int64_t)key_l[l].size();
            int32_t blocks = 0;
            for (int64_t i = 0; i < nl; ++i) {
                const uint64_t k = key_at(l, i);
                if (!sorted_has(inner[l], k)) continue;
                const KeyParts p = decode_key(k);
                child_l[l][(size_t)i] = blocks;
                for (int r = 0; r < 8; ++r) {
                    const int code = m->T.list[p.q][r][0], cq = m->T.list[p.q][r][1];
                    const int64_t cc[3] = {2 * p.c[0] + (code & 1), 2 * p.c[1] + ((code >> 1) & 1),
                                           2 * p.c[2] + ((code >> 2) & 1)};
                    const uint64_t ck = encode_key(l + 1, cq, cc);
                    key_l[l + 1].push_back(ck);
                    child_l[l + 1].push_back(-1);
                    auto it = std::lower_bound(leaf[l + 1].begin(), leaf[l + 1].end(),
                                               std::make_pair(ck, INT32_MIN));
                    lab_l[l + 1].push_back(it != leaf[l + 1].end() && it->first == ck ? it->second : -2);
                }
                ++blocks;
            }
        }
        // upload (everything is allocated before the mesh changes)
        for (int l = 1; l <= deepest; ++l) {
            sal_status st = ensure_level(m, l, (int64_t)key_l[l].size(), s);
            if (st != SAL_OK) return st;
        }
        for (int l = 0; l <= deepest; ++l) {
            const int64_t nl = l == 0 ? n0 : (int64_t)key_l[l].size();
            if (l > 0)
                SAL_HIP(hipMemcpyAsync(m->key[l], key_l[l].data(), (size_t)nl * sizeof(uint64_t),
                                       hipMemcpyHostToDevice, s));
            SAL_HIP(hipMemcpyAsync(m->label[l], lab_l[l].data(), (size_t)nl * sizeof(int32_t),
                                   hipMemcpyHostToDevice, s));
            SAL_HIP(hipMemcpyAsync(m->child[l], child_l[l].data(), (size_t)nl * sizeof(int32_t),
                                   hipMemcpyHostToDevice, s));
            SAL_HIP(launch_fill_u8(m->flag[l], 0, nl, s));
        }
        SAL_HIP(hipStreamSynchronize(s));
        for (int l = 1; l <= deepest; ++l) m->n[l] = (int64_t)key_l[l].size();
        m->max_level = deepest;
        m->n_leaves = n;
        m->rule = SAL_RULE_CENTROID;
        m->labeled0 = true;
        return SAL_OK;
    } catch (const std::bad_alloc &) {
        return set_error(SAL_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_tet_mesh_import");
    }
}

sal_status sal_tet_mesh_export(sal_context *ctx, const sal_tet_mesh *mc, uint64_t *keys,
                               int32_t *labels, float *cx, float *cy, float *cz) {
    try {
        if (!ctx || !mc) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
        auto *m = const_cast<sal_tet_mesh *>(mc);
        SAL_HIP(hipSetDevice(ctx->device));
        hipStream_t s = ctx->stream;
        int64_t total_entries = 0;
        for (int l = 0; l <= m->max_level; ++l) total_entries += m->n[l];
        sal_status st = ensure_buf(&m->list, &m->list_cap, total_entries, s);
        if (st != SAL_OK) return st;
        int64_t off[kMaxLevels + 2] = {0};
        for (int l = 0; l <= m->max_level; ++l) {
            off[l + 1] = off[l] + m->n[l];
            CompactSrc src{nullptr, m->child[l]};
            if ((st = compact(m, src, m->n[l], m->list + off[l], m->totals + l, s)) != SAL_OK)
                return st;
        }
        int64_t count[kMaxLevels + 1] = {0};
        SAL_HIP(hipMemcpyAsync(count, m->totals, sizeof(int64_t) * (m->max_level + 1),
                               hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        int64_t out_base = 0;
        LevelPtrs L = ptrs(m);
        for (int l = 0; l <= m->max_level; ++l) {
            SAL_HIP(launch_export(L, m->g, l, m->list + off[l], count[l], out_base, keys, labels, cx,
                                  cy, cz, s));
            out_base += count[l];
        }
        if (out_base != m->n_leaves) return set_error(SAL_ERR_INTERNAL, "leaf count mismatch");
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_tet_mesh_export");
    }
}

}  // extern "C"
