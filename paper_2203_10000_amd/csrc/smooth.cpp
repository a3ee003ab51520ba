// Taubin smoothing of the conforming mesh (paper section 2.2.1): host side.
// The edge graph is built once per conforming mesh with radix sorts (edge
// occurrences; the nodes by Morton code; both directions of each distinct
// edge in Morton ranks); the phases then
// run half steps until the stopping ratio is met, reading one double back
// per iteration.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "post_internal.h"
#include "runtime.h"

namespace sal {

void smooth_cache_free(SmoothCache *c) {
    if (!c) return;
    void *p[] = {c->rowptr, c->cols, c->cls, c->order, c->list[0], c->list[1], c->seg[0], c->seg[1],
                 c->head[0], c->head[1],
                 c->pos[0], c->pos[1], c->partials, c->sum};
    for (void *q : p)
        if (q) (void)hipFree(q);
    delete c;
}

namespace {

int bits_for(int64_t n) {
    int b = 1;
    while (b < 63 && (int64_t(1) << b) <= n) ++b;
    return b;
}

template <typename T>
sal_status dev_alloc(T **p, int64_t n) {
    if (dev_malloc((void **)p, (size_t)std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess)
        return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(smoothing)");
    return SAL_OK;
}

// Frees its buffers when the graph construction ends.
struct Temp {
    std::vector<void *> p;
    ~Temp() {
        for (void *q : p) (void)hipFree(q);
    }
    template <typename T>
    sal_status get(T **out, int64_t n) {
        sal_status st = dev_alloc(out, n);
        if (st == SAL_OK) p.push_back(*out);
        return st;
    }
};

sal_status build_graph(const ConformView &v, SmoothCache *c, hipStream_t s) {
    if (v.n_nodes >= (int64_t(1) << 28)) return set_error(SAL_ERR_CAPACITY, "smoothing: 2^28 nodes or more");
    if (6 * v.n_tets > INT32_MAX) return set_error(SAL_ERR_CAPACITY, "smoothing: too many tetrahedra");
    sal_status st;
    Temp t;
    const int64_t n_occ = 6 * v.n_tets;
    uint64_t *occ = nullptr, *occ_sorted = nullptr;
    int32_t *head = nullptr;
    int64_t *pos = nullptr;
    if ((st = t.get(&occ, n_occ)) != SAL_OK || (st = t.get(&occ_sorted, n_occ)) != SAL_OK ||
        (st = t.get(&head, n_occ)) != SAL_OK || (st = t.get(&pos, n_occ)) != SAL_OK)
        return st;
    unsigned long long *cnt = nullptr;   // [0] bad labels, [1] interface edges
    if ((st = t.get(&cnt, 2)) != SAL_OK) return st;
    SAL_HIP(launch_fill_u64(cnt, 0ull, 2, s));
    SAL_HIP(launch_edge_occurrences(v.ids, v.labels, v.n_tets, occ, cnt, s));
    const int nb = bits_for(v.n_nodes - 1);
    size_t b1 = 0, b2 = 0;
    SAL_HIP(sort_keys_u64(occ, occ_sorted, n_occ, 36 + nb, nullptr, &b1, s));
    SAL_HIP(exclusive_sum_head(head, pos, n_occ, nullptr, &b2, s));
    char *tmp = nullptr;
    size_t tmp_bytes = std::max(b1, b2);
    if ((st = t.get(&tmp, (int64_t)tmp_bytes)) != SAL_OK) return st;
    SAL_HIP(sort_keys_u64(occ, occ_sorted, n_occ, 36 + nb, tmp, &tmp_bytes, s));
    SAL_HIP(launch_edge_heads(occ_sorted, n_occ, head, s));
    tmp_bytes = std::max(b1, b2);
    SAL_HIP(exclusive_sum_head(head, pos, n_occ, tmp, &tmp_bytes, s));
    int64_t last_pos = 0;
    int32_t last_head = 0;
    SAL_HIP(hipMemcpyAsync(&last_pos, pos + n_occ - 1, sizeof(last_pos), hipMemcpyDeviceToHost, s));
    SAL_HIP(hipMemcpyAsync(&last_head, head + n_occ - 1, sizeof(last_head), hipMemcpyDeviceToHost, s));
    SAL_HIP(hipStreamSynchronize(s));
    unsigned long long bad = 0;
    SAL_HIP(hipMemcpy(&bad, cnt, sizeof(bad), hipMemcpyDeviceToHost));
    if (bad) return set_error(SAL_ERR_CAPACITY, "smoothing: labels outside [-1, 254]");
    const int64_t n_edges = last_pos + last_head;
    const int64_t n2 = 2 * n_edges;
    int64_t *start = nullptr;
    uint64_t *dkeys = nullptr, *dsorted = nullptr;
    if ((st = t.get(&start, n_edges)) != SAL_OK || (st = t.get(&dkeys, n2)) != SAL_OK ||
        (st = t.get(&dsorted, n2)) != SAL_OK)
        return st;
    // Morton ranks of the nodes
    uint64_t *code = nullptr, *code_sorted = nullptr;
    int32_t *ids = nullptr, *rank = nullptr;
    if ((st = t.get(&code, v.n_nodes)) != SAL_OK || (st = t.get(&code_sorted, v.n_nodes)) != SAL_OK ||
        (st = t.get(&ids, v.n_nodes)) != SAL_OK || (st = t.get(&rank, v.n_nodes)) != SAL_OK ||
        (st = dev_alloc(&c->order, v.n_nodes)) != SAL_OK)
        return st;
    size_t bm = 0;
    SAL_HIP(launch_morton_order(v.keys, v.n_nodes, code, code_sorted, ids, c->order, rank, nullptr, &bm, s));
    char *tmpm = nullptr;
    if ((st = t.get(&tmpm, (int64_t)bm)) != SAL_OK) return st;
    SAL_HIP(launch_morton_order(v.keys, v.n_nodes, code, code_sorted, ids, c->order, rank, tmpm, &bm, s));
    SAL_HIP(launch_edge_directed(occ_sorted, head, pos, n_occ, n_edges, start, rank, dkeys, cnt + 1, s));
    size_t b3 = 0;
    SAL_HIP(sort_keys_u64(dkeys, dsorted, n2, 32 + nb, nullptr, &b3, s));
    char *tmp3 = nullptr;
    if ((st = t.get(&tmp3, (int64_t)b3)) != SAL_OK) return st;
    SAL_HIP(sort_keys_u64(dkeys, dsorted, n2, 32 + nb, tmp3, &b3, s));
    if ((st = dev_alloc(&c->rowptr, v.n_nodes + 1)) != SAL_OK || (st = dev_alloc(&c->cols, n2)) != SAL_OK ||
        (st = dev_alloc(&c->cls, v.n_nodes)) != SAL_OK)
        return st;
    SAL_HIP(launch_csr(dsorted, n2, v.n_nodes, c->rowptr, c->cols, s));
    SAL_HIP(launch_node_class(c->rowptr, c->cols, v.keys, c->order, v.n_nodes, v.g, c->cls, s));
    // node lists of the two phases, in node order
    int64_t *blocks = nullptr, *totals = nullptr;
    if ((st = t.get(&blocks, compact_blocks(v.n_nodes) + 1)) != SAL_OK || (st = t.get(&totals, 2)) != SAL_OK)
        return st;
    for (int ph = 0; ph < 2; ++ph) {
        if ((st = dev_alloc(&c->list[ph], v.n_nodes)) != SAL_OK) return st;
        CompactSrc src{c->cls, nullptr, (uint8_t)(ph == 0 ? 1 : 2)};
        SAL_HIP(launch_compact(src, v.n_nodes, blocks, totals + ph, c->list[ph], s));
    }
    SAL_HIP(hipMemcpyAsync(c->n_list, totals, sizeof(c->n_list), hipMemcpyDeviceToHost, s));
    unsigned long long hcnt[2] = {0, 0};
    SAL_HIP(hipMemcpyAsync(hcnt, cnt, sizeof(hcnt), hipMemcpyDeviceToHost, s));
    SAL_HIP(hipStreamSynchronize(s));
    c->n_surface_edges = (int64_t)hcnt[1];
    c->n_nodes = v.n_nodes;
    c->n_edges = n_edges;
    c->partials_cap = taubin_blocks(std::max(c->n_list[0], c->n_list[1]));
    if ((st = dev_alloc(&c->partials, c->partials_cap)) != SAL_OK || (st = dev_alloc(&c->sum, 1)) != SAL_OK ||
        (st = dev_alloc(&c->pos[0], v.n_nodes)) != SAL_OK || (st = dev_alloc(&c->pos[1], v.n_nodes)) != SAL_OK)
        return st;
    if (n2 >= (int64_t(1) << 32)) return set_error(SAL_ERR_CAPACITY, "smoothing: 2^32 row entries or more");
    for (int ph = 0; ph < 2; ++ph) {
        if ((st = dev_alloc(&c->seg[ph], c->n_list[ph])) != SAL_OK) return st;
        SAL_HIP(launch_row_segments(c->rowptr, c->list[ph], c->n_list[ph], c->seg[ph], s));
        if ((st = dev_alloc(&c->head[ph], c->n_list[ph] * kTaubinGroup * kTaubinUnroll)) != SAL_OK)
            return st;
        SAL_HIP(launch_row_heads(c->rowptr, c->cols, c->list[ph], c->n_list[ph], c->head[ph], s));
        double e = 0.0;
        SAL_HIP(launch_row_entries(c->rowptr, c->list[ph], c->n_list[ph], c->partials, c->sum, s));
        SAL_HIP(hipMemcpyAsync(&e, c->sum, sizeof(e), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        c->n_entries[ph] = (int64_t)e;
    }
    return SAL_OK;
}

sal_status read_sum(const SmoothCache *c, double *out, hipStream_t s) {
    SAL_HIP(hipMemcpyAsync(out, c->sum, sizeof(double), hipMemcpyDeviceToHost, s));
    SAL_HIP(hipStreamSynchronize(s));
    return SAL_OK;
}

// One phase on c->pos[0] (the result ends there).
sal_status run_phase(SmoothCache *c, int ph, double lam, double mu, double xi, int max_iter,
                     int32_t *iters, double *ratio, hipStream_t s) {
    *iters = 0;
    *ratio = 0.0;
    const int64_t n = c->n_list[ph];
    if (max_iter <= 0 || n == 0) return SAL_OK;
    sal_status st;
    double norm0 = 0.0, step = 0.0;
    // the second buffer starts equal to the first: the nodes this phase does
    // not move (moved by an earlier phase, or fixed) read the same in both
    SAL_HIP(hipMemcpyAsync(c->pos[1], c->pos[0], (size_t)c->n_nodes * sizeof(float4),
                           hipMemcpyDeviceToDevice, s));
    SAL_HIP(launch_norm_sq(c->pos[0], c->list[ph], n, c->partials, c->sum, s));
    if ((st = read_sum(c, &norm0, s)) != SAL_OK) return st;
    norm0 = std::sqrt(norm0);
    for (int k = 0; k < max_iter; ++k) {
        SAL_HIP(launch_taubin_half(c->pos[0], c->pos[1], c->seg[ph], c->head[ph], c->cols,
                                   c->list[ph], n, lam, ph == 0, c->partials, c->sum, s));
        SAL_HIP(hipMemcpyAsync(&step, c->sum, sizeof(double), hipMemcpyDeviceToHost, s));
        SAL_HIP(launch_taubin_half(c->pos[1], c->pos[0], c->seg[ph], c->head[ph], c->cols,
                                   c->list[ph], n, -mu, ph == 0, c->partials, c->sum, s));
        SAL_HIP(hipStreamSynchronize(s));
        *iters = k + 1;
        *ratio = norm0 > 0.0 ? std::sqrt(step) / norm0 : 0.0;
        if (*ratio <= xi) break;
    }
    return SAL_OK;
}

}  // namespace

sal_status ensure_smooth_graph(const ConformView &v, hipStream_t s) {
    if (*v.cache) return SAL_OK;
    auto *c = new SmoothCache();
    const sal_status st = build_graph(v, c, s);
    if (st != SAL_OK) {
        smooth_cache_free(c);
        return st;
    }
    *v.cache = c;
    return SAL_OK;
}

namespace {

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : 0.0f;
}

}  // namespace
}  // namespace sal

using namespace sal;

extern "C" {

void sal_smooth_params_default(sal_smooth_params *p) {
    if (!p) return;
    p->lambda = 0.4;
    p->mu = 0.4;
    p->xi_surface = 0.1;
    p->xi_volume = 0.9;
    p->max_iter_surface = 100;
    p->max_iter_volume = 100;
}

sal_status sal_tet_mesh_smooth(sal_context *ctx, sal_tet_mesh *m, const sal_smooth_params *params,
                               sal_smooth_info *info) {
    try {
        if (!ctx || !m) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
        if (mesh_device(m) != ctx->device) return set_error(SAL_ERR_INVALID_ARG, "mesh lives on another device");
        ConformView v{};
        if (!conform_view(m, &v)) return set_error(SAL_ERR_INVALID_ARG, "call sal_tet_mesh_conform first");
        sal_smooth_params p;
        sal_smooth_params_default(&p);
        if (params) p = *params;
        if (!(p.lambda > 0.0 && p.lambda < 1.0 && p.mu > 0.0 && p.mu < 1.0))
            return set_error(SAL_ERR_INVALID_ARG, "lambda and mu must lie in (0, 1)");
        SAL_HIP(hipSetDevice(ctx->device));
        hipStream_t s = ctx->stream;
        sal_status st;
        float ms_build = 0.0f;
        if (!*v.cache) {
            SAL_HIP(hipEventRecord(ctx->ev[0], s));
            if ((st = ensure_smooth_graph(v, s)) != SAL_OK) return st;
            SAL_HIP(hipEventRecord(ctx->ev[1], s));
            SAL_HIP(hipEventSynchronize(ctx->ev[1]));
            ms_build = elapsed_ms(ctx->ev[0], ctx->ev[1]);
        }
        SmoothCache *c = *v.cache;
        SAL_HIP(launch_pack_pos(v.xyz, c->order, v.n_nodes, c->pos[0], c->pos[1], s));
        int32_t it[2] = {0, 0};
        double ratio[2] = {0.0, 0.0};
        float ms[2] = {0.0f, 0.0f};
        const double xi[2] = {p.xi_surface, p.xi_volume};
        const int cap[2] = {p.max_iter_surface, p.max_iter_volume};
        for (int ph = 0; ph < 2; ++ph) {
            SAL_HIP(hipEventRecord(ctx->ev[2], s));
            if ((st = run_phase(c, ph, p.lambda, p.mu, xi[ph], cap[ph], &it[ph], &ratio[ph], s)) != SAL_OK)
                return st;
            SAL_HIP(hipEventRecord(ctx->ev[3], s));
            SAL_HIP(hipEventSynchronize(ctx->ev[3]));
            ms[ph] = elapsed_ms(ctx->ev[2], ctx->ev[3]);
        }
        SAL_HIP(launch_unpack_pos(c->pos[0], c->order, v.n_nodes, v.xyz, s));
        SAL_HIP(hipStreamSynchronize(s));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->n_edges = c->n_edges;
            info->n_surface_edges = c->n_surface_edges;
            info->n_surface_nodes = c->n_list[0];
            info->n_volume_nodes = c->n_list[1];
            info->iters_surface = it[0];
            info->iters_volume = it[1];
            info->ratio_surface = ratio[0];
            info->ratio_volume = ratio[1];
            info->ms_build = ms_build;
            info->ms_surface = ms[0];
            info->ms_volume = ms[1];
            info->n_entries_surface = c->n_entries[0];
            info->n_entries_volume = c->n_entries[1];
        }
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_tet_mesh_smooth");
    }
}

}  // extern "C"
