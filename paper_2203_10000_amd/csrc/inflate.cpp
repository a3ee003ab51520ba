// Inflation of the compartment boundaries (paper section 2.2.2): host side.
// Per call the surface set's strips are unrolled into float32 triangles and
// binned on the level-0 lattice; the interface nodes of the conforming mesh
// then move in one launch that reads the positions from before the call.
#include <algorithm>
#include <cstring>
#include <vector>

#include "post_internal.h"
#include "runtime.h"

namespace sal {
namespace {

struct Buffers {
    std::vector<void *> p;
    ~Buffers() {
        for (void *q : p) (void)hipFree(q);
    }
    template <typename T>
    sal_status get(T **out, int64_t n) {
        if (dev_malloc((void **)out, (size_t)std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess)
            return set_error(SAL_ERR_OUT_OF_MEMORY, "hipMalloc(inflation)");
        p.push_back(*out);
        return SAL_OK;
    }
};

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : 0.0f;
}

}  // namespace
}  // namespace sal

using namespace sal;

extern "C" {

sal_status sal_tet_mesh_inflate(sal_context *ctx, sal_tet_mesh *m, const sal_surface_set *set, double zeta,
                                sal_inflate_info *info) {
    try {
        if (!ctx || !m || !set) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
        if (mesh_device(m) != ctx->device || set->device != ctx->device)
            return set_error(SAL_ERR_INVALID_ARG, "mesh or surfaces live on another device");
        if (!(zeta >= 0.0 && zeta < 1.0)) return set_error(SAL_ERR_INVALID_ARG, "zeta must lie in [0, 1)");
        ConformView v{};
        if (!conform_view(m, &v)) return set_error(SAL_ERR_INVALID_ARG, "call sal_tet_mesh_conform first");
        const int64_t n_bins = (int64_t)v.g.cells[0] * v.g.cells[1] * v.g.cells[2];
        if (n_bins + 1 > INT32_MAX) return set_error(SAL_ERR_CAPACITY, "inflation: too many lattice cells");
        SAL_HIP(hipSetDevice(ctx->device));
        hipStream_t s = ctx->stream;
        sal_status st;
        SAL_HIP(hipEventRecord(ctx->ev[0], s));
        if ((st = ensure_smooth_graph(v, s)) != SAL_OK) return st;
        SmoothCache *c = *v.cache;
        Buffers b;
        // triangles, first index of each strip's
        std::vector<int64_t> base(set->host_strip_tris.size());
        int64_t n_tri = 0;
        for (size_t k = 0; k < base.size(); ++k) {
            base[k] = n_tri;
            n_tri += set->host_strip_tris[k];
        }
        int64_t *tri_base = nullptr;
        float *tri = nullptr;
        if ((st = b.get(&tri_base, (int64_t)base.size())) != SAL_OK || (st = b.get(&tri, 9 * n_tri)) != SAL_OK)
            return st;
        SAL_HIP(hipMemcpyAsync(tri_base, base.data(), base.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        SAL_HIP(launch_strip_triangles(set->rec64, set->strip_off, tri_base, (int64_t)base.size(), tri, s));
        // bins: count, scan, place
        int32_t *count = nullptr, *items = nullptr;
        int64_t *start = nullptr;
        if ((st = b.get(&count, n_bins + 1)) != SAL_OK || (st = b.get(&start, n_bins + 1)) != SAL_OK) return st;
        SAL_HIP(launch_fill_i32(count, 0, n_bins + 1, s));
        SAL_HIP(launch_bin_triangles(tri, n_tri, v.g, 0, count, nullptr, nullptr, s));
        size_t tb = 0;
        SAL_HIP(exclusive_sum_bins(count, start, n_bins + 1, nullptr, &tb, s));
        char *tmp = nullptr;
        if ((st = b.get(&tmp, (int64_t)tb)) != SAL_OK) return st;
        SAL_HIP(exclusive_sum_bins(count, start, n_bins + 1, tmp, &tb, s));
        int64_t n_items = 0;
        SAL_HIP(hipMemcpyAsync(&n_items, start + n_bins, sizeof(n_items), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        if ((st = b.get(&items, n_items)) != SAL_OK) return st;
        SAL_HIP(launch_fill_i32(count, 0, n_bins + 1, s));
        SAL_HIP(launch_bin_triangles(tri, n_tri, v.g, 1, count, start, items, s));
        float *bin_tri = nullptr;
        if ((st = b.get(&bin_tri, 9 * n_items)) != SAL_OK) return st;
        SAL_HIP(launch_gather_binned(tri, items, n_items, bin_tri, s));
        SAL_HIP(hipEventRecord(ctx->ev[1], s));
        // move the interface nodes
        const int64_t n = c->n_list[0];
        double *partials = nullptr, *sums = nullptr;
        if ((st = b.get(&partials, 2 * inflate_blocks(n))) != SAL_OK || (st = b.get(&sums, 2)) != SAL_OK)
            return st;
        SAL_HIP(launch_pack_pos(v.xyz, c->order, v.n_nodes, c->pos[0], c->pos[1], s));
        SAL_HIP(launch_inflate(c->pos[0], c->pos[1], c->seg[0], c->cols, c->list[0], n, c->order, v.keys,
                               bin_tri, start, v.g, zeta, partials, sums, s));
        SAL_HIP(hipEventRecord(ctx->ev[2], s));
        SAL_HIP(launch_unpack_pos(c->pos[1], c->order, v.n_nodes, v.xyz, s));
        double hs[2] = {0.0, 0.0};
        SAL_HIP(hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, s));
        SAL_HIP(hipStreamSynchronize(s));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->n_candidates = n;
            info->n_moved = (int64_t)hs[0];
            info->n_edges_tested = c->n_entries[0];
            info->n_triangle_tests = (int64_t)hs[1];
            info->n_triangles = n_tri;
            info->n_bin_items = n_items;
            info->ms_prepare = elapsed_ms(ctx->ev[0], ctx->ev[1]);
            info->ms_inflate = elapsed_ms(ctx->ev[1], ctx->ev[2]);
        }
        return SAL_OK;
    } catch (...) {
        return set_error(SAL_ERR_INTERNAL, "exception in sal_tet_mesh_inflate");
    }
}

}  // extern "C"
