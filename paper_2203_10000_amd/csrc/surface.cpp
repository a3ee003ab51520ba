// Surface-set construction: validation of closed oriented manifolds, greedy
// triangle strips, float32 / float64 strip records on the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <unordered_map>
#include <vector>

#include "runtime.h"
#include "surface_host.h"

namespace sal {

sal_status build_surface_set(sal_context *ctx, const sal_surface_desc *desc, int32_t n,
                             uint32_t flags, sal_surface_set **out) {
    if (!ctx || !desc || !out) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
    SurfaceRecords rec;
    sal_status st0 = build_surface_records(desc, n, flags, &rec);
    if (st0 != SAL_OK) return st0;
    const std::vector<Rec32> &r32 = rec.r32;
    const std::vector<Rec64> &r64 = rec.r64;
    const std::vector<int64_t> &strip_off = rec.strip_off;
    const std::vector<int32_t> &strip_tris = rec.strip_tris;
    const std::vector<SurfaceDev> &table = rec.table;
    const int64_t total_tri = rec.total_tri;
    SAL_HIP(hipSetDevice(ctx->device));
    static std::atomic<uint64_t> next_uid{1};
    auto *set = new sal_surface_set();
    set->uid = next_uid++;
    set->device = ctx->device;
    set->n_surf = n;
    set->n_tri = total_tri;
    set->n_strips = (int64_t)strip_off.size();
    set->n_rec = (int64_t)r32.size();
    set->host_table.assign(table.begin(), table.begin() + n);
    set->host_strip_off = strip_off;
    set->host_strip_tris = strip_tris;
    sal_status st = SAL_OK;
    auto up = [&](void **dst, const void *src, size_t bytes) -> sal_status {
        hipError_t e = dev_malloc(dst, bytes);
        if (e != hipSuccess) return hip_error(e, "hipMalloc(surface set)");
        e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_error(e, "hipMemcpy(surface set)");
        set->bytes += bytes;
        return SAL_OK;
    };
    if ((st = up((void **)&set->rec32, r32.data(), r32.size() * sizeof(Rec32))) != SAL_OK ||
        (st = up((void **)&set->rec64, r64.data(), r64.size() * sizeof(Rec64))) != SAL_OK ||
        (st = up((void **)&set->surf, table.data(), table.size() * sizeof(SurfaceDev))) != SAL_OK ||
        (st = up((void **)&set->strip_off, strip_off.data(), strip_off.size() * sizeof(int64_t))) !=
            SAL_OK) {
        destroy_surface_set(set);
        return st;
    }
    set->tune_surf = set->surf + n;
    *out = set;
    return SAL_OK;
}

sal_status ensure_surface_balls(sal_context *ctx, const sal_surface_set *cset) {
    auto *set = const_cast<sal_surface_set *>(cset);
    if (set->balls_ready) return SAL_OK;
    const int n = set->n_surf;
    std::vector<SurfaceDev> table = set->host_table;
    std::vector<float> c(3 * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) c[(size_t)(a * n + i)] = table[(size_t)i].ball[a];
    float *dc = nullptr;
    int32_t *dl = nullptr;
    unsigned long long *dm = nullptr;
    std::vector<unsigned long long> masks((size_t)n, 0);
    hipError_t e = dev_malloc((void **)&dc, c.size() * sizeof(float));
    if (e == hipSuccess) e = dev_malloc((void **)&dl, (size_t)n * sizeof(int32_t));
    if (e == hipSuccess) e = dev_malloc((void **)&dm, (size_t)n * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemcpy(dc, c.data(), c.size() * sizeof(float), hipMemcpyHostToDevice);
    // each centre against its own surface only: one FP64 launch per surface
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        PairloopArgs a{};
        a.rec32 = set->rec32;
        a.rec64 = set->rec64;
        a.surf = set->surf + i;
        a.n_surf = 1;
        a.x = dc + i;
        a.y = dc + n + i;
        a.z = dc + 2 * n + i;
        a.n = 1;
        a.kappa = 0.03125f;
        a.threshold = 0.5;
        a.band = 0.0;
        a.labels = dl + i;
        a.masks = dm + i;
        a.counters = ctx->counters;
        e = launch_pairloop_f64(a, 1, ctx->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipMemcpy(masks.data(), dm, (size_t)n * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (dc) (void)hipFree(dc);
    if (dl) (void)hipFree(dl);
    if (dm) (void)hipFree(dm);
    if (e != hipSuccess) return hip_error(e, "surface ball centres");
    for (int i = 0; i < n; ++i) {
        SurfaceDev &sd = table[(size_t)i];
        sd.ball_w = sd.ball[3] > 0.0f ? (int32_t)(masks[(size_t)i] & 1ull) : -1;
    }
    e = hipMemcpy(set->surf, table.data(), (size_t)n * sizeof(SurfaceDev), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "hipMemcpy(surface table)");
    set->host_table = table;
    set->balls_ready = true;
    return SAL_OK;
}

void destroy_surface_set(sal_surface_set *set) {
    if (!set) return;
    (void)hipSetDevice(set->device);
    if (set->rec32) (void)hipFree(set->rec32);
    if (set->rec64) (void)hipFree(set->rec64);
    if (set->surf) (void)hipFree(set->surf);
    if (set->strip_off) (void)hipFree(set->strip_off);
    delete set;
}

}  // namespace sal
