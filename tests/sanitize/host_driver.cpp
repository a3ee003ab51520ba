// Runs the host-only parts of libsal (surface validation and strip building
// through sal_surface_set_check, the tuner's cache file) on inputs written by
// the test, for a build under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// argv[1]: cases, little-endian: int32 n_cases; per case int32 flags,
//          int32 n_surf; per surface int64 nv, int64 nt, int32 label,
//          float xyz[3 nv], int32 tri[3 nt]
// argv[2]: output: per case int32 status, int32 n_surfaces, int64
//          n_triangles, int64 n_strips, int64 device_bytes
// argv[3]: a tuner cache file to read; argv[4]: where to write it back;
//          the entry count is printed.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "sal.h"
#include "tune_cache.h"

namespace sal {
// libsal's error sink lives with the device code; the driver keeps the last message
static std::string g_msg;
sal_status set_error(sal_status s, const std::string &msg) {
    g_msg = msg;
    return s;
}
}  // namespace sal

static bool rd(FILE *f, void *p, size_t bytes) { return !bytes || fread(p, 1, bytes, f) == bytes; }

int main(int argc, char **argv) {
    if (argc != 5) return 2;
    FILE *in = std::fopen(argv[1], "rb");
    FILE *out = std::fopen(argv[2], "wb");
    if (!in || !out) return 2;
    int32_t n_cases = 0;
    if (!rd(in, &n_cases, 4)) return 2;
    for (int c = 0; c < n_cases; ++c) {
        int32_t flags = 0, ns = 0;
        if (!rd(in, &flags, 4) || !rd(in, &ns, 4) || ns < 0 || ns > 100) return 2;
        std::vector<std::vector<float>> xyz((size_t)ns);
        std::vector<std::vector<int32_t>> tri((size_t)ns);
        std::vector<sal_surface_desc> desc((size_t)ns);
        for (int s = 0; s < ns; ++s) {
            int64_t nv = 0, nt = 0;
            int32_t label = 0;
            if (!rd(in, &nv, 8) || !rd(in, &nt, 8) || !rd(in, &label, 4)) return 2;
            xyz[s].resize((size_t)(3 * nv));
            tri[s].resize((size_t)(3 * nt));
            if (!rd(in, xyz[s].data(), 12 * (size_t)nv) || !rd(in, tri[s].data(), 12 * (size_t)nt))
                return 2;
            desc[s].n_vertices = nv;
            desc[s].xyz = xyz[s].data();
            desc[s].n_triangles = nt;
            desc[s].tri = tri[s].data();
            desc[s].label = label;
        }
        sal_surface_set_info info{};
        const int32_t st = sal_surface_set_check(ns ? desc.data() : nullptr, ns, (uint32_t)flags, &info);
        std::fwrite(&st, 4, 1, out);
        std::fwrite(&info.n_surfaces, 4, 1, out);
        std::fwrite(&info.n_triangles, 8, 1, out);
        std::fwrite(&info.n_strips, 8, 1, out);
        std::fwrite(&info.device_bytes, 8, 1, out);
    }
    std::fclose(in);
    std::fclose(out);
    sal::TuneMap m;
    sal::tune_cache_read(argv[3], &m);
    if (!sal::tune_cache_write(argv[4], m)) return 3;
    sal::TuneMap again;
    sal::tune_cache_read(argv[4], &again);
    std::printf("tune entries %zu %zu\n", m.size(), again.size());
    return again == m ? 0 : 4;
}
