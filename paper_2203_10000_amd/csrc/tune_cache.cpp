// The launch-shape tuner's file cache: plain text, one entry per line.
#include "tune_cache.h"

#include <cstdio>

namespace sal {

bool tune_cache_read(const char *path, TuneMap *out) {
    if (!path || !out) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char arch[128];
    int dev, prec, tb, nb, rp, rb, ppl, bw;
    while (std::fscanf(f, "%127s %d %d %d %d %d %d %d %d", arch, &dev, &prec, &tb, &nb, &rp, &rb,
                       &ppl, &bw) == 9)
        (*out)[TuneKey(dev, prec, tb, nb, arch, rp, rb)] = {ppl, bw};
    std::fclose(f);
    return true;
}

bool tune_cache_write(const char *path, const TuneMap &m) {
    if (!path) return false;
    FILE *f = std::fopen(path, "w");
    if (!f) return false;
    for (const auto &kv : m)
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", std::get<4>(kv.first).c_str(),
                     std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                     std::get<3>(kv.first), std::get<5>(kv.first), std::get<6>(kv.first),
                     kv.second.first, kv.second.second);
    return std::fclose(f) == 0;
}

}  // namespace sal
