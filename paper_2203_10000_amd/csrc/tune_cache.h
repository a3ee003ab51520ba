// The launch-shape tuner's file cache (host only, no device calls).
#pragma once

#include <map>
#include <string>
#include <tuple>
#include <utility>

namespace sal {

// (device, precision, log2 triangles, log2 trial points, arch name, requested
// points per lane, requested wavefronts per workgroup)
using TuneKey = std::tuple<int, int, int, int, std::string, int, int>;
// -> (points per lane, wavefronts per workgroup)
using TuneMap = std::map<TuneKey, std::pair<int, int>>;

// One entry per line: "arch dev prec tb nb rp rb ppl bw".  Reading stops at
// the first line that does not parse (or has an arch name over 127 bytes)
// and keeps the entries before it; a missing file reads as empty.
bool tune_cache_read(const char *path, TuneMap *out);
bool tune_cache_write(const char *path, const TuneMap &m);

}  // namespace sal
