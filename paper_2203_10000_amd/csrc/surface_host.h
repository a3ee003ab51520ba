// Host-only surface-set construction (no device calls).
#pragma once

#include <cstdint>
#include <vector>

#include "sal_internal.h"

namespace sal {

// Everything a surface set uploads: strip records in both precisions, the
// record index and triangle count of every strip, and the per-surface table
// (n entries, then the tuner's two entries).
struct SurfaceRecords {
    std::vector<Rec32> r32;
    std::vector<Rec64> r64;
    std::vector<int64_t> strip_off;
    std::vector<int32_t> strip_tris;
    std::vector<SurfaceDev> table;
    int64_t total_tri = 0;
};

// Validates the surfaces (section 2.1.3: closed, consistently oriented
// boundaries; SAL_SURF_AUTO_ORIENT reverses inward ones) and builds their
// records.  Errors as sal_surface_set_create's, with nothing built.
sal_status build_surface_records(const sal_surface_desc *desc, int32_t n, uint32_t flags,
                                 SurfaceRecords *rec);

}  // namespace sal
