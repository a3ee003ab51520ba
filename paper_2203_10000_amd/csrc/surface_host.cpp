// Host side of surface-set construction, with no device call: validation
// of closed oriented manifolds, greedy triangle strips, the float32 /
// float64 strip records and the per-surface table.  Kept apart from the
// upload so that validation runs (and is tested) without a GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "surface_host.h"

namespace sal {

namespace {

inline uint64_t edge_key(uint32_t a, uint32_t b) { return ((uint64_t)a << 32) | b; }

struct HostSurface {
    const float *xyz;
    int64_t nv, nt;
    std::vector<int32_t> tri;  // possibly reoriented copy
    int32_t label;
};

// One strip: the vertex sequence and, per triangle, its index in the surface.
struct Strip {
    std::vector<int32_t> verts;
    std::vector<int32_t> tris;
};

sal_status validate(HostSurface &s, int idx, bool auto_orient) {
    const std::string who = "surface " + std::to_string(idx) + ": ";
    if (s.nv < 3 || s.nt < 4 || !s.xyz || s.tri.empty())
        return set_error(SAL_ERR_INVALID_ARG, who + "needs >= 3 vertices and >= 4 triangles");
    if (s.label <= 0) return set_error(SAL_ERR_INVALID_ARG, who + "label must be > 0");
    if (s.nt > (int64_t)1 << 30 || s.nv > (int64_t)1 << 30)
        return set_error(SAL_ERR_CAPACITY, who + "more than 2^30 vertices or triangles");
    for (int64_t i = 0; i < 3 * s.nv; ++i)
        if (!std::isfinite(s.xyz[i]))
            return set_error(SAL_ERR_INVALID_ARG, who + "non-finite vertex coordinate");
    std::unordered_map<uint64_t, int64_t> dir;
    dir.reserve((size_t)(3 * s.nt * 2));
    for (int64_t t = 0; t < s.nt; ++t) {
        const int32_t *f = &s.tri[3 * t];
        for (int c = 0; c < 3; ++c)
            if (f[c] < 0 || f[c] >= s.nv)
                return set_error(SAL_ERR_INVALID_ARG, who + "vertex index out of range");
        if (f[0] == f[1] || f[1] == f[2] || f[0] == f[2])
            return set_error(SAL_ERR_INVALID_ARG, who + "triangle repeats a vertex");
        const float *A = s.xyz + 3 * f[0], *B = s.xyz + 3 * f[1], *C = s.xyz + 3 * f[2];
        const double e1[3] = {(double)B[0] - A[0], (double)B[1] - A[1], (double)B[2] - A[2]};
        const double e2[3] = {(double)C[0] - A[0], (double)C[1] - A[1], (double)C[2] - A[2]};
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0)
            return set_error(SAL_ERR_INVALID_ARG, who + "zero-area triangle");
        for (int c = 0; c < 3; ++c) {
            const uint64_t k = edge_key((uint32_t)f[c], (uint32_t)f[(c + 1) % 3]);
            if (!dir.emplace(k, t).second)
                return set_error(SAL_ERR_NOT_CLOSED, who + "a directed edge is used twice");
        }
    }
    for (const auto &kv : dir) {
        const uint32_t a = (uint32_t)(kv.first >> 32), b = (uint32_t)kv.first;
        if (!dir.count(edge_key(b, a)))
            return set_error(SAL_ERR_NOT_CLOSED, who + "boundary edge (surface is open)");
    }
    // enclosed volume, about the vertex centroid for accuracy
    double c[3] = {0, 0, 0};
    for (int64_t i = 0; i < s.nv; ++i)
        for (int d = 0; d < 3; ++d) c[d] += s.xyz[3 * i + d];
    for (int d = 0; d < 3; ++d) c[d] /= (double)s.nv;
    double vol = 0.0;
    for (int64_t t = 0; t < s.nt; ++t) {
        const int32_t *f = &s.tri[3 * t];
        double v[3][3];
        for (int r = 0; r < 3; ++r)
            for (int d = 0; d < 3; ++d) v[r][d] = (double)s.xyz[3 * f[r] + d] - c[d];
        vol += v[0][0] * (v[1][1] * v[2][2] - v[1][2] * v[2][1]) +
               v[0][1] * (v[1][2] * v[2][0] - v[1][0] * v[2][2]) +
               v[0][2] * (v[1][0] * v[2][1] - v[1][1] * v[2][0]);
    }
    if (!(vol != 0.0)) return set_error(SAL_ERR_ORIENTATION, who + "encloses zero volume");
    if (vol < 0.0) {
        if (!auto_orient)
            return set_error(SAL_ERR_ORIENTATION,
                             who + "triangles are clockwise seen from outside (negative volume)");
        for (int64_t t = 0; t < s.nt; ++t) std::swap(s.tri[3 * t + 1], s.tri[3 * t + 2]);
    }
    return SAL_OK;
}

// Greedy strips: from each unused seed triangle try the three rotations,
// walk across the edge formed by the two newest vertices while the next
// triangle is unused, and keep the longest walk.
std::vector<Strip> make_strips(const HostSurface &s) {
    const int64_t nt = s.nt;
    std::unordered_map<uint64_t, int32_t> dir;
    dir.reserve((size_t)(3 * nt * 2));
    for (int64_t t = 0; t < nt; ++t)
        for (int c = 0; c < 3; ++c)
            dir[edge_key((uint32_t)s.tri[3 * t + c], (uint32_t)s.tri[3 * t + (c + 1) % 3])] =
                (int32_t)t;
    auto across = [&](int32_t cur, int32_t a, int32_t b) -> int32_t {
        auto it = dir.find(edge_key((uint32_t)a, (uint32_t)b));
        int32_t t1 = it == dir.end() ? -1 : it->second;
        if (t1 != cur) return t1;
        auto it2 = dir.find(edge_key((uint32_t)b, (uint32_t)a));
        return it2 == dir.end() ? -1 : it2->second;
    };
    auto third = [&](int32_t t, int32_t a, int32_t b) -> int32_t {
        for (int c = 0; c < 3; ++c) {
            const int32_t v = s.tri[3 * t + c];
            if (v != a && v != b) return v;
        }
        return -1;
    };
    std::vector<uint8_t> used((size_t)nt, 0);
    std::vector<int32_t> stamp((size_t)nt, -1);
    std::vector<Strip> out;
    int32_t attempt = 0;
    for (int64_t seed = 0; seed < nt; ++seed) {
        if (used[seed]) continue;
        int best_rot = 0;
        int64_t best_len = -1;
        for (int rot = 0; rot < 3; ++rot) {
            ++attempt;
            int32_t y = s.tri[3 * seed + (rot + 1) % 3], z = s.tri[3 * seed + (rot + 2) % 3];
            int32_t cur = (int32_t)seed;
            stamp[cur] = attempt;
            int64_t len = 1;
            for (;;) {
                const int32_t nb = across(cur, y, z);
                if (nb < 0 || used[nb] || stamp[nb] == attempt) break;
                stamp[nb] = attempt;
                const int32_t w = third(nb, y, z);
                y = z;
                z = w;
                cur = nb;
                ++len;
            }
            if (len > best_len) { best_len = len; best_rot = rot; }
        }
        Strip st;
        const int32_t x0 = s.tri[3 * seed + best_rot], y0 = s.tri[3 * seed + (best_rot + 1) % 3],
                      z0 = s.tri[3 * seed + (best_rot + 2) % 3];
        st.verts = {x0, y0, z0};
        st.tris = {(int32_t)seed};
        used[seed] = 1;
        int32_t y = y0, z = z0, cur = (int32_t)seed;
        for (;;) {
            const int32_t nb = across(cur, y, z);
            if (nb < 0 || used[nb]) break;
            used[nb] = 1;
            const int32_t w = third(nb, y, z);
            st.verts.push_back(w);
            st.tris.push_back(nb);
            y = z;
            z = w;
            cur = nb;
        }
        out.push_back(std::move(st));
    }
    return out;
}

// +1 when (p, q, r) is a rotation of the triangle's stored order, else -1.
double parity(const int32_t *f, int32_t p, int32_t q, int32_t r) {
    for (int c = 0; c < 3; ++c)
        if (f[c] == p && f[(c + 1) % 3] == q && f[(c + 2) % 3] == r) return 1.0;
    return -1.0;
}

// Squared distance from p to triangle (a, b, c), in double: the closest
// point found by the Voronoi-region walk over vertices, edges and face
// (Ericson, Real-Time Collision Detection, section 5.1.5).
double dist2_point_triangle(const double p[3], const double a[3], const double b[3], const double c[3]) {
    auto sub = [](const double *u, const double *v, double *o) {
        for (int k = 0; k < 3; ++k) o[k] = u[k] - v[k];
    };
    auto dot = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    double ab[3], ac[3], ap[3], q[3];
    sub(b, a, ab);
    sub(c, a, ac);
    sub(p, a, ap);
    const double d1 = dot(ab, ap), d2 = dot(ac, ap);
    auto at = [&](double u, double v) {   // a + u ab + v ac
        for (int k = 0; k < 3; ++k) q[k] = a[k] + u * ab[k] + v * ac[k];
    };
    if (d1 <= 0 && d2 <= 0) {
        at(0, 0);
    } else {
        double bp[3];
        sub(p, b, bp);
        const double d3 = dot(ab, bp), d4 = dot(ac, bp);
        if (d3 >= 0 && d4 <= d3) {
            at(1, 0);
        } else {
            const double vc = d1 * d4 - d3 * d2;
            if (vc <= 0 && d1 >= 0 && d3 <= 0) {
                at(d1 / (d1 - d3), 0);
            } else {
                double cp[3];
                sub(p, c, cp);
                const double d5 = dot(ab, cp), d6 = dot(ac, cp);
                if (d6 >= 0 && d5 <= d6) {
                    at(0, 1);
                } else {
                    const double vb = d5 * d2 - d1 * d6;
                    if (vb <= 0 && d2 >= 0 && d6 <= 0) {
                        at(0, d2 / (d2 - d6));
                    } else {
                        const double va = d3 * d6 - d5 * d4;
                        if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
                            const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
                            at(1 - w, w);
                        } else {
                            const double den = 1.0 / (va + vb + vc);
                            at(vb * den, vc * den);
                        }
                    }
                }
            }
        }
    }
    double d[3];
    sub(p, q, d);
    return dot(d, d);
}

}  // namespace


sal_status build_surface_records(const sal_surface_desc *desc, int32_t n, uint32_t flags,
                                 SurfaceRecords *rec) {
    if (!desc || !rec) return set_error(SAL_ERR_INVALID_ARG, "NULL argument");
    if (n < 1 || n > kMaxSurfaces)
        return set_error(SAL_ERR_INVALID_ARG, "n_surfaces must be in 1..64");
    std::vector<Rec32> &r32 = rec->r32;
    std::vector<Rec64> &r64 = rec->r64;
    std::vector<int64_t> &strip_off = rec->strip_off;
    std::vector<int32_t> &strip_tris = rec->strip_tris;
    std::vector<SurfaceDev> &table = rec->table;
    r32.clear();
    r64.clear();
    strip_off.clear();
    strip_tris.clear();
    table.assign((size_t)n, SurfaceDev{});
    int64_t &total_tri = rec->total_tri;
    total_tri = 0;
    for (int32_t i = 0; i < n; ++i) {
        HostSurface hs;
        hs.xyz = desc[i].xyz;
        hs.nv = desc[i].n_vertices;
        hs.nt = desc[i].n_triangles;
        hs.label = desc[i].label;
        if (hs.nt < 4 || !desc[i].tri || !desc[i].xyz)
            return set_error(SAL_ERR_INVALID_ARG,
                             "surface " + std::to_string(i) + ": needs >= 4 triangles");
        hs.tri.assign(desc[i].tri, desc[i].tri + 3 * hs.nt);
        sal_status st = validate(hs, i, (flags & SAL_SURF_AUTO_ORIENT) != 0);
        if (st != SAL_OK) return st;
        const std::vector<Strip> strips = make_strips(hs);
        SurfaceDev &sd = table[(size_t)i];
        sd.rec_begin = (int64_t)r32.size();
        sd.strip_begin = (int64_t)strip_off.size();
        sd.n_tri = hs.nt;
        sd.label = hs.label;
        sd.pad = 0;
        for (int c = 0; c < 3; ++c) {
            sd.lo[c] = INFINITY;
            sd.hi[c] = -INFINITY;
        }
        for (int64_t v = 0; v < hs.nv; ++v)
            for (int c = 0; c < 3; ++c) {
                sd.lo[c] = std::min(sd.lo[c], hs.xyz[3 * v + c]);
                sd.hi[c] = std::max(sd.hi[c], hs.xyz[3 * v + c]);
            }
        // a ball about the vertex mean (rounded to float) that the surface
        // does not cross: radius = distance to the nearest triangle, less a
        // margin far above the rounding of the device's float distance test
        {
            double m[3] = {0, 0, 0};
            for (int64_t v = 0; v < hs.nv; ++v)
                for (int c = 0; c < 3; ++c) m[c] += hs.xyz[3 * v + c];
            double cen[3];
            for (int c = 0; c < 3; ++c) {
                sd.ball[c] = (float)(m[c] / (double)hs.nv);
                cen[c] = sd.ball[c];
            }
            double r2 = INFINITY;
            for (int64_t t = 0; t < hs.nt; ++t) {
                double P[3][3];
                for (int q = 0; q < 3; ++q)
                    for (int c = 0; c < 3; ++c) P[q][c] = hs.xyz[3 * (int64_t)hs.tri[3 * t + q] + c];
                r2 = std::min(r2, dist2_point_triangle(cen, P[0], P[1], P[2]));
            }
            const double scale = std::max({std::fabs(cen[0]), std::fabs(cen[1]), std::fabs(cen[2])});
            const double r = std::sqrt(r2) - 1e-5 * (std::sqrt(r2) + scale);
            sd.ball[3] = r > 0 ? (float)(r * r * (1.0 - 1e-6)) : 0.0f;
            sd.ball_w = -1;   // set by ensure_surface_balls, on first use
            sd.pad2 = 0;
        }
        total_tri += hs.nt;
        const float *V = hs.xyz;
        for (const Strip &s : strips) {
            strip_off.push_back((int64_t)r32.size());
            const int m = (int)s.tris.size();
            strip_tris.push_back(m);
            Rec32 h32{};
            Rec64 h64{};
            for (int c = 0; c < 3; ++c) {
                h32.v[c] = V[3 * s.verts[0] + c];
                h32.v[3 + c] = V[3 * s.verts[1] + c];
                h64.v[c] = V[3 * s.verts[0] + c];
                h64.v[3 + c] = V[3 * s.verts[1] + c];
            }
            int32_t mi = m;
            std::memcpy(&h32.v[6], &mi, 4);
            int64_t ml = m;
            std::memcpy(&h64.v[6], &ml, 8);
            r32.push_back(h32);
            r64.push_back(h64);
            for (int t = 0; t < m; ++t) {
                const int32_t *f = &hs.tri[3 * (size_t)s.tris[t]];
                const float *A = V + 3 * f[0], *B = V + 3 * f[1], *C = V + 3 * f[2];
                const double e1[3] = {(double)B[0] - A[0], (double)B[1] - A[1], (double)B[2] - A[2]};
                const double e2[3] = {(double)C[0] - A[0], (double)C[1] - A[1], (double)C[2] - A[2]};
                const double nn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                      e1[0] * e2[1] - e1[1] * e2[0]};
                const double nlen = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
                const double nb = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]) *
                                  std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
                const int32_t z = s.verts[t + 2];
                Rec32 q32{};
                Rec64 q64{};
                for (int c = 0; c < 3; ++c) {
                    q32.v[c] = V[3 * z + c];
                    q32.v[3 + c] = (float)(kNScale * nn[c]);
                    q64.v[c] = V[3 * z + c];
                    q64.v[3 + c] = nn[c];
                }
                q32.v[6] = (float)nlen;
                q32.v[7] = (float)(kKnSmall * nlen);
                // the exact-sign guard's bound factor: 32 eps |B - A||C - A| (a
                // power-of-two scaling, so exact), slightly enlarged
                q64.v[6] = kGuardEps * (nb * (1.0 + 1e-12));
                q64.v[7] = parity(f, s.verts[t], s.verts[t + 1], s.verts[t + 2]);
                r32.push_back(q32);
                r64.push_back(q64);
            }
        }
        sd.rec_end = (int64_t)r32.size();
        sd.strip_end = (int64_t)strip_off.size();
    }

    // Extra table entries for the launch-shape tuner: the leading whole
    // strips of the record stream up to about kTuneTri[i] triangles, so that
    // a trial launch costs a bounded number of pairs on any mesh.
    for (int i = 0; i < kTuneEntries; ++i) {
        SurfaceDev t{};
        int64_t s = 0, tris = 0;
        while (s < (int64_t)strip_off.size() && tris < kTuneTri[i]) tris += strip_tris[(size_t)s++];
        t.rec_begin = 0;
        t.rec_end = s < (int64_t)strip_off.size() ? strip_off[(size_t)s] : (int64_t)r32.size();
        t.strip_begin = 0;
        t.strip_end = s;
        t.n_tri = tris;
        t.label = 1;
        for (int c = 0; c < 3; ++c) {
            t.lo[c] = -INFINITY;
            t.hi[c] = INFINITY;
        }
        t.ball_w = -1;
        table.push_back(t);
    }
    return SAL_OK;
}

}  // namespace sal

extern "C" sal_status sal_surface_set_check(const sal_surface_desc *surfaces, int32_t n_surfaces,
                                            uint32_t flags, sal_surface_set_info *info) {
    try {
        sal::SurfaceRecords rec;
        const sal_status st = sal::build_surface_records(surfaces, n_surfaces, flags, &rec);
        if (st != SAL_OK) return st;
        if (info) {
            info->n_surfaces = n_surfaces;
            info->n_triangles = rec.total_tri;
            info->n_strips = (int64_t)rec.strip_off.size();
            info->device_bytes = (int64_t)(rec.r32.size() * sizeof(sal::Rec32) +
                                           rec.r64.size() * sizeof(sal::Rec64) +
                                           rec.table.size() * sizeof(sal::SurfaceDev) +
                                           rec.strip_off.size() * sizeof(int64_t));
        }
        return SAL_OK;
    } catch (const std::bad_alloc &) {
        return sal::set_error(SAL_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return sal::set_error(SAL_ERR_INTERNAL, "exception in sal_surface_set_check");
    }
}
