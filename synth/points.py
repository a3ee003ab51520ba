"""Query point sets (float32 SoA arrays of shape [3, N])."""
import numpy as np


def uniform_box(rng, n, lo, hi):
    """n points uniform in the cube [lo, hi]^3."""
    return rng.uniform(lo, hi, (3, n)).astype(np.float32)


def _unit_normals(v, f):
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(b - a, c - a)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def near_surface_points(rng, surfaces, n, max_offset):
    """Surface uniform among `surfaces`, triangle uniform by index, point
    uniform in the triangle (square-root trick), then an offset drawn
    U[-max_offset, max_offset] mm along the unit face normal.  Built in float64
    and rounded once to float32."""
    out = np.empty((3, n), dtype=np.float32)
    which = rng.integers(0, len(surfaces), n)
    for k, s in enumerate(surfaces):
        idx = np.nonzero(which == k)[0]
        if idx.size == 0:
            continue
        v = s.v.astype(np.float64)
        f = s.f
        t = rng.integers(0, f.shape[0], idx.size)
        r1 = np.sqrt(rng.uniform(0.0, 1.0, idx.size))
        r2 = rng.uniform(0.0, 1.0, idx.size)
        a, b, c = v[f[t, 0]], v[f[t, 1]], v[f[t, 2]]
        p = ((1 - r1)[:, None] * a + (r1 * (1 - r2))[:, None] * b
             + (r1 * r2)[:, None] * c)
        nrm = _unit_normals(v, f[t])
        d = rng.uniform(-max_offset, max_offset, idx.size)
        out[:, idx] = (p + d[:, None] * nrm).T.astype(np.float32)
    return out


def precision_ladder(surface, rng, n_sites=64, offsets=(1e-9, 1e-8, 1e-7, 1e-6, 1e-5,
                                                          1e-4, 1e-3)):
    """Points at +-offset (mm) along the face normal from face interiors, edge
    midpoints and vertices of random sites on `surface`.  Returns float32 [3, N]."""
    v = surface.v.astype(np.float64)
    f = surface.f
    t = rng.integers(0, f.shape[0], n_sites)
    a, b, c = v[f[t, 0]], v[f[t, 1]], v[f[t, 2]]
    nrm = _unit_normals(v, f[t])
    w = rng.dirichlet((2.0, 2.0, 2.0), n_sites)
    bases = [w[:, :1] * a + w[:, 1:2] * b + w[:, 2:] * c,   # face interior
             0.5 * (a + b),                                  # edge midpoint
             a]                                              # vertex
    pts = []
    for base in bases:
        for off in offsets:
            for sgn in (-1.0, 1.0):
                pts.append(base + sgn * off * nrm)
    return np.concatenate(pts).T.astype(np.float32)


def face_centroids_on_surface(surface, count=None):
    """Points lying exactly on the surface: its vertices plus every edge
    midpoint that float32 represents exactly."""
    v = surface.v.astype(np.float64)
    f = surface.f
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    m = 0.5 * (v[e[:, 0]] + v[e[:, 1]])
    exact = np.all(m.astype(np.float32).astype(np.float64) == m, axis=1)
    pts = np.concatenate([v, m[exact]])
    if count is not None:
        pts = pts[:count]
    return pts.T.astype(np.float32)
