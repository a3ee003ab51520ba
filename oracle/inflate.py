"""Inflation of the compartment boundaries -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper section 2.2.2, zeta = 0.05 in section 2.6.1: the nodes of a compartment
boundary dV are slid along their edges toward the points where those edges
cross the segmentation surface S, x_i <- x_i + zeta d e, with e the unit
vector along the edge and d the distance from x_i to S.  Read as:

* the nodes that move are the interface nodes (an edge of the node joins
  tetrahedra of two or more labels) that are not on the lattice box;
* for such a node every incident edge is a segment from x_i to the
  neighbour x_j; its crossing with S is the smallest parameter t in [0, 1]
  at which it meets a triangle of any surface of the set (segment-triangle
  intersection by the Moller-Trumbore construction, boundaries included);
* d = t |x_j - x_i| on the edge with the smallest d (ties: the neighbour
  with the smaller node key), e = (x_j - x_i) / |x_j - x_i|;
* nodes whose edges cross no triangle do not move; all moves read the
  positions before inflation.

Brute force over every triangle, float64, in the order written above.
"""
import numpy as np


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], -1)


def segment_hits(p, q, tris):
    """Parameters t in [0, 1] where segment p -> q meets each triangle
    (tris [T, 3, 3]); NaN where it does not (parallel included).  Products
    and sums are written out one by one (no fused operations)."""
    p = np.asarray(p, dtype=np.float64)
    d = np.asarray(q, dtype=np.float64) - p
    v0, v1, v2 = tris[:, 0], tris[:, 1], tris[:, 2]
    e1 = v1 - v0
    e2 = v2 - v0
    h = _cross(d, e2)
    a = _dot(e1, h)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = 1.0 / a
        s = p - v0
        u = f * _dot(s, h)
        qv = _cross(s, e1)
        v = f * _dot(d, qv)
        t = f * _dot(e2, qv)
        ok = (a != 0) & (u >= 0) & (u <= 1) & (v >= 0) & (u + v <= 1) & (t >= 0) & (t <= 1)
    return np.where(ok, t, np.nan)


def triangles(surfaces):
    """All triangles of the set as float64 [T, 3, 3], each with its vertices
    in lexicographic (x, y, z) order so that the crossing arithmetic does not
    depend on how a triangle was listed."""
    tri = np.concatenate([s.v.astype(np.float64)[s.f] for s in surfaces])
    order = np.lexsort((tri[:, :, 2], tri[:, :, 1], tri[:, :, 0]), axis=-1)
    return np.take_along_axis(tri, order[:, :, None], axis=1)


def inflate(xyz, edges, movable, node_keys, tris, zeta=0.05):
    """xyz [n, 3]; edges [E, 2] undirected; movable [n]; node_keys [n] (tie
    break).  Returns (new positions, per node the chosen neighbour or -1,
    per node d)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    n = len(xyz)
    nbrs = [[] for _ in range(n)]
    for a, b in np.asarray(edges):
        nbrs[a].append(b)
        nbrs[b].append(a)
    out = xyz.copy()
    chosen = np.full(n, -1, dtype=np.int64)
    dist = np.full(n, np.nan)
    for i in np.nonzero(movable)[0]:
        best = None
        for j in nbrs[i]:
            t = segment_hits(xyz[i], xyz[j], tris)
            if np.all(np.isnan(t)):
                continue
            length = np.sqrt(_dot(xyz[j] - xyz[i], xyz[j] - xyz[i]))
            d = np.nanmin(t) * length
            cand = (d, int(node_keys[j]), j, length)
            if best is None or cand[:2] < best[:2]:
                best = cand
        if best is None:
            continue
        d, _, j, length = best
        e = (xyz[j] - xyz[i]) / length
        out[i] = xyz[i] + zeta * d * e
        chosen[i] = j
        dist[i] = d
    return out, chosen, dist
