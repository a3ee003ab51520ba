"""Pins of the inflation oracle (paper section 2.2.2): segment-triangle
crossings in closed form and against a plain 3x3 linear solve, the node move
on a plane in closed form, and the nearest-crossing rule by brute force."""
import numpy as np
import pytest

import oracle
import synth
from oracle import conform, inflate, kuhn, smooth

TRI = np.array([[[0.0, 0.0, 1.0], [2.0, 0.0, 1.0], [0.0, 2.0, 1.0]]])


@pytest.mark.parametrize("p,q,want", [
    ((0.25, 0.25, 0.0), (0.25, 0.25, 2.0), 0.5),        # through the interior
    ((0.25, 0.25, 2.0), (0.25, 0.25, 0.0), 0.5),        # reversed
    ((0.5, 0.5, 0.5), (0.5, 0.5, 1.5), 0.5),
    ((1.0, 1.0, 0.0), (1.0, 1.0, 4.0), 0.25),           # on the hypotenuse: included
    ((0.0, 0.0, 1.0), (0.0, 0.0, 3.0), 0.0),            # starts on a vertex
    ((3.0, 0.0, 0.0), (3.0, 0.0, 2.0), np.nan),         # beside the triangle
    ((0.25, 0.25, 0.0), (0.25, 0.25, 0.9), np.nan),     # stops short
    ((0.0, 0.5, 0.5), (2.0, 0.5, 0.5), np.nan),         # parallel to the plane
])
def test_segment_crossings_in_closed_form(p, q, want):
    t = inflate.segment_hits(p, q, TRI)[0]
    if np.isnan(want):
        assert np.isnan(t)
    else:
        assert t == pytest.approx(want, abs=1e-15)


def _solve(p, q, tri):
    """p + t (q - p) = v0 + u (v1 - v0) + v (v2 - v0) as a linear system."""
    m = np.stack([q - p, tri[0] - tri[1], tri[0] - tri[2]], 1)
    t, u, v = np.linalg.solve(m, tri[0] - p)
    return t, u, v


def test_crossings_agree_with_a_linear_solve():
    rng = np.random.default_rng(11)
    tris = rng.normal(size=(400, 3, 3))
    hits = 0
    for _ in range(200):
        p, q = rng.normal(size=3), rng.normal(size=3)
        got = inflate.segment_hits(p, q, tris)
        for k in range(len(tris)):
            t, u, v = _solve(p, q, tris[k])
            inside = u > 1e-9 and v > 1e-9 and u + v < 1 - 1e-9 and 1e-9 < t < 1 - 1e-9
            outside = u < -1e-9 or v < -1e-9 or u + v > 1 + 1e-9 or t < -1e-9 or t > 1 + 1e-9
            if inside:
                hits += 1
                assert got[k] == pytest.approx(t, rel=1e-9, abs=1e-12)
            elif outside:
                assert np.isnan(got[k])
    assert hits > 100


def test_node_moves_a_fraction_zeta_toward_the_nearest_crossing():
    """Node at the origin, planes z = 1 and z = 1.5: the vertical edge
    crosses first at d = 1, the slanted one at d = sqrt(5)/2; the node moves
    to z = zeta."""
    big = np.array([[[-10.0, -10.0, 1.0], [10.0, -10.0, 1.0], [0.0, 10.0, 1.0]],
                    [[-10.0, -10.0, 1.5], [10.0, -10.0, 1.5], [0.0, 10.0, 1.5]]])
    xyz = np.array([[0, 0, 0], [0, 0, 2], [1, 0, 2], [0, 0, -1]], dtype=np.float64)
    edges = np.array([[0, 1], [0, 2], [0, 3]])
    mv = np.array([True, False, False, False])
    keys = np.arange(4)
    for zeta in (0.05, 0.3):
        out, chosen, d = inflate.inflate(xyz, edges, mv, keys, big, zeta)
        assert chosen[0] == 1 and d[0] == pytest.approx(1.0, abs=1e-15)
        np.testing.assert_allclose(out[0], [0, 0, zeta], atol=1e-15)
        assert np.array_equal(out[1:], xyz[1:])
    out, _, _ = inflate.inflate(xyz, edges, mv, keys, big, 0.0)
    assert np.array_equal(out, xyz)
    out, chosen, _ = inflate.inflate(xyz, edges, np.zeros_like(mv), keys, big)
    assert np.array_equal(out, xyz) and np.all(chosen == -1)


def test_equal_distances_go_to_the_smaller_key():
    big = np.array([[[-10.0, -10.0, 1.0], [10.0, -10.0, 1.0], [0.0, 10.0, 1.0]]])
    xyz = np.array([[0, 0, 0], [1, 0, 2], [0, 1, 2]], dtype=np.float64)
    edges = np.array([[0, 1], [0, 2]])
    mv = np.array([True, False, False])
    for keys, want in ((np.array([0, 5, 7]), 1), (np.array([0, 9, 7]), 2)):
        _, chosen, _ = inflate.inflate(xyz, edges, mv, keys, big)
        assert chosen[0] == want


def test_nearest_crossing_by_brute_force_on_a_sphere_mesh():
    cfg = synth.config_small("sphere", cells=4, subdiv=1)
    leaves, _ = kuhn.refine_relabel(cfg.lattice, lambda p: oracle.label(p, cfg.surfaces), 1)
    t, lab, _ = conform.conforming_mesh(leaves.keys, leaves.labels, cfg.lattice.cells)
    nodes, inv = np.unique(t.reshape(-1), return_inverse=True)
    ids = inv.reshape(-1, 4)
    lat = cfg.lattice
    xyz = np.asarray(lat.origin)[None, :] + (lat.h / kuhn._FINE) * conform.unkey(nodes)
    e, surf = smooth.edges(ids, lab)
    mv = np.zeros(len(nodes), bool)
    mv[e[surf].reshape(-1)] = True
    mv &= ~smooth.on_box(nodes, lat.cells)
    tris = inflate.triangles(cfg.surfaces)
    out, chosen, dist = inflate.inflate(xyz, e, mv, nodes, tris)
    assert np.sum(chosen >= 0) > 0.5 * mv.sum()
    rng = np.random.default_rng(2)
    for i in rng.choice(np.nonzero(mv)[0], 40, replace=False):
        nb = np.concatenate([e[e[:, 0] == i, 1], e[e[:, 1] == i, 0]])
        best = np.inf
        for j in nb:
            for k in range(len(tris)):
                try:
                    tt, u, v = _solve(xyz[i], xyz[j], tris[k])
                except np.linalg.LinAlgError:
                    continue
                if u >= 0 and v >= 0 and u + v <= 1 and 0 <= tt <= 1:
                    best = min(best, tt * np.linalg.norm(xyz[j] - xyz[i]))
        if np.isinf(best):
            assert chosen[i] == -1 and np.array_equal(out[i], xyz[i])
        else:
            assert dist[i] == pytest.approx(best, rel=1e-9)
            step = out[i] - xyz[i]
            assert np.linalg.norm(step) == pytest.approx(0.05 * best, rel=1e-9)
            edge = xyz[chosen[i]] - xyz[i]
            assert np.linalg.norm(np.cross(step, edge)) <= 1e-9 * np.linalg.norm(edge)
            assert np.dot(step, edge) > 0
    assert np.array_equal(out[~mv], xyz[~mv])
