"""Pins of the lattice / refinement oracle (paper sections 2.1.1-2.1.3) against
exact integer geometry and brute force."""
import json
import os
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import oracle
import synth
from oracle import kuhn

F32 = np.float32


def _vol6(v):
    """6 x signed volume of tetrahedra v [n, 4, 3] (exact for dyadic inputs)."""
    a, b, c = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def test_six_tetrahedra_tile_the_cube():
    keys = kuhn.level0_keys((1, 1, 1))
    v = kuhn.vertices_units(keys)
    vol6 = np.abs(_vol6(v))            # integer: 6 x volume
    assert np.all(vol6 == 1.0) and vol6.sum() == 6.0
    rng = np.random.default_rng(0)
    y = rng.uniform(0, 1, (2000, 3))
    k, inside = kuhn.locate(y, 0, (1, 1, 1))
    assert inside.all()
    # located tetrahedron really contains the point: all barycentric weights >= 0
    for key, p in zip(k[:300], y[:300]):
        t = kuhn.vertices_units(np.array([key], np.uint64))[0]
        T = np.stack([t[1] - t[0], t[2] - t[0], t[3] - t[0]], 1)
        lam = np.linalg.solve(T, p - t[0])
        assert lam.min() > -1e-12 and lam.sum() < 1 + 1e-12


def test_centroid_locates_back_to_its_tetrahedron():
    rng = np.random.default_rng(1)
    cells = (5, 4, 3)
    for lv in range(3):
        n = 500
        keys = kuhn.encode(np.full(n, lv), rng.integers(0, 6, n),
                           rng.integers(0, cells[0] << lv, n), rng.integers(0, cells[1] << lv, n),
                           rng.integers(0, cells[2] << lv, n))
        got, inside = kuhn.locate(kuhn.centroid_units(keys), lv, cells)
        assert inside.all() and np.array_equal(got, keys)


def test_children_are_the_red_refinement():
    """Section 2.1.2: each refined element becomes 8 tetrahedra whose vertices
    are the parent's vertices and edge midpoints, 1/8 of its volume each."""
    for q in range(6):
        key = kuhn.encode([0], [q], [0], [0], [0])
        kids = kuhn.children(key, (1, 1, 1))[0]
        assert len(set(kids.tolist())) == 8
        pv = kuhn.vertices_units(key)[0]
        allowed = {tuple(x) for x in pv}
        for a, b in combinations(range(4), 2):
            allowed.add(tuple((pv[a] + pv[b]) / 2))
        kv = kuhn.vertices_units(kids)
        for t in kv:
            assert all(tuple(x) in allowed for x in t)
        assert np.allclose(np.abs(_vol6(kv)), np.abs(_vol6(pv[None]))[0] / 8)
        assert np.array_equal(kuhn.parent(kids, (1, 1, 1)), np.repeat(key, 8))


def test_face_neighbour_shares_the_three_vertices():
    rng = np.random.default_rng(2)
    cells = (4, 4, 4)
    keys = kuhn.level0_keys(cells)[rng.choice(384, 60, replace=False)]
    v = kuhn.vertices_units(keys)
    for t, key in zip(v, keys):
        for m in range(4):
            face = t[[x for x in range(4) if x != m]]
            s = face.mean(0)
            y = s + 2.0 ** -8 * (s - t[m])
            nk, inside = kuhn.locate(y[None], 0, cells)
            if not inside[0]:
                continue
            assert nk[0] != key
            nv = {tuple(x) for x in kuhn.vertices_units(nk)[0]}
            assert all(tuple(x) in nv for x in face)


def _random_mesh(rng, cells, levels):
    """Leaves of a random nested refinement, with random labels."""
    leaves = list(kuhn.level0_keys(cells))
    for _ in range(levels):
        lv = kuhn.decode(np.array(leaves, np.uint64))[0]
        cand = [k for k, l in zip(leaves, lv) if l == lv.max()]
        pick = rng.choice(len(cand), max(1, len(cand) // 4), replace=False)
        chosen = {cand[i] for i in pick}
        kids = kuhn.children(np.array(sorted(chosen), np.uint64), cells).reshape(-1)
        leaves = [k for k in leaves if k not in chosen] + list(kids)
    keys = np.array(leaves, np.uint64)
    return kuhn.LeafSet(keys, rng.integers(0, 3, len(keys)))


def _bruteforce_boundary(ls):
    """Two leaves touch in 2-D when a face of one and a face of the other are
    coplanar, lie on opposite sides, and the centroid of the smaller face is
    strictly inside the larger one (faces of nested Kuhn lattices are nested)."""
    V = [[tuple(Fraction(x) for x in p) for p in t] for t in kuhn.vertices_units(ls.keys)]
    faces = []
    for ti, t in enumerate(V):
        for m in range(4):
            f = [t[x] for x in range(4) if x != m]
            faces.append((ti, f, t[m]))

    def sub(a, b):
        return tuple(x - y for x, y in zip(a, b))

    def cross(a, b):
        return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])

    def dot(a, b):
        return sum(x * y for x, y in zip(a, b))

    def area2(f):
        c = cross(sub(f[1], f[0]), sub(f[2], f[0]))
        return dot(c, c)

    def strictly_inside(g, f):
        n = cross(sub(f[1], f[0]), sub(f[2], f[0]))
        s = [dot(cross(sub(f[(i + 1) % 3], f[i]), sub(g, f[i])), n) for i in range(3)]
        return all(x > 0 for x in s)

    def plane(f):
        # the face's plane, scaled so its first nonzero normal component is 1
        n = cross(sub(f[1], f[0]), sub(f[2], f[0]))
        lead = next(x for x in n if x != 0)
        n = tuple(x / lead for x in n)
        return n + (dot(n, f[0]),)

    # only faces in one plane can touch in 2-D: pair them within each plane
    by_plane = {}
    for fc in faces:
        by_plane.setdefault(plane(fc[1]), []).append(fc)
    pairs = (pq for group in by_plane.values() for pq in combinations(group, 2))
    flag = np.zeros(len(V), bool)
    for (ti, f, ot), (ui, g, ou) in pairs:
        if ti == ui or ls.labels[ti] == ls.labels[ui]:
            continue
        n = cross(sub(f[1], f[0]), sub(f[2], f[0]))
        if any(dot(n, sub(x, f[0])) != 0 for x in g):
            continue
        if dot(n, sub(ot, f[0])) * dot(n, sub(ou, f[0])) >= 0:
            continue
        small, big = (f, g) if area2(f) <= area2(g) else (g, f)
        cen = tuple(sum(x[i] for x in small) / 3 for i in range(3))
        if strictly_inside(cen, big):
            flag[ti] = flag[ui] = True
    return flag


@pytest.mark.parametrize("seed", [3, 4])
def test_boundary_marking_matches_bruteforce(seed):
    rng = np.random.default_rng(seed)
    cells = (2, 2, 1)
    ls = _random_mesh(rng, cells, 2)
    got = kuhn.boundary_mask(ls, cells, 2)
    want = _bruteforce_boundary(ls)
    assert np.array_equal(got, want)


def test_refinement_counts_and_volume_partition():
    cfg = synth.config_small("sphere", cells=8, subdiv=2)
    lat = cfg.lattice
    leaves, stats = kuhn.refine_relabel(lat, lambda p: oracle.label(p, cfg.surfaces), 2)
    n0 = lat.n_points
    assert stats[-1]["leaves"] == n0 + 7 * sum(s["boundary"] for s in stats)
    assert len(leaves.keys) == stats[-1]["leaves"]
    vol = np.abs(_vol6(kuhn.vertices_units(leaves.keys))).sum() / 6
    assert vol == pytest.approx(np.prod(lat.cells), abs=1e-9)
    # every leaf label is the label of its centroid
    cen = kuhn.centroids_mm(leaves.keys, lat.origin, lat.h)
    assert np.array_equal(oracle.label(cen, cfg.surfaces), leaves.labels)
    assert stats[1]["boundary"] > 0 and stats[2]["boundary"] > 0


def test_centroids_in_mm_are_exact_dyadics():
    lat = synth.Lattice(origin=(-100.0, -100.0, -100.0), h=6.25, cells=(32, 32, 32))
    keys = kuhn.level0_keys(lat.cells)[:5000]
    c = kuhn.centroids_mm(keys, lat.origin, lat.h).astype(np.float64)
    ref = np.array(lat.origin)[:, None] + lat.h * kuhn.centroid_units(keys).T
    assert np.array_equal(c, ref)


# ------------------------------------------------- node-based labeling (f1)
def _ary_surfaces(subdiv=3):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ary_three_sphere.json")))
    uv, f = synth.icosphere(subdiv)
    return [synth.Surface(v=(uv * r).astype(np.float32), f=f.astype(np.int32), label=lab,
                          center=np.zeros(3))
            for r, lab in zip(g["radii_mm"], g["labels_outermost_first"])]


def _node_run(lattice, surfaces, rounds):
    return kuhn.refine_relabel_nodes(lattice, lambda p: oracle.enclosure(p, surfaces),
                                     lambda m: oracle.mask_label(m, surfaces), rounds)


def test_node_rule_on_nested_shells_is_the_outermost_vertex_label():
    """For nested shells (the Ary model) a node's enclosure set is every shell
    out to its own, so "all four nodes enclosed" gives the vertex label that is
    least deep in the nesting: here the smallest label id.  Vertex labels come
    from point labels of the vertices, positions recomputed here."""
    surfs = _ary_surfaces()
    lat = synth.Lattice(origin=(-110.0, -110.0, -110.0), h=220.0 / 10, cells=(10, 10, 10))
    leaves, st = _node_run(lat, surfs, 2)
    v = kuhn.vertices_units(leaves.keys)                        # [n, 4, 3]
    pos = (np.asarray(lat.origin)[None, None, :] + lat.h * v).astype(np.float32)
    vl = oracle.label(np.ascontiguousarray(pos.reshape(-1, 3).T), surfs).reshape(-1, 4)
    assert np.array_equal(leaves.labels, vl.min(axis=1))
    assert st[1]["boundary"] > 0 and st[2]["boundary"] > 0


def test_node_rule_on_a_sphere_matches_the_exact_radial_test():
    """Element label 1 exactly when all four nodes are inside the sphere by
    the exact star-shaped test (no solid angles involved)."""
    cfg = synth.config_small("sphere", cells=8, subdiv=2)
    s = cfg.surfaces[0]
    leaves, _ = _node_run(cfg.lattice, [s], 2)
    v = kuhn.vertices_units(leaves.keys)
    pos = (np.asarray(cfg.lattice.origin)[None, None, :] + cfg.lattice.h * v).astype(np.float32)
    inside = oracle.radial_inside(np.ascontiguousarray(pos.reshape(-1, 3).T), s).reshape(-1, 4) > 0
    want = np.where(inside.all(axis=1), s.label, 0)
    assert np.array_equal(leaves.labels, want)


def test_node_rule_counts_and_partition():
    cfg = synth.config_small("head", cells=6, subdiv=2)
    leaves, st = _node_run(cfg.lattice, cfg.surfaces, 2)
    n0 = 6 * int(np.prod(cfg.lattice.cells))
    assert len(leaves.keys) == n0 + 7 * sum(r["boundary"] for r in st)
    vol = sum(1.0 / 6.0 * 8.0 ** -lv for lv in kuhn.decode(leaves.keys)[0])
    assert abs(vol - np.prod(cfg.lattice.cells)) < 1e-9
    # every node of every leaf has been labeled exactly once: a split keeps
    # the parent's four vertices among its children's, so the nodes of the
    # final leaves are every node ever created
    nk = np.unique(kuhn.node_keys(kuhn.vertices_units(leaves.keys)).reshape(-1))
    assert sum(r["nodes"] for r in st) == len(nk)


def test_node_rule_labels_each_node_once_by_brute_force():
    """Records every point handed to the enclosure test: no node is
    evaluated twice, and the evaluated nodes are exactly the vertices of the
    final leaves (found here from the leaves' corners, independently of the
    oracle's node store)."""
    cfg = synth.config_small("head", cells=5, subdiv=2)
    lat = cfg.lattice
    seen = []

    def mask_fn(p):
        seen.append(np.asarray(p, dtype=np.float32).T.copy())
        return oracle.enclosure(p, cfg.surfaces)

    leaves, st = kuhn.refine_relabel_nodes(lat, mask_fn,
                                           lambda m: oracle.mask_label(m, cfg.surfaces), 2)
    pts = np.concatenate(seen)
    assert st[1]["boundary"] > 0 and st[2]["boundary"] > 0
    assert len(np.unique(pts, axis=0)) == len(pts)          # no node labeled twice
    corners = set()
    for key in leaves.keys.tolist():
        v = kuhn.vertices_units(np.array([key], dtype=np.uint64))[0]     # [4, 3] lattice units
        for c in v:
            corners.add(tuple(float(x) for x in c))
    got = set(tuple(float(x) for x in c) for c in
              np.round((pts.astype(np.float64) - np.asarray(lat.origin)) / lat.h, 9))
    assert got == corners


@pytest.mark.parametrize("mutant", ["any_node", "three_nodes"])
def test_node_pins_catch_a_wrong_element_rule(monkeypatch, mutant):
    """A plausible mistake in the four-node rule (any node instead of all, or
    a node dropped) is caught by the pins above."""
    def any_node(keys, store):
        m = store.get(kuhn.node_keys(kuhn.vertices_units(keys)).reshape(-1)).reshape(-1, 4)
        return m[:, 0] | m[:, 1] | m[:, 2] | m[:, 3]

    def three_nodes(keys, store):
        m = store.get(kuhn.node_keys(kuhn.vertices_units(keys)).reshape(-1)).reshape(-1, 4)
        return m[:, 0] & m[:, 1] & m[:, 2]

    monkeypatch.setattr(kuhn, "element_masks", {"any_node": any_node,
                                                "three_nodes": three_nodes}[mutant])
    with pytest.raises(AssertionError):
        test_node_rule_on_a_sphere_matches_the_exact_radial_test()


# ------------------------------------------- recursion until convergence
def _plane_label(p):
    """A compartment bounded by an oblique plane (label 1 above it)."""
    p = np.asarray(p, dtype=np.float64)
    return (p[0] + 0.37 * p[1] + 0.11 * p[2] > 13.0).astype(np.int32)


def test_converging_recursion_is_a_fixed_point_by_brute_force():
    """Fig. 3: the recursion ends when the boundary no longer changes.  With
    finest level L, the final leaves have no label-boundary leaf coarser than
    L (checked by exact pairwise face contact); the fixed two-round form on
    the same input leaves such leaves behind, so the two forms differ."""
    lat = synth.Lattice(origin=(-100.0, -100.0, -100.0), h=100.0, cells=(2, 2, 1))
    fixed, _ = kuhn.refine_relabel(lat, _plane_label, 2)
    conv, st = kuhn.refine_relabel(lat, _plane_label, 2, converge=True)
    lv_fixed = kuhn.decode(fixed.keys)[0]
    assert (_bruteforce_boundary(fixed) & (lv_fixed < 2)).any()
    lv = kuhn.decode(conv.keys)[0]
    assert lv.max() == 2
    assert not (_bruteforce_boundary(conv) & (lv < 2)).any()
    assert len(st) - 1 > 2                      # more steps than levels
    assert all(s["boundary"] > 0 for s in st[1:])
    n0 = lat.n_points
    assert len(conv.keys) == n0 + 7 * sum(s["boundary"] for s in st)
    vol = np.abs(_vol6(kuhn.vertices_units(conv.keys))).sum() / 6
    assert vol == pytest.approx(np.prod(lat.cells), abs=1e-12)
    assert np.array_equal(_plane_label(kuhn.centroids_mm(conv.keys, lat.origin, lat.h)),
                          conv.labels)


def test_converging_recursion_contains_the_fixed_rounds():
    """Every leaf of the fixed form is a leaf or an ancestor of leaves of the
    converged form (the converging recursion only adds splits), and with no
    boundary at all both forms keep the lattice."""
    cfg = synth.config_small("sphere", cells=6, subdiv=2)
    lat = cfg.lattice
    fn = lambda p: oracle.label(p, cfg.surfaces)          # noqa: E731
    fixed, _ = kuhn.refine_relabel(lat, fn, 2)
    conv, st = kuhn.refine_relabel(lat, fn, 2, converge=True)
    assert len(conv.keys) >= len(fixed.keys)
    # locate an interior point of each converged leaf (generic barycentric
    # weights, so it lies on no facet of any level) in the fixed mesh: the
    # containing fixed leaf must be the leaf itself or an ancestor (not finer)
    wts = np.array([0.4012, 0.2987, 0.1993, 0.1008])
    inner = np.einsum("k,nkd->nd", wts, kuhn.vertices_units(conv.keys).astype(np.float64))
    owner = kuhn.containing_leaf(fixed, inner, lat.cells, 2)
    assert (owner >= 0).all()
    assert (kuhn.decode(fixed.keys[owner])[0] <= kuhn.decode(conv.keys)[0]).all()
    empty, st0 = kuhn.refine_relabel(lat, lambda p: np.zeros(p.shape[1], np.int32), 2,
                                     converge=True)
    assert len(st0) == 1 and len(empty.keys) == lat.n_points


def test_converging_node_rule_labels_each_node_once():
    """The four-node rule under the converging recursion: no node evaluated
    twice, the evaluated nodes are the final leaves' vertices, and no
    boundary leaf coarser than the finest level is left."""
    cfg = synth.config_small("head", cells=5, subdiv=2)
    lat = cfg.lattice
    seen = []

    def mask_fn(p):
        seen.append(np.asarray(p, dtype=np.float32).T.copy())
        return oracle.enclosure(p, cfg.surfaces)

    leaves, st = kuhn.refine_relabel_nodes(lat, mask_fn,
                                           lambda m: oracle.mask_label(m, cfg.surfaces), 2,
                                           converge=True)
    pts = np.concatenate(seen)
    assert len(np.unique(pts, axis=0)) == len(pts)
    assert sum(s["nodes"] for s in st) == len(pts)
    lv = kuhn.decode(leaves.keys)[0]
    assert not (kuhn.boundary_mask(leaves, lat.cells, 2) & (lv < 2)).any()
    corners = set()
    for c in kuhn.vertices_units(leaves.keys).reshape(-1, 3):
        corners.add(tuple(float(x) for x in c))
    got = set(tuple(float(x) for x in c) for c in
              np.round((pts.astype(np.float64) - np.asarray(lat.origin)) / lat.h, 9))
    assert got == corners
