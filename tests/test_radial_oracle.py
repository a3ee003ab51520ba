"""Pins of the indexed exact radial test (oracle/radial.c) and of the checkers
that form lattice and leaf points themselves.

The radial test decides inside / on / outside of a star-shaped surface from
exact orientation predicates (paper section 2.1.3: enclosed when the solid
angle over 4 pi reaches T, or on the surface).  It is pinned against facts it
does not share code with: the winding-number oracle (the Van Oosterom-Strackee
sum), the unindexed O(T) radial scan, analytic spheres (section 2.5's Ary
radii), brute-force point sets on and around the surfaces, and the Kuhn
lattice conventions of `oracle.kuhn`.  Planted mistakes in radial.c each fail
one of these pins.
"""
import ctypes
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import kuhn

F32 = np.float32
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ORACLE_DIR = os.path.dirname(oracle.__file__)


def _hard_points(surfaces, rng, n=1500):
    """Uniform box points, points within 0.5 mm of the surfaces, points at
    1e-9 .. 1e-3 mm from faces, edges and vertices, every vertex (on the
    surface), exact edge midpoints and the centres."""
    parts = [synth.uniform_box(rng, n, -100, 100),
             synth.near_surface_points(rng, surfaces, n, 0.5)]
    for s in surfaces[:3]:
        parts.append(synth.precision_ladder(s, rng, n_sites=8))
        parts.append(synth.face_centroids_on_surface(s, count=400))
    parts.append(np.array([s.center for s in surfaces], dtype=F32).T)
    return np.ascontiguousarray(np.concatenate(parts, 1))


def _surface_points(surfaces):
    return np.ascontiguousarray(np.concatenate([s.v.T for s in surfaces], 1))


# ------------------------------------------------------------ inside test
def test_indexed_radial_labels_equal_winding_labels_on_a_head_mesh():
    cfg = synth.config_small("head", subdiv=3)
    rng = np.random.default_rng(71)
    pts = _hard_points(cfg.surfaces, rng)
    rs = oracle.RadialSet(cfg.surfaces)
    assert np.array_equal(rs.label(pts), oracle.label(pts, cfg.surfaces))
    assert rs.fallbacks() == 0


def test_indexed_radial_equals_the_unindexed_scan_per_surface():
    cfg = synth.config_small("head", subdiv=2)
    rng = np.random.default_rng(72)
    pts = _hard_points(cfg.surfaces, rng, 800)
    for s in cfg.surfaces:
        r = oracle.RadialIndex(s)
        assert np.array_equal(r.query(pts), oracle.radial_inside(pts, s))
        assert r.stats()["fallbacks"] == 0


def test_every_vertex_is_on_the_surface_and_centres_are_inside():
    cfg = synth.config_small("head", subdiv=2)
    for s in cfg.surfaces:
        r = oracle.RadialIndex(s)
        assert np.all(r.query(s.v.T.copy()) == 2)
        assert r.query(np.array(s.center, dtype=F32).reshape(3, 1))[0] == 1


def test_geodesic_spheres_and_ellipsoids_of_the_batched_workload():
    """Geodesic frequency-nu surfaces (the batched and precision-stress
    workloads) at small sizes, against the winding oracle."""
    rng = np.random.default_rng(73)
    for i in range(6):
        surfs, pts = synth.c4_instance(i, t_lo=200, t_hi=3000, n_lo=300, n_hi=600)
        q = np.concatenate([pts, synth.near_surface_points(rng, surfs, 600, 0.5),
                            _surface_points(surfs)[:, :300]], 1)
        rs = oracle.RadialSet(surfs)
        assert np.array_equal(rs.label(q), oracle.label(q, surfs)), i
        assert rs.fallbacks() == 0


def test_wide_cones_of_an_icosahedron():
    """Every cone of an icosahedron spans 63 degrees: all go to the wide list."""
    uv, f = synth.icosahedron()
    s = synth.Surface(v=(uv * 50).astype(F32), f=f.astype(np.int32), label=1, center=np.zeros(3))
    r = oracle.RadialIndex(s)
    assert r.stats()["wide"] == 20
    rng = np.random.default_rng(74)
    pts = np.concatenate([synth.uniform_box(rng, 4000, -60, 60), s.v.T], 1)
    w, on = oracle.winding(pts, s.v, s.f)
    q = r.query(pts)
    assert np.array_equal(q > 0, (w >= 0.5) | on)
    assert np.array_equal(q == 2, on)
    assert r.stats()["fallbacks"] == 0


def test_ary_three_spheres_are_analytic():
    """Section 2.5's concentric spheres: the label of the smallest sphere
    enclosing the point, away from the triangulation's sagitta band."""
    g = json.load(open(os.path.join(GOLDEN, "ary_three_sphere.json")))
    uv, f = synth.icosphere(4)
    surfs = [synth.Surface(v=(uv * r).astype(F32), f=f.astype(np.int32), label=lab,
                           center=np.zeros(3))
             for r, lab in zip(g["radii_mm"], g["labels_outermost_first"])]
    rng = np.random.default_rng(75)
    d = rng.standard_normal((3, 20000))
    d /= np.linalg.norm(d, axis=0)
    rad = rng.uniform(0, 120, 20000)
    keep = np.all(np.abs(rad[:, None] - np.array(g["radii_mm"])[None, :]) > 0.2, axis=1)
    pts = (d * rad)[:, keep].astype(F32)
    r = np.linalg.norm(pts.astype(np.float64), axis=0)
    want = np.zeros(pts.shape[1], np.int32)
    for rr, lab in zip(g["radii_mm"], g["labels_outermost_first"]):
        want[r < rr] = lab
    assert np.array_equal(oracle.RadialSet(surfs).label(pts), want)


def test_priority_the_later_surface_wins():
    uv, f = synth.icosphere(3)
    big = synth.Surface(v=(uv * 50).astype(F32), f=f.astype(np.int32), label=7, center=np.zeros(3))
    shifted = synth.Surface(v=(uv * 20 + np.array([40, 0, 0])).astype(F32), f=f.astype(np.int32),
                            label=3, center=np.array([40.0, 0, 0]))
    pts = np.array([[0, 0, 0], [30, 0, 0], [55, 0, 0], [70, 0, 0], [-40, 0, 0]], F32).T
    assert list(oracle.RadialSet([big, shifted]).label(pts)) == [7, 3, 3, 0, 7]
    assert list(oracle.RadialSet([shifted, big]).label(pts)) == [7, 7, 3, 0, 7]
    _, m = oracle.RadialSet([big, shifted]).label(pts, want_masks=True)
    assert list(m) == [1, 3, 2, 0, 1]


def test_preconditions_are_checked():
    uv, f = synth.icosphere(2)
    v = (uv * 30).astype(F32)
    # the centre outside the surface: some cones are negatively oriented
    with pytest.raises(ValueError, match="positively oriented"):
        oracle.RadialIndex(synth.Surface(v=v, f=f.astype(np.int32), label=1,
                                         center=np.array([45.0, 0, 0])))
    # every triangle twice: all cones positive but the directions covered twice
    with pytest.raises(ValueError, match="winding number"):
        oracle.RadialIndex(synth.Surface(v=v, f=np.concatenate([f, f]).astype(np.int32), label=1,
                                         center=np.zeros(3)))


# ------------------------------------------------------- lattice checkers
def _small_lattice():
    cfg = synth.config_small("head", cells=10, subdiv=2)
    return cfg, cfg.lattice


def test_lattice_centroids_and_leaf_points_follow_the_kuhn_conventions():
    for h, origin in ((6.25, (-100.0, -100.0, -100.0)), (0.3, (-1.7, 2.9, -0.1))):
        cells = (5, 4, 3)
        rng = np.random.default_rng(76)
        lv = rng.integers(0, 4, 500)
        q = rng.integers(0, 6, 500)
        ijk = [rng.integers(0, c << 3, 500) >> (3 - lv) for c in cells]
        keys = kuhn.encode(lv, q, *ijk)
        assert np.array_equal(oracle.leaf_points(origin, h, keys),
                              kuhn.centroids_mm(keys, origin, h))
        want = kuhn.nodes_mm(kuhn.vertices_units(keys).reshape(-1, 3), origin, h)
        got = oracle.leaf_points(origin, h, keys, rule="four_nodes").reshape(-1, 3).T
        assert np.array_equal(got, want)
        lat = synth.Lattice(origin=origin, h=h, cells=cells)
        k0 = kuhn.level0_keys(cells)
        assert np.array_equal(oracle.leaf_points(origin, h, k0), kuhn.centroids_mm(k0, origin, h))
        assert lat.n_points == len(k0)


def test_lattice_check_counts_planted_mismatches_exactly():
    cfg, lat = _small_lattice()
    keys = kuhn.level0_keys(lat.cells)
    want = oracle.label(kuhn.centroids_mm(keys, lat.origin, lat.h), cfg.surfaces)
    rs = oracle.RadialSet(cfg.surfaces)
    assert rs.check_lattice(lat, want)[0] == 0
    rng = np.random.default_rng(77)
    bad = np.sort(rng.choice(len(want), 37, replace=False))
    got = want.copy()
    got[bad] = (got[bad] + 1) % 6
    n, where = rs.check_lattice(lat, got)
    assert n == 37 and np.array_equal(where, bad)
    # in chunks, numbered globally
    lo, hi = 1234, 4321
    n, where = rs.check_lattice(lat, got[lo:hi], first=lo)
    sel = bad[(bad >= lo) & (bad < hi)]
    assert n == len(sel) and np.array_equal(where, sel)


def test_key_check_under_both_element_rules():
    cfg, lat = _small_lattice()
    rng = np.random.default_rng(78)
    lv = rng.integers(0, 4, 3000)
    q = rng.integers(0, 6, 3000)
    ijk = [rng.integers(0, c << 3, 3000) >> (3 - lv) for c in lat.cells]
    keys = kuhn.encode(lv, q, *ijk)
    rs = oracle.RadialSet(cfg.surfaces)
    cen = kuhn.centroids_mm(keys, lat.origin, lat.h)
    want_c = oracle.label(cen, cfg.surfaces)
    assert rs.check_keys(lat.origin, lat.h, keys, want_c)[0] == 0
    v = kuhn.nodes_mm(kuhn.vertices_units(keys).reshape(-1, 3), lat.origin, lat.h)
    m = oracle.enclosure(v, cfg.surfaces).reshape(-1, 4)
    want_n = oracle.mask_label(m[:, 0] & m[:, 1] & m[:, 2] & m[:, 3], cfg.surfaces)
    assert rs.check_keys(lat.origin, lat.h, keys, want_n, rule="four_nodes")[0] == 0
    # the two rules differ somewhere on this mesh, and each check sees it
    diff = np.nonzero(want_c != want_n)[0]
    assert len(diff) > 0
    n, where = rs.check_keys(lat.origin, lat.h, keys, want_n, cap=10000)
    assert n == len(diff) and np.array_equal(where, diff)


# ------------------------------------------------------------- mutants
RADIAL_SRC = os.path.join(ORACLE_DIR, "radial.c")
MUTANTS = {
    "side flipped": ("return s > 0 ? 1 : (s == 0 ? 2 : 0);", "return s < 0 ? 1 : (s == 0 ? 2 : 0);"),
    "on-surface outside": ("return s > 0 ? 1 : (s == 0 ? 2 : 0);", "return s > 0 ? 1 : 0;"),
    "cone test drops a side": ("\n        && oracle_orient3d(r->c, v2, v0, p) >= 0;", ";"),
    "box reject on the box": ("if (p[i] < r->lo[i] || p[i] > r->hi[i])",
                              "if (p[i] <= r->lo[i] || p[i] >= r->hi[i])"),
    "wide list skipped": ("for (int64_t k = 0; k < r->n_wide; ++k)", "for (int64_t k = 0; k < 0; ++k)"),
    "first surface wins": ("            label = surf_label[s];\n            m |=",
                           "            if (!label) label = surf_label[s];\n            m |="),
    "centroid weights swapped": ("c[PERM[q][0]] = 0.75;", "c[PERM[q][0]] = 0.25;"),
    "four-node OR": ("        all &= m;", "        all |= m;"),
    "lattice i and j swapped": ("int64_t cell[3] = {cl % c->cells[0], (cl / c->cells[0]) % c->cells[1],",
                                "int64_t cell[3] = {(cl / c->cells[0]) % c->cells[1], cl % c->cells[0],"),
    "no winding precondition": ("if (!(fabs(wc - 1.0) < 0.25)) {", "if (0) {"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(RADIAL_SRC).read()
    assert src.count(old) >= 1, name
    c = tmp_path / "radial_mut.c"
    c.write_text(src.replace(old, new, 1))
    so = tmp_path / ("m_%d.so" % abs(hash(name)))
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-I", ORACLE_DIR,
                           "-o", str(so), os.path.join(ORACLE_DIR, "sal_oracle.c"), str(c),
                           "-lpthread", "-lm"])
    return oracle.declare(ctypes.CDLL(str(so)))


def _radial_pins_pass(L):
    """The pins above, run against library L; False when any fails."""
    try:
        cfg = synth.config_small("head", cells=8, subdiv=2)
        rng = np.random.default_rng(79)
        pts = _hard_points(cfg.surfaces, rng, 500)
        rs = oracle.RadialSet(cfg.surfaces, L=L)
        if not np.array_equal(rs.label(pts), oracle.label(pts, cfg.surfaces)):
            return False
        for s in cfg.surfaces:
            r = oracle.RadialIndex(s, L=L)
            if not np.all(r.query(s.v.T.copy()) == 2):
                return False
        uv, f = synth.icosahedron()
        ico = synth.Surface(v=(uv * 50).astype(F32), f=f.astype(np.int32), label=1,
                            center=np.zeros(3))
        r = oracle.RadialIndex(ico, L=L)
        r.query(synth.uniform_box(rng, 500, -60, 60))
        if rs.fallbacks() or r.stats()["fallbacks"]:
            return False
        try:
            oracle.RadialIndex(synth.Surface(v=ico.v, f=np.concatenate([f, f]).astype(np.int32),
                                             label=1, center=np.zeros(3)), L=L)
            return False
        except ValueError:
            pass
        lat = cfg.lattice
        keys = kuhn.level0_keys(lat.cells)
        want = oracle.label(kuhn.centroids_mm(keys, lat.origin, lat.h), cfg.surfaces)
        if rs.check_lattice(lat, want)[0] != 0:
            return False
        lv = rng.integers(0, 4, 800)
        ijk = [rng.integers(0, c << 3, 800) >> (3 - lv) for c in lat.cells]
        k = kuhn.encode(lv, rng.integers(0, 6, 800), *ijk)
        if rs.check_keys(lat.origin, lat.h, k, oracle.label(kuhn.centroids_mm(k, lat.origin, lat.h),
                                                            cfg.surfaces))[0]:
            return False
        v = kuhn.nodes_mm(kuhn.vertices_units(k).reshape(-1, 3), lat.origin, lat.h)
        m = oracle.enclosure(v, cfg.surfaces).reshape(-1, 4)
        wn = oracle.mask_label(m[:, 0] & m[:, 1] & m[:, 2] & m[:, 3], cfg.surfaces)
        if rs.check_keys(lat.origin, lat.h, k, wn, rule="four_nodes")[0]:
            return False
        return True
    except (RuntimeError, ValueError):
        return False


def test_radial_pins_pass_on_the_oracle_itself():
    assert _radial_pins_pass(oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_radial_pins_catch_planted_mistakes(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _radial_pins_pass(_build_mutant(tmp_path, name, old, new)), name
