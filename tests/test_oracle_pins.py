"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, an independent spherical-excess formula, 50-digit arithmetic,
exact rationals and analytic inside/outside geometry.

Paper section 2.1.3 (Eq. 1) defines the quantity: the solid angle of a closed
surface seen from a point, over 4 pi; per flat triangle it is given exactly by
the Van Oosterom-Strackee formula.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

F32 = np.float32
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def om(p, a, b, c):
    return oracle.tri_solid_angle(np.array(p, F32), np.array(a, F32), np.array(b, F32),
                                  np.array(c, F32))[0]


# ----------------------------------------------------------- single triangle
def test_octant_triangle_is_half_pi():
    # N = 1, D = 1: the octant seen from the origin is exactly pi/2 sr.
    assert om((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)) == pytest.approx(math.pi / 2, abs=1e-15)


def _cube_faces():
    """Cube [-1, 1]^3 as 12 outward triangles grouped by face."""
    faces = []
    for axis in range(3):
        for s in (-1.0, 1.0):
            u, v = [a for a in range(3) if a != axis]
            quad = []
            for du, dv in ((-1, -1), (1, -1), (1, 1), (-1, 1)):
                p = [0.0, 0.0, 0.0]
                p[axis], p[u], p[v] = s, du, dv
                quad.append(p)
            n = np.cross(np.subtract(quad[1], quad[0]), np.subtract(quad[2], quad[0]))
            if n[axis] * s < 0:
                quad = quad[::-1]
            faces.append([(quad[0], quad[1], quad[2]), (quad[0], quad[2], quad[3])])
    return faces


def test_cube_face_from_centre_is_two_thirds_pi():
    for tri_pair in _cube_faces():
        tot = sum(om((0, 0, 0), *t) for t in tri_pair)
        assert tot == pytest.approx(2 * math.pi / 3, abs=1e-14)


def test_regular_tetrahedron_faces_from_centroid_are_pi():
    v = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]
    for skip in range(4):
        f = [v[i] for i in range(4) if i != skip]
        n = np.cross(np.subtract(f[1], f[0]), np.subtract(f[2], f[0]))
        if np.dot(n, f[0]) < 0:
            f = [f[0], f[2], f[1]]
        assert om((0, 0, 0), *f) == pytest.approx(math.pi, abs=1e-14)


def test_coplanar_outside_is_zero_and_on_triangle_flagged():
    a, b, c = (0, 0, 0), (4, 0, 0), (0, 4, 0)
    val, on = oracle.tri_solid_angle(np.array((5, 5, 0), F32), *(np.array(x, F32) for x in (a, b, c)))
    assert val == 0.0 and not on
    for p in [(1, 1, 0), (2, 0, 0), (0, 0, 0), (2, 2, 0)]:   # interior, edge, vertex, hypotenuse
        val, on = oracle.tri_solid_angle(np.array(p, F32), *(np.array(x, F32) for x in (a, b, c)))
        assert on, p


def test_orientation_flip_negates():
    rng = np.random.default_rng(3)
    for _ in range(200):
        p, a, b, c = rng.uniform(-5, 5, (4, 3)).astype(F32)
        assert om(p, a, b, c) == pytest.approx(-om(p, a, c, b), rel=2e-15, abs=1e-15)


def test_midpoint_split_is_additive():
    rng = np.random.default_rng(4)
    for _ in range(200):
        a, b, c = (rng.integers(-40, 40, (3, 3)) * 2).astype(F32)   # even: exact midpoints
        p = rng.uniform(-30, 30, 3).astype(F32)
        ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
        whole = om(p, a, b, c)
        parts = om(p, a, ab, ca) + om(p, ab, b, bc) + om(p, ca, bc, c) + om(p, ab, bc, ca)
        assert whole == pytest.approx(parts, abs=1e-12)


def test_lhuilier_spherical_excess():
    """L'Huilier: tan(E/4)^2 = tan(s/2) tan((s-a)/2) tan((s-b)/2) tan((s-c)/2)
    with a, b, c the arcs between the unit vectors and s their half sum."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        p = rng.uniform(-3, 3, 3).astype(F32)
        v = rng.uniform(-10, 10, (3, 3)).astype(F32)
        u = (v.astype(np.float64) - p.astype(np.float64))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        arcs = [math.acos(np.clip(np.dot(u[i], u[j]), -1, 1)) for i, j in ((1, 2), (0, 2), (0, 1))]
        s = sum(arcs) / 2
        t = math.tan(s / 2) * math.tan((s - arcs[0]) / 2) * math.tan((s - arcs[1]) / 2) \
            * math.tan((s - arcs[2]) / 2)
        e = 4 * math.atan(math.sqrt(max(t, 0.0)))
        got = om(p, *v)
        assert abs(got) == pytest.approx(e, rel=1e-8, abs=1e-10)


def test_vos_against_fifty_digit_arithmetic():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(6)
    for _ in range(100):
        p = rng.uniform(-20, 20, 3).astype(F32)
        v = rng.uniform(-20, 20, (3, 3)).astype(F32)
        a, b, c = ([mpmath.mpf(float(x)) - mpmath.mpf(float(y)) for x, y in zip(v[i], p)]
                   for i in range(3))
        num = (a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2])
               + a[2] * (b[0] * c[1] - b[1] * c[0]))
        n_ = [mpmath.sqrt(sum(x * x for x in w)) for w in (a, b, c)]
        dot = lambda x, y: sum(i * j for i, j in zip(x, y))
        den = n_[0] * n_[1] * n_[2] + dot(a, b) * n_[2] + dot(a, c) * n_[1] + dot(b, c) * n_[0]
        ref = float(2 * mpmath.atan2(num, den))
        assert om(p, *v) == pytest.approx(ref, abs=1e-14)


def test_far_field_matches_projected_area_over_r2():
    a, b, c = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0)], F32)
    area_n = np.array([0, 0, 0.5])
    for r in (1e2, 1e3):
        for d in ([0, 0, 1], [0.3, 0.4, 0.866]):
            d = np.array(d) / np.linalg.norm(d)
            p = (d * r).astype(F32)
            approx = -np.dot(area_n, p) / r ** 3     # outward normal +z, point above -> negative
            assert om(p, a, b, c) == pytest.approx(approx, rel=3.0 / r)


# ------------------------------------------------------------ exact predicate
def _frac_det(p, a, b, c):
    rows = [[Fraction(float(x)) - Fraction(float(y)) for x, y in zip(v, p)] for v in (a, b, c)]
    (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = rows
    return a0 * (b1 * c2 - b2 * c1) + a1 * (b2 * c0 - b0 * c2) + a2 * (b0 * c1 - b1 * c0)


def test_orient3d_exact_against_rationals():
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(300):
        cases.append(rng.uniform(-100, 100, (4, 3)).astype(F32))
    for _ in range(300):        # points on / next to a plane: near-degenerate
        a, b, c = rng.uniform(-100, 100, (3, 3))
        w = rng.dirichlet((1, 1, 1))
        p = (w[0] * a + w[1] * b + w[2] * c).astype(F32)
        if rng.uniform() < 0.5:
            p = np.nextafter(p, np.float32(1e9))
        cases.append(np.stack([p, a.astype(F32), b.astype(F32), c.astype(F32)]))
    for _ in range(100):        # exactly coplanar: integer lattice points on z = const
        xy = rng.integers(-1000, 1000, (4, 2))
        pts = np.concatenate([xy, np.full((4, 1), 7)], 1).astype(F32)
        cases.append(pts)
    for p, a, b, c in cases:
        exact = _frac_det(p, a, b, c)
        want = (exact > 0) - (exact < 0)
        assert oracle.orient3d_sign(p, a, b, c) == want


# ------------------------------------------------------------------ surfaces
def test_closed_icosphere_winding_is_one_inside_zero_outside():
    uv, f = synth.icosphere(3)
    v = (uv * 80.0).astype(F32)
    a, b, c = (v[f[:, i]].astype(np.float64) for i in range(3))
    n = np.cross(b - a, c - a)
    r_in = np.min(np.abs(np.einsum("ij,ij->i", a, n)) / np.linalg.norm(n, axis=1))
    rng = np.random.default_rng(8)
    d = rng.standard_normal((3, 400))
    d /= np.linalg.norm(d, axis=0)
    inside = (d * rng.uniform(0, r_in * 0.999, 400)).astype(F32)
    outside = (d * rng.uniform(80.001, 300, 400)).astype(F32)
    w_in, _ = oracle.winding(inside, v, f)
    w_out, _ = oracle.winding(outside, v, f)
    assert np.max(np.abs(w_in - 1.0)) < 1e-12
    assert np.max(np.abs(w_out)) < 1e-12


def test_ary_three_sphere_labels_are_analytic():
    g = json.load(open(os.path.join(GOLDEN, "ary_three_sphere.json")))
    uv, f = synth.icosphere(4)
    surfs = []
    for r, lab in zip(g["radii_mm"], g["labels_outermost_first"]):
        surfs.append(synth.Surface(v=(uv * r).astype(F32), f=f.astype(np.int32), label=lab,
                                   center=np.zeros(3)))
    rng = np.random.default_rng(9)
    d = rng.standard_normal((3, 3000))
    d /= np.linalg.norm(d, axis=0)
    rad = rng.uniform(0, 120, 3000)
    # sagitta of subdiv 4 at R = 100 mm is below 0.1 mm: stay 0.2 mm away
    keep = np.all(np.abs(rad[:, None] - np.array(g["radii_mm"])[None, :]) > 0.2, axis=1)
    pts = (d * rad)[:, keep].astype(F32)
    r = np.linalg.norm(pts.astype(np.float64), axis=0)
    want = np.zeros(pts.shape[1], np.int32)
    for rr, lab in zip(g["radii_mm"], g["labels_outermost_first"]):
        want[r < rr] = lab
    got = oracle.label(pts, surfs)
    assert np.array_equal(got, want)


def test_radial_test_matches_winding_labels_on_shells_and_ellipsoids():
    cfg = synth.config_small("head", subdiv=3)
    rng = np.random.default_rng(10)
    pts = np.concatenate([synth.uniform_box(rng, 1500, -100, 100),
                          synth.near_surface_points(rng, cfg.surfaces, 1500, 0.5)], 1)
    assert np.array_equal(oracle.label(pts, cfg.surfaces), oracle.radial_label(pts, cfg.surfaces))


def test_priority_and_background():
    uv, f = synth.icosphere(3)
    big = synth.Surface(v=(uv * 50).astype(F32), f=f.astype(np.int32), label=7, center=np.zeros(3))
    shifted = synth.Surface(v=(uv * 20 + np.array([40, 0, 0])).astype(F32), f=f.astype(np.int32),
                            label=3, center=np.array([40.0, 0, 0]))
    # x = 0: big only; 30: both; 55: shifted only; 70: neither; -40: big only
    pts = np.array([[0, 0, 0], [30, 0, 0], [55, 0, 0], [70, 0, 0], [-40, 0, 0]], F32).T
    # the later surface in the list wins where both enclose the point
    assert list(oracle.label(pts, [big, shifted])) == [7, 3, 3, 0, 7]
    assert list(oracle.label(pts, [shifted, big])) == [7, 7, 3, 0, 7]


def test_points_on_surface_count_as_inside():
    cfg = synth.config_small("sphere", subdiv=2)
    s = cfg.surfaces[0]
    on = synth.face_centroids_on_surface(s)
    lab = oracle.label(on, [s])
    assert np.all(lab == s.label)
    _, on_flag = oracle.winding(on, s.v, s.f)
    assert np.all(on_flag)
