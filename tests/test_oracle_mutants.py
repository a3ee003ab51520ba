"""The pins must catch plausible mistakes in the oracle: each mutant below is
a copy of the oracle source with one planted error (built on the CPU in a
temporary directory); at least one pin must fail on it."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

SRC = os.path.join(os.path.dirname(oracle.__file__), "sal_oracle.c")
F32 = np.float32

MUTANTS = {
    "D sign of (a.b)|c|": ("double den = la * lb * lc + ab * lc", "double den = la * lb * lc - ab * lc"),
    "D drops (b.c)|a|": (" + ac * lb + bc * la;", " + ac * lb;"),
    "N transposed term": ("double bxc0 = b[1] * c[2] - b[2] * c[1];",
                          "double bxc0 = b[2] * c[1] - b[1] * c[2];"),
    "atan instead of atan2": ("return 2.0 * atan2(num, den);", "return 2.0 * atan(num / den);"),
    "w over 2 pi": ("return (s + comp) / (4.0 * M_PI);", "return (s + comp) / (2.0 * M_PI);"),
    "first surface wins": ("if (on || w >= c->threshold)",
                           "if (label == 0 && (on || w >= c->threshold))"),
    "on-surface ignored": ("if (on || w >= c->threshold)", "if (w >= c->threshold)"),
    "no exact guard": ("if (fabs(num) <= 16.0 * DBL_EPSILON * perm) {", "if (0) {"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, name
    mut = src.replace(old, new, 1)
    c = tmp_path / ("m_%d.c" % abs(hash(name)))
    so = tmp_path / ("m_%d.so" % abs(hash(name)))
    c.write_text(mut)
    inc = os.path.dirname(SRC)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-I", inc,
                           "-o", str(so), str(c), "-lpthread", "-lm"])
    return ctypes.CDLL(str(so))


def _pins_pass(L):
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    L.oracle_tri_solid_angle.argtypes = [f32p] * 4 + [ctypes.POINTER(ctypes.c_int)]
    L.oracle_tri_solid_angle.restype = ctypes.c_double
    L.oracle_label.argtypes = [ctypes.c_int64, f32p, f32p, f32p, ctypes.c_int, i64p, i64p, f32p,
                               i32p, i32p, ctypes.c_double, ctypes.c_int, i32p, ctypes.c_void_p]
    L.oracle_label.restype = ctypes.c_int64
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    L.oracle_winding.argtypes = [ctypes.c_int64, f32p, f32p, f32p, ctypes.c_int64, f32p,
                                 ctypes.c_int64, i32p, ctypes.c_int, f64p, u8p]

    def om(p, a, b, c):
        on = ctypes.c_int(0)
        return L.oracle_tri_solid_angle(*(np.array(x, F32) for x in (p, a, b, c)), ctypes.byref(on))

    def label(pts, surfs):
        vo, to, v, t, lab = oracle.pack_surfaces(surfs)
        out = np.empty(pts.shape[1], np.int32)
        x, y, z = (np.ascontiguousarray(pts[i], F32) for i in range(3))
        L.oracle_label(pts.shape[1], x, y, z, len(surfs), vo, to, v, t, lab, 0.5, 1, out, None)
        return out

    ok = abs(om((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)) - math.pi / 2) < 1e-15
    # regular tetrahedron from its centroid: pi per face
    v = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]
    for skip in range(4):
        f = [v[i] for i in range(4) if i != skip]
        if np.dot(np.cross(np.subtract(f[1], f[0]), np.subtract(f[2], f[0])), f[0]) < 0:
            f = [f[0], f[2], f[1]]
        ok &= abs(om((0, 0, 0), *f) - math.pi) < 1e-14
    # a point behind a face at close range: solid angle beyond pi
    ok &= abs(om((0.1, 0.1, -0.01), (0, 0, 0), (1, 0, 0), (0, 1, 0)) - 5.9) < 0.5
    uv, fc = synth.icosphere(3)
    big = synth.Surface(v=(uv * 50).astype(F32), f=fc.astype(np.int32), label=7, center=np.zeros(3))
    sm = synth.Surface(v=(uv * 20 + np.array([40, 0, 0])).astype(F32), f=fc.astype(np.int32),
                       label=3, center=np.array([40.0, 0, 0]))
    pts = np.array([[0, 0, 0], [30, 0, 0], [55, 0, 0], [70, 0, 0]], F32).T
    ok &= list(label(pts, [big, sm])) == [7, 3, 3, 0]
    # closed sphere: winding number exactly 1 at interior points
    inner = np.array([[0, 0, 0], [10, -5, 3], [-20, 12, 8]], F32).T
    w = np.empty(3, np.float64)
    o = np.empty(3, np.uint8)
    vv = np.ascontiguousarray(big.v.reshape(-1))
    L.oracle_winding(3, *(np.ascontiguousarray(inner[i]) for i in range(3)), len(big.v), vv,
                     len(big.f), np.ascontiguousarray(big.f.reshape(-1)), 1, w, o)
    ok &= bool(np.all(np.abs(w - 1.0) < 1e-12))
    on = synth.face_centroids_on_surface(big, count=50)
    ok &= bool(np.all(label(on, [big]) == 7))
    return bool(ok)


def test_unmutated_copy_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "none", "M_PI", "M_PI"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    assert not _pins_pass(_build(tmp_path, name, old, new))
