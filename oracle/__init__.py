"""FP64 CPU oracle for recursive solid-angle labeling -- TEST INFRASTRUCTURE.

Plain, slow, obviously correct.  Only `tests/`, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library neither
imports nor links it, and the two share no code.

* `liboracle.so` (built from sal_oracle.c with gcc) holds the FP64 pair loop:
  Van Oosterom-Strackee solid angles with an exact-sign guard, compensated
  sums, the label rule and an independent radial inside test.
* `radial.c` (linked into the same library) holds an exact radial inside
  test for star-shaped surfaces with a cube-map index over the cone
  directions, and checkers that form lattice / leaf points themselves and
  count label mismatches, for checking every label of a full-size run.
* `oracle.kuhn` holds the lattice, refinement and boundary rules, written as
  point location in exact dyadic coordinates.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sal_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "radial.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile liboracle.so with gcc (-O2, no FP contraction, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall",
                           "-shared", "-fPIC", "-o", tmp] + _SRCS + ["-lpthread", "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def declare(L):
    """Sets the argument and result types of the oracle's C entry points on a
    loaded library (the oracle itself, or a test's modified copy of it)."""
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    L.oracle_orient3d_sign.argtypes = [f32p] * 4
    L.oracle_orient3d_sign.restype = ctypes.c_int
    L.oracle_orient2d_sign.argtypes = [f32p] * 3 + [ctypes.c_int]
    L.oracle_orient2d_sign.restype = ctypes.c_int
    L.oracle_tri_solid_angle.argtypes = [f32p] * 4 + [ctypes.POINTER(ctypes.c_int)]
    L.oracle_tri_solid_angle.restype = ctypes.c_double
    L.oracle_winding.argtypes = [ctypes.c_int64, f32p, f32p, f32p, ctypes.c_int64, f32p,
                                 ctypes.c_int64, i32p, ctypes.c_int, f64p, u8p]
    L.oracle_winding.restype = None
    L.oracle_label.argtypes = [ctypes.c_int64, f32p, f32p, f32p, ctypes.c_int, i64p, i64p,
                               f32p, i32p, i32p, ctypes.c_double, ctypes.c_int, i32p,
                               ctypes.c_void_p]
    L.oracle_label.restype = ctypes.c_int64
    L.oracle_radial_inside.argtypes = [ctypes.c_int64, f32p, f32p, f32p, f32p, f32p,
                                       ctypes.c_int64, i32p, ctypes.c_int, u8p]
    L.oracle_radial_inside.restype = None
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    L.oracle_enclosure.argtypes = [ctypes.c_int64, f32p, f32p, f32p, ctypes.c_int, i64p,
                                   i64p, f32p, i32p, ctypes.c_double, ctypes.c_int, u64p]
    L.oracle_enclosure.restype = ctypes.c_int64
    vp = ctypes.c_void_p
    L.oracle_radial_new.argtypes = [f32p, ctypes.c_int64, f32p, ctypes.c_int64, i32p,
                                    ctypes.POINTER(ctypes.c_int)]
    L.oracle_radial_new.restype = vp
    L.oracle_radial_free.argtypes = [vp]
    L.oracle_radial_free.restype = None
    L.oracle_radial_stats.argtypes = [vp, i64p]
    L.oracle_radial_stats.restype = None
    L.oracle_radial_query.argtypes = [vp, ctypes.c_int64, f32p, f32p, f32p, ctypes.c_int, u8p]
    L.oracle_radial_query.restype = None
    L.oracle_radial_label.argtypes = [ctypes.c_int64, f32p, f32p, f32p, ctypes.c_int, vp,
                                      i32p, ctypes.c_int, vp, vp]
    L.oracle_radial_label.restype = ctypes.c_int64
    L.oracle_radial_check_lattice.argtypes = [f64p, ctypes.c_double, i64p, ctypes.c_int64,
                                              ctypes.c_int64, i32p, ctypes.c_int, vp, i32p,
                                              ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                              i64p, ctypes.c_int64]
    L.oracle_radial_check_lattice.restype = ctypes.c_int64
    L.oracle_radial_check_keys.argtypes = [f64p, ctypes.c_double, ctypes.c_int64, u64p, i32p,
                                           ctypes.c_int, ctypes.c_int, vp, i32p, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int64), i64p,
                                           ctypes.c_int64]
    L.oracle_radial_check_keys.restype = ctypes.c_int64
    L.oracle_leaf_points.argtypes = [f64p, ctypes.c_double, ctypes.c_int64, u64p,
                                     ctypes.c_int, f32p]
    L.oracle_leaf_points.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def host_threads():
    """Host cores this process may run on."""
    return len(os.sched_getaffinity(0))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def orient3d_sign(p, v0, v1, v2):
    """Exact sign of det[v0 - p, v1 - p, v2 - p] for float32 inputs."""
    return lib().oracle_orient3d_sign(_f32(p), _f32(v0), _f32(v1), _f32(v2))


def orient2d_sign(a, b, c, drop):
    return lib().oracle_orient2d_sign(_f32(a), _f32(b), _f32(c), int(drop))


def tri_solid_angle(p, v0, v1, v2):
    """(Omega, on_triangle) for one triangle seen from p (float32 inputs)."""
    on = ctypes.c_int(0)
    om = lib().oracle_tri_solid_angle(_f32(p), _f32(v0), _f32(v1), _f32(v2), ctypes.byref(on))
    return om, bool(on.value)


def _soa(points):
    pts = np.asarray(points)
    assert pts.ndim == 2 and pts.shape[0] == 3
    return _f32(pts[0]), _f32(pts[1]), _f32(pts[2])


def winding(points, v, f, n_threads=0):
    """Winding numbers w = Omega / 4 pi of one surface at points [3, N]."""
    x, y, z = _soa(points)
    n = x.size
    w = np.empty(n, dtype=np.float64)
    on = np.empty(n, dtype=np.uint8)
    vv = _f32(v).reshape(-1)
    ff = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
    lib().oracle_winding(n, x, y, z, vv.size // 3, vv, ff.size // 3, ff, int(n_threads), w, on)
    return w, on.astype(bool)


def pack_surfaces(surfaces):
    """Concatenate surfaces (objects with .v, .f, .label) for the C calls."""
    vert_off = np.zeros(len(surfaces) + 1, dtype=np.int64)
    tri_off = np.zeros(len(surfaces) + 1, dtype=np.int64)
    for i, s in enumerate(surfaces):
        vert_off[i + 1] = vert_off[i] + s.v.shape[0]
        tri_off[i + 1] = tri_off[i] + s.f.shape[0]
    verts = _f32(np.concatenate([s.v for s in surfaces]).reshape(-1))
    tris = np.ascontiguousarray(np.concatenate([s.f for s in surfaces]), dtype=np.int32).reshape(-1)
    labels = np.array([s.label for s in surfaces], dtype=np.int32)
    return vert_off, tri_off, verts, tris, labels


def label(points, surfaces, threshold=0.5, n_threads=0, want_w=False):
    """Compartment labels (int32 [N]) of points [3, N]; surfaces outermost
    first, the later one winning.  Optionally the winding numbers [K, N]."""
    x, y, z = _soa(points)
    n = x.size
    vert_off, tri_off, verts, tris, labs = pack_surfaces(surfaces)
    out = np.empty(n, dtype=np.int32)
    w = np.empty((len(surfaces), n), dtype=np.float64) if want_w else None
    lib().oracle_label(n, x, y, z, len(surfaces), vert_off, tri_off, verts, tris, labs,
                       float(threshold), int(n_threads), out,
                       w.ctypes.data if want_w else None)
    return (out, w) if want_w else out


def enclosure(points, surfaces, threshold=0.5, n_threads=0):
    """uint64 [N]: bit s set when the point is enclosed by surface s (the
    test of label(): w >= threshold or on the surface)."""
    x, y, z = _soa(points)
    n = x.size
    vert_off, tri_off, verts, tris, _ = pack_surfaces(surfaces)
    out = np.empty(n, dtype=np.uint64)
    r = lib().oracle_enclosure(n, x, y, z, len(surfaces), vert_off, tri_off, verts, tris,
                               float(threshold), int(n_threads), out)
    if r < 0:
        raise ValueError("at most 64 surfaces")
    return out


def mask_label(masks, surfaces):
    """Label of each enclosure mask: the latest surface in the list whose bit
    is set (surfaces outermost first), 0 when none is."""
    masks = np.asarray(masks, dtype=np.uint64)
    labs = np.zeros(masks.shape, dtype=np.int32)
    for s, surf in enumerate(surfaces):
        labs[(masks >> np.uint64(s)) & np.uint64(1) == 1] = surf.label
    return labs


def radial_inside(points, surface, n_threads=0):
    """Exact star-shaped inside test: 1 inside, 0 outside, 2 on the surface."""
    x, y, z = _soa(points)
    n = x.size
    out = np.empty(n, dtype=np.uint8)
    c = _f32(np.asarray(surface.center, dtype=np.float64))
    vv = _f32(surface.v).reshape(-1)
    ff = np.ascontiguousarray(surface.f, dtype=np.int32).reshape(-1)
    lib().oracle_radial_inside(n, x, y, z, c, vv, ff.size // 3, ff, int(n_threads), out)
    return out


def radial_label(points, surfaces, n_threads=0):
    """Labels from the radial test alone (every surface star-shaped about its
    centre): the later enclosing (or touching) surface wins."""
    pts = np.asarray(points)
    out = np.zeros(pts.shape[1], dtype=np.int32)
    for s in surfaces:
        r = radial_inside(pts, s, n_threads)
        out[r > 0] = s.label
    return out


# ------------------------------------------------ indexed exact radial test
RADIAL_STATUS = {1: "a cone (centre, triangle) is not positively oriented",
                 2: "the winding number at the centre is not 1",
                 3: "bad arguments or out of memory"}


class RadialIndex:
    """Exact radial inside test of one star-shaped surface with a direction
    index (radial.c): O(1) expected per query instead of O(triangles)."""

    def __init__(self, surface, L=None):
        L = lib() if L is None else L
        self._L = L
        c = _f32(np.asarray(surface.center, dtype=np.float64))
        vv = _f32(surface.v).reshape(-1)
        ff = np.ascontiguousarray(surface.f, dtype=np.int32).reshape(-1)
        st = ctypes.c_int(0)
        self._h = L.oracle_radial_new(c, vv.size // 3, vv, ff.size // 3, ff, ctypes.byref(st))
        if not self._h:
            raise ValueError("radial index: " + RADIAL_STATUS.get(st.value, str(st.value)))
        self.label = int(surface.label)

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            self._L.oracle_radial_free(h)

    def stats(self):
        out = np.zeros(6, dtype=np.int64)
        self._L.oracle_radial_stats(self._h, out)
        return dict(zip(("triangles", "grid", "entries", "wide", "fallbacks", "undecided"),
                        (int(x) for x in out)))

    def query(self, points, n_threads=0):
        """0 outside, 1 inside, 2 on the surface, 3 no cone holds the point."""
        x, y, z = _soa(points)
        out = np.empty(x.size, dtype=np.uint8)
        self._L.oracle_radial_query(self._h, x.size, x, y, z, int(n_threads), out)
        return out


class RadialSet:
    """Indexes of a list of surfaces (outermost first, the later one winning)."""

    def __init__(self, surfaces, L=None):
        self._L = lib() if L is None else L
        self.index = [RadialIndex(s, self._L) for s in surfaces]
        self._ptrs = (ctypes.c_void_p * len(self.index))(*[r._h for r in self.index])
        self.labels = np.array([r.label for r in self.index], dtype=np.int32)

    def __len__(self):
        return len(self.index)

    def fallbacks(self):
        return sum(r.stats()["fallbacks"] for r in self.index)

    def label(self, points, n_threads=0, want_masks=False):
        """Labels (int32 [N]) and, optionally, enclosure masks (uint64 [N])."""
        x, y, z = _soa(points)
        n = x.size
        lab = np.empty(n, dtype=np.int32)
        masks = np.empty(n, dtype=np.uint64) if want_masks else None
        if want_masks and len(self) > 64:
            raise ValueError("at most 64 surfaces")
        und = self._L.oracle_radial_label(n, x, y, z, len(self), ctypes.cast(self._ptrs, ctypes.c_void_p),
                                        self.labels, int(n_threads), lab.ctypes.data,
                                        masks.ctypes.data if want_masks else None)
        if und:
            raise RuntimeError("radial test: %d undecided queries" % und)
        return (lab, masks) if want_masks else lab

    def _result(self, mism, und, bad, cap):
        if und.value:
            raise RuntimeError("radial test: %d undecided queries" % und.value)
        return int(mism), np.sort(bad[:min(int(mism), cap)])

    def check_lattice(self, lattice, got, first=0, n_threads=0, cap=64):
        """Mismatches between `got` (labels of lattice points first .. first +
        len(got) - 1) and the radial labels of those centroids: (count,
        sorted point numbers of up to `cap` of them)."""
        got = np.ascontiguousarray(got, dtype=np.int32)
        bad = np.zeros(max(cap, 1), dtype=np.int64)
        und = ctypes.c_int64(0)
        mism = self._L.oracle_radial_check_lattice(
            np.asarray(lattice.origin, dtype=np.float64), float(lattice.h),
            np.asarray(lattice.cells, dtype=np.int64), int(first), got.size, got, len(self),
            ctypes.cast(self._ptrs, ctypes.c_void_p), self.labels, int(n_threads),
            ctypes.byref(und), bad, int(cap))
        return self._result(mism, und, bad, cap)

    def check_keys(self, origin, h, keys, got, rule="centroid", n_threads=0, cap=64):
        """The same for leaves given by key, under the centroid rule or the
        four-node rule; the returned positions index `keys`."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        got = np.ascontiguousarray(got, dtype=np.int32)
        assert keys.size == got.size
        r = {"centroid": 0, "four_nodes": 1}[rule]
        if r == 1 and len(self) > 64:
            raise ValueError("at most 64 surfaces")
        bad = np.zeros(max(cap, 1), dtype=np.int64)
        und = ctypes.c_int64(0)
        mism = self._L.oracle_radial_check_keys(
            np.asarray(origin, dtype=np.float64), float(h), keys.size, keys, got, r, len(self),
            ctypes.cast(self._ptrs, ctypes.c_void_p), self.labels, int(n_threads),
            ctypes.byref(und), bad, int(cap))
        return self._result(mism, und, bad, cap)


def leaf_points(origin, h, keys, rule="centroid", L=None):
    """The points radial checks form from keys: centroids float32 [3, n]
    (centroid rule) or vertices float32 [n, 4, 3] (four-node rule)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    r = {"centroid": 0, "four_nodes": 1}[rule]
    out = np.empty((keys.size, 4 if r else 1, 3), dtype=np.float32)
    (lib() if L is None else L).oracle_leaf_points(np.asarray(origin, dtype=np.float64), float(h), keys.size, keys, r,
                             out.reshape(-1))
    return out[:, 0, :].T.copy() if r == 0 else out
