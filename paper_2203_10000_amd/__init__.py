"""Solid-angle labeling of tetrahedral lattices on AMD Instinct MI355X.

Thin ctypes binding of libsal.so (C ABI in include/sal.h).  Every step of the
computation runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory (tensors) and the HIP stream.

The names mirror the C entry points without the `sal_` prefix:
    context_create, surface_set_create, label_points,
    tet_mesh_create_lattice, refine_relabel, tet_mesh_export, label_batch.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsal.so")

SAL_OK = 0
STATUS_NAMES = {0: "SAL_OK", 1: "SAL_ERR_INVALID_ARG", 2: "SAL_ERR_NOT_CLOSED",
                3: "SAL_ERR_ORIENTATION", 4: "SAL_ERR_OUT_OF_MEMORY", 5: "SAL_ERR_DEVICE",
                6: "SAL_ERR_CAPACITY", 7: "SAL_ERR_INTERNAL"}
PREC = {"fp64": 0, "fp32": 1}
WINDING = {None: 0, "f32": 1, "f64": 2}
SURF_AUTO_ORIENT = 1


class SalError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


class SurfaceDesc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("xyz", ctypes.c_void_p),
                ("n_triangles", ctypes.c_int64), ("tri", ctypes.c_void_p),
                ("label", ctypes.c_int32)]


class SurfaceSetInfo(ctypes.Structure):
    _fields_ = [("n_surfaces", ctypes.c_int32), ("n_triangles", ctypes.c_int64),
                ("n_strips", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


class LabelOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("winding_type", ctypes.c_int32),
                ("threshold", ctypes.c_double), ("recheck_band", ctypes.c_double),
                ("kappa", ctypes.c_double), ("points_per_lane", ctypes.c_int32),
                ("block_waves", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("element_rule", ctypes.c_int32), ("cull_bounds", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class LabelStats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_recheck_points", ctypes.c_int64), ("n_recheck_pairs", ctypes.c_int64),
                ("n_band_flags", ctypes.c_int64), ("n_cond_flags", ctypes.c_int64),
                ("n_exact_fallbacks", ctypes.c_int64),
                ("n_recheck_f64_terms", ctypes.c_int64), ("ms_pairloop", ctypes.c_float),
                ("ms_recheck", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("points_per_lane", ctypes.c_int32), ("block_waves", ctypes.c_int32),
                ("n_pairs_culled", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RefineStats(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int64), ("n_boundary", ctypes.c_int64),
                ("n_labeled", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_recheck_pairs", ctypes.c_int64), ("ms_mark", ctypes.c_float),
                ("ms_compact", ctypes.c_float), ("ms_split", ctypes.c_float),
                ("ms_label", ctypes.c_float), ("ms_recheck", ctypes.c_float),
                ("ms_total", ctypes.c_float), ("graph", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ConformInfo(ctypes.Structure):
    _fields_ = [("n_tets", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("n_by_pieces", ctypes.c_int64 * 4),
                ("closure_rounds", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["n_by_pieces"] = list(self.n_by_pieces)
        return d


class SmoothParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("mu", ctypes.c_double),
                ("xi_surface", ctypes.c_double), ("xi_volume", ctypes.c_double),
                ("max_iter_surface", ctypes.c_int32), ("max_iter_volume", ctypes.c_int32)]


class SmoothInfo(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("n_surface_edges", ctypes.c_int64),
                ("n_surface_nodes", ctypes.c_int64), ("n_volume_nodes", ctypes.c_int64),
                ("iters_surface", ctypes.c_int32), ("iters_volume", ctypes.c_int32),
                ("ratio_surface", ctypes.c_double), ("ratio_volume", ctypes.c_double),
                ("ms_build", ctypes.c_float), ("ms_surface", ctypes.c_float),
                ("ms_volume", ctypes.c_float), ("reserved", ctypes.c_int32),
                ("n_entries_surface", ctypes.c_int64), ("n_entries_volume", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class InflateInfo(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int64), ("n_moved", ctypes.c_int64),
                ("n_edges_tested", ctypes.c_int64), ("n_triangle_tests", ctypes.c_int64),
                ("n_triangles", ctypes.c_int64), ("n_bin_items", ctypes.c_int64),
                ("ms_prepare", ctypes.c_float), ("ms_inflate", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [("surfaces", ctypes.c_void_p), ("n_points", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("labels", ctypes.c_void_p)]


_lib = None

# (name, restype, argtypes) for every entry point of include/sal.h
_P = ctypes.c_void_p
_SIGNATURES = [
    ("sal_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("sal_last_error_message", ctypes.c_char_p, []),
    ("sal_abi_version", ctypes.c_int, []),
    ("sal_context_create", ctypes.c_int, [ctypes.c_int, _P, ctypes.POINTER(_P)]),
    ("sal_context_set_stream", ctypes.c_int, [_P, _P]),
    ("sal_context_destroy", None, [_P]),
    ("sal_surface_set_create", ctypes.c_int,
     [_P, ctypes.POINTER(SurfaceDesc), ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(_P)]),
    ("sal_surface_set_destroy", None, [_P]),
    ("sal_surface_set_get_info", ctypes.c_int, [_P, ctypes.POINTER(SurfaceSetInfo)]),
    ("sal_debug_fail_allocation", None, [ctypes.c_int64]),
    ("sal_surface_set_check", ctypes.c_int,
     [ctypes.POINTER(SurfaceDesc), ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(SurfaceSetInfo)]),
    ("sal_label_options_default", None, [ctypes.POINTER(LabelOptions)]),
    ("sal_label_points", ctypes.c_int,
     [_P, _P, ctypes.c_int64, _P, _P, _P, ctypes.POINTER(LabelOptions), _P, _P,
      ctypes.POINTER(LabelStats)]),
    ("sal_label_points_noalloc", ctypes.c_int,
     [_P, _P, ctypes.c_int64, _P, _P, _P, ctypes.POINTER(LabelOptions), _P, _P,
      ctypes.POINTER(LabelStats)]),
    ("sal_tet_mesh_create_lattice", ctypes.c_int,
     [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
      ctypes.POINTER(_P)]),
    ("sal_tet_mesh_destroy", None, [_P]),
    ("sal_refine_relabel", ctypes.c_int,
     [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(LabelOptions), ctypes.POINTER(RefineStats)]),
    ("sal_refine_relabel_converge", ctypes.c_int,
     [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(LabelOptions),
      ctypes.POINTER(RefineStats), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    ("sal_tet_mesh_size", ctypes.c_int,
     [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    ("sal_tet_mesh_export", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    ("sal_tet_mesh_import", ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    ("sal_tet_mesh_conform", ctypes.c_int, [_P, _P, ctypes.POINTER(ConformInfo)]),
    ("sal_tet_mesh_export_conforming", ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    ("sal_smooth_params_default", None, [ctypes.POINTER(SmoothParams)]),
    ("sal_tet_mesh_smooth", ctypes.c_int,
     [_P, _P, ctypes.POINTER(SmoothParams), ctypes.POINTER(SmoothInfo)]),
    ("sal_tet_mesh_inflate", ctypes.c_int,
     [_P, _P, _P, ctypes.c_double, ctypes.POINTER(InflateInfo)]),
    ("sal_label_batch", ctypes.c_int,
     [_P, ctypes.POINTER(Instance), ctypes.c_int32, ctypes.POINTER(LabelOptions),
      ctypes.POINTER(LabelStats)]),
]


def lib():
    """The loaded libsal.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsal.so is not built (run __graft_entry__.build() or "
                              "python paper_2203_10000_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != SAL_OK:
        msg = lib().sal_last_error_message()
        raise SalError(status, msg.decode() if msg else "")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


RULE = {"centroid": 0, "four_nodes": 1}


def label_options(precision="fp32", winding=None, threshold=0.5, band=1e-3, kappa=0.0,
                  points_per_lane=0, block_waves=0, use_graph=False, rule="centroid", cull=False):
    o = LabelOptions()
    lib().sal_label_options_default(ctypes.byref(o))
    o.precision = PREC[precision]
    o.winding_type = WINDING[winding]
    o.threshold = threshold
    o.recheck_band = band
    o.kappa = kappa
    o.points_per_lane = points_per_lane
    o.block_waves = block_waves
    o.use_graph = 1 if use_graph else 0
    o.element_rule = RULE[rule]
    o.cull_bounds = 1 if cull else 0
    return o


class Context:
    """sal_context_create: a device and a HIP stream (torch's current stream
    by default)."""

    def __init__(self, device=0, stream=None):
        import torch
        self.device = device
        with torch.cuda.device(device):
            h = _stream_handle(stream)
        p = ctypes.c_void_p()
        _check(lib().sal_context_create(device, h, ctypes.byref(p)))
        self.handle = p

    def set_stream(self, stream):
        _check(lib().sal_context_set_stream(self.handle, _stream_handle(stream)))

    def close(self):
        if self.handle:
            lib().sal_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def context_create(device=0, stream=None):
    return Context(device, stream)


class SurfaceSet:
    """sal_surface_set_create: surfaces = [(vertices float32 [V,3],
    triangles int32 [T,3], label)], outermost first."""

    def __init__(self, ctx, surfaces, auto_orient=False):
        self.ctx = ctx
        keep = []
        descs = (SurfaceDesc * len(surfaces))()
        for i, s in enumerate(surfaces):
            v, f, label = (s.v, s.f, s.label) if hasattr(s, "v") else s
            v = np.ascontiguousarray(v, dtype=np.float32)
            f = np.ascontiguousarray(f, dtype=np.int32)
            keep += [v, f]
            descs[i].n_vertices = v.shape[0]
            descs[i].xyz = v.ctypes.data
            descs[i].n_triangles = f.shape[0]
            descs[i].tri = f.ctypes.data
            descs[i].label = int(label)
        p = ctypes.c_void_p()
        flags = SURF_AUTO_ORIENT if auto_orient else 0
        _check(lib().sal_surface_set_create(ctx.handle, descs, len(surfaces), flags,
                                            ctypes.byref(p)))
        self.handle = p
        self.n_surfaces = len(surfaces)

    @property
    def info(self):
        i = SurfaceSetInfo()
        _check(lib().sal_surface_set_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in i._fields_}

    def close(self):
        if self.handle:
            lib().sal_surface_set_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def surface_set_check(surfaces, auto_orient=False):
    """sal_surface_set_check: validates surfaces (same list as SurfaceSet) on
    the host, without a device; returns the info dict or raises SalError."""
    keep = []
    descs = (SurfaceDesc * len(surfaces))()
    for i, s in enumerate(surfaces):
        v, f, label = (s.v, s.f, s.label) if hasattr(s, "v") else s
        v = np.ascontiguousarray(v, dtype=np.float32)
        f = np.ascontiguousarray(f, dtype=np.int32)
        keep += [v, f]
        descs[i].n_vertices = v.shape[0]
        descs[i].xyz = v.ctypes.data
        descs[i].n_triangles = f.shape[0]
        descs[i].tri = f.ctypes.data
        descs[i].label = int(label)
    info = SurfaceSetInfo()
    _check(lib().sal_surface_set_check(descs, len(surfaces), SURF_AUTO_ORIENT if auto_orient else 0,
                                       ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def surface_set_create(ctx, surfaces, auto_orient=False):
    return SurfaceSet(ctx, surfaces, auto_orient)


def label_points(ctx, sset, points, precision="fp32", winding=None, stats=False, out=None,
                 **opt):
    """sal_label_points.  points: float32 device tensor [3, N] (or a tuple of
    three [N] tensors).  Returns (labels int32 [N], winding [K, N] or None,
    stats dict or None)."""
    import torch
    x, y, z = (points[0], points[1], points[2])
    for t in (x, y, z):
        assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous()
    n = x.numel()
    labels = out if out is not None else torch.empty(n, dtype=torch.int32, device=x.device)
    w = None
    if winding is not None:
        dt = torch.float32 if winding == "f32" else torch.float64
        w = torch.empty((sset.n_surfaces, n), dtype=dt, device=x.device)
    o = label_options(precision=precision, winding=winding, **opt)
    st = LabelStats() if stats else None
    _check(lib().sal_label_points(ctx.handle, sset.handle, n, _ptr(x), _ptr(y), _ptr(z),
                                  ctypes.byref(o), _ptr(labels), _ptr(w),
                                  ctypes.byref(st) if st is not None else None))
    return labels, w, (st.as_dict() if st is not None else None)


def label_points_noalloc(ctx, sset, points, precision="fp32", winding=None, stats=False,
                         out=None, **opt):
    """sal_label_points_noalloc (same arguments and results as label_points;
    at most 2^20 points; the library allocates no device memory)."""
    import torch
    x, y, z = (points[0], points[1], points[2])
    for t in (x, y, z):
        assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous()
    n = x.numel()
    labels = out if out is not None else torch.empty(n, dtype=torch.int32, device=x.device)
    w = None
    if winding is not None:
        dt = torch.float32 if winding == "f32" else torch.float64
        w = torch.empty((sset.n_surfaces, n), dtype=dt, device=x.device)
    o = label_options(precision=precision, winding=winding, **opt)
    st = LabelStats() if stats else None
    _check(lib().sal_label_points_noalloc(ctx.handle, sset.handle, n, _ptr(x), _ptr(y), _ptr(z),
                                          ctypes.byref(o), _ptr(labels), _ptr(w),
                                          ctypes.byref(st) if st is not None else None))
    return labels, w, (st.as_dict() if st is not None else None)


class TetMesh:
    """sal_tet_mesh_create_lattice / sal_refine_relabel / sal_tet_mesh_export /
    sal_tet_mesh_conform / sal_tet_mesh_export_conforming."""

    def __init__(self, ctx, origin, h, cells):
        self.ctx = ctx
        o = (ctypes.c_double * 3)(*[float(v) for v in origin])
        c = (ctypes.c_int32 * 3)(*[int(v) for v in cells])
        p = ctypes.c_void_p()
        _check(lib().sal_tet_mesh_create_lattice(ctx.handle, o, float(h), c, ctypes.byref(p)))
        self.handle = p

    def size(self):
        n = ctypes.c_int64()
        lv = ctypes.c_int32()
        _check(lib().sal_tet_mesh_size(self.handle, ctypes.byref(n), ctypes.byref(lv)))
        return n.value, lv.value

    def refine_relabel(self, sset, rounds, precision="fp32", **opt):
        o = label_options(precision=precision, **opt)
        st = (RefineStats * (rounds + 1))()
        _check(lib().sal_refine_relabel(self.ctx.handle, self.handle, sset.handle, int(rounds),
                                        ctypes.byref(o), st))
        return [s.as_dict() for s in st]

    def refine_converge(self, sset, finest_level, max_steps=32, precision="fp32", **opt):
        """sal_refine_relabel_converge: (per-step stats, converged)."""
        o = label_options(precision=precision, **opt)
        st = (RefineStats * (max_steps + 1))()
        n = ctypes.c_int32()
        conv = ctypes.c_int32()
        _check(lib().sal_refine_relabel_converge(self.ctx.handle, self.handle, sset.handle,
                                                 int(finest_level), int(max_steps),
                                                 ctypes.byref(o), st, ctypes.byref(n),
                                                 ctypes.byref(conv)))
        return [s.as_dict() for s in st[:n.value + 1]], bool(conv.value)

    def export(self, keys=True, labels=True, centroids=True):
        import torch
        n, _ = self.size()
        dev = torch.device("cuda", self.ctx.device)
        out = {}
        out["keys"] = torch.empty(n, dtype=torch.int64, device=dev) if keys else None
        out["labels"] = torch.empty(n, dtype=torch.int32, device=dev) if labels else None
        cen = torch.empty((3, n), dtype=torch.float32, device=dev) if centroids else None
        out["centroids"] = cen
        _check(lib().sal_tet_mesh_export(
            self.ctx.handle, self.handle, _ptr(out["keys"]), _ptr(out["labels"]),
            _ptr(cen[0] if cen is not None else None), _ptr(cen[1] if cen is not None else None),
            _ptr(cen[2] if cen is not None else None)))
        return out

    def import_leaves(self, keys, labels):
        """sal_tet_mesh_import: keys int64/uint64 and labels int32 device tensors [n]."""
        assert keys.is_cuda and labels.is_cuda and keys.numel() == labels.numel()
        _check(lib().sal_tet_mesh_import(self.ctx.handle, self.handle, keys.numel(),
                                         _ptr(keys.contiguous()), _ptr(labels.contiguous())))

    def conform(self):
        """sal_tet_mesh_conform: the conforming transition mesh; returns its info."""
        info = ConformInfo()
        _check(lib().sal_tet_mesh_conform(self.ctx.handle, self.handle, ctypes.byref(info)))
        self.conform_info = info.as_dict()
        return self.conform_info

    def export_conforming(self):
        """sal_tet_mesh_export_conforming: {"tets" [m, 4] int32 node ids,
        "labels" [m], "xyz" [n, 3] float32, "node_keys" [n] int64}."""
        import torch
        info = self.conform_info
        dev = torch.device("cuda", self.ctx.device)
        out = {"tets": torch.empty((info["n_tets"], 4), dtype=torch.int32, device=dev),
               "labels": torch.empty(info["n_tets"], dtype=torch.int32, device=dev),
               "xyz": torch.empty((info["n_nodes"], 3), dtype=torch.float32, device=dev),
               "node_keys": torch.empty(info["n_nodes"], dtype=torch.int64, device=dev)}
        _check(lib().sal_tet_mesh_export_conforming(
            self.ctx.handle, self.handle, _ptr(out["tets"]), _ptr(out["labels"]),
            _ptr(out["xyz"]), _ptr(out["node_keys"])))
        return out

    def smooth(self, **params):
        """sal_tet_mesh_smooth on the conforming mesh.  params: lam, mu,
        xi_surface, xi_volume, max_iter_surface, max_iter_volume (defaults:
        sal_smooth_params_default).  Returns the info as a dict."""
        p = SmoothParams()
        lib().sal_smooth_params_default(ctypes.byref(p))
        for k, v in params.items():
            if not hasattr(p, k):
                raise TypeError("unknown smoothing parameter %r" % k)
            setattr(p, k, v)
        info = SmoothInfo()
        _check(lib().sal_tet_mesh_smooth(self.ctx.handle, self.handle, ctypes.byref(p),
                                         ctypes.byref(info)))
        return info.as_dict()

    def inflate(self, sset, zeta=0.05):
        """sal_tet_mesh_inflate against the surfaces of `sset`; returns the info."""
        info = InflateInfo()
        _check(lib().sal_tet_mesh_inflate(self.ctx.handle, self.handle, sset.handle, float(zeta),
                                          ctypes.byref(info)))
        return info.as_dict()

    def close(self):
        if self.handle:
            lib().sal_tet_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tet_mesh_create_lattice(ctx, origin, h, cells):
    return TetMesh(ctx, origin, h, cells)


def refine_relabel(ctx, mesh, sset, rounds, **opt):
    assert mesh.ctx is ctx
    return mesh.refine_relabel(sset, rounds, **opt)


def label_batch(ctx, instances, stats=False, **opt):
    """sal_label_batch.  instances: [(SurfaceSet, points [3, N] float32 device
    tensor, labels int32 [N] device tensor)]."""
    arr = (Instance * len(instances))()
    for i, (ss, pts, lab) in enumerate(instances):
        arr[i].surfaces = ss.handle.value
        arr[i].n_points = pts.shape[1]
        arr[i].x = pts[0].data_ptr()
        arr[i].y = pts[1].data_ptr()
        arr[i].z = pts[2].data_ptr()
        arr[i].labels = lab.data_ptr()
    o = label_options(**opt)
    st = (LabelStats * len(instances))() if stats else None
    _check(lib().sal_label_batch(ctx.handle, arr, len(instances), ctypes.byref(o), st))
    return [s.as_dict() for s in st] if stats else None


def exported_names():
    """Entry points this binding declares (all of include/sal.h)."""
    return [s[0] for s in _SIGNATURES]
