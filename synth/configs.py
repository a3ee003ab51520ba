"""The synthetic workloads, one function per configuration.

Each config stands in for the paper's head models (Ary three-sphere and the
FreeSurfer segmentation, whose data are not available): layered shells in the
scalp / skull / CSF / brain order plus small ellipsoids in place of deep
nuclei, with triangle counts and lattice spacings in the paper's range.

Seeds: numpy PCG64 with seed SEED_BASE + 1000 * config + item.
Surfaces are listed outermost first; a later surface has higher priority.
"""
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

from .meshes import (icosphere, geodesic_sphere, sh_shell, ellipsoid,
                     random_rotation, check_closed_oriented, signed_volume,
                     star_shaped_about)
from .points import uniform_box, near_surface_points

SEED_BASE = 220310000
SHELL_RADII = (92.0, 86.0, 80.0, 76.0)      # scalp, skull, CSF, brain (mm)
SHELL_NAMES = ("scalp", "skull", "csf", "brain")
N_SH = 49                                   # (lmax + 1)^2 with lmax = 6


@dataclass
class Surface:
    v: np.ndarray            # float32 [V, 3], mm
    f: np.ndarray            # int32 [T, 3], counter-clockwise seen from outside
    label: int               # compartment id (> 0)
    center: np.ndarray       # float64 [3]; the surface is star-shaped about it
    kind: str = "sphere"

    @property
    def n_tri(self):
        return int(self.f.shape[0])


@dataclass
class Lattice:
    origin: tuple            # (x, y, z) of cell (0, 0, 0), mm
    h: float                 # cell edge, mm
    cells: tuple             # (nx, ny, nz)

    @property
    def n_points(self):
        nx, ny, nz = self.cells
        return 6 * nx * ny * nz


@dataclass
class Config:
    name: str
    surfaces: list
    lattice: Lattice = None
    points: np.ndarray = None          # float32 [3, N] SoA, or None
    rounds: int = 0
    precision: str = "fp32"            # "fp64" (plain) or "fp32" (+ FP64 recheck)
    threshold: float = 0.5
    band: float = 1e-3
    extra: dict = field(default_factory=dict)

    @property
    def n_tri(self):
        return sum(s.n_tri for s in self.surfaces)


def _rng(cfg, item):
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * cfg + item))


@lru_cache(maxsize=None)
def _unit_icosphere(subdiv):
    v, f = icosphere(subdiv)
    return v, f


@lru_cache(maxsize=None)
def _unit_geodesic(nu):
    v, f = geodesic_sphere(nu)
    return v, f


def _finish(v64, f, label, center, kind):
    """Round once to float32 and check the mesh is usable."""
    v32 = v64.astype(np.float32)
    f32 = f.astype(np.int32)
    assert check_closed_oriented(f32), "surface is not a closed oriented manifold"
    assert signed_volume(v32.astype(np.float64), f32) > 0
    assert star_shaped_about(v32.astype(np.float64), f32, center) > 0
    return Surface(v=v32, f=f32, label=int(label),
                   center=np.asarray(center, dtype=np.float64), kind=kind)


def shell_coeffs(cfg=2):
    """Per-shell SH coefficients c_lm ~ N(0, 1) (shared by the c2 and c3 shells)."""
    return [_rng(cfg, k).standard_normal(N_SH) for k in range(4)]


def head_shells(unit_mesh, radii=SHELL_RADII, coeffs=None):
    uv, f = unit_mesh
    coeffs = shell_coeffs() if coeffs is None else coeffs
    out = []
    for k, (r, c) in enumerate(zip(radii, coeffs)):
        out.append(_finish(sh_shell(uv, r, c), f, k + 1, (0.0, 0.0, 0.0),
                           SHELL_NAMES[k] if k < 4 else "shell"))
    return out


def brain_radius(direction, coeffs=None, radius=SHELL_RADII[3], unit_mesh=None):
    """Radial function of the innermost shell along unit `direction`, using the
    same scale as the mesh it was built on."""
    from .meshes import real_sph_harm
    c = shell_coeffs()[3] if coeffs is None else coeffs
    uv = unit_mesh[0]
    fv = c @ real_sph_harm(6, uv)
    s = 0.05 * radius / np.max(np.abs(fv))
    fd = c @ real_sph_harm(6, np.atleast_2d(direction))
    return radius + s * fd


def deep_ellipsoids(rng, n, unit_mesh, axes_lo, axes_hi, first_label,
                    brain_mesh, margin=0.95):
    """Ellipsoids centred inside the innermost shell (rejection sampling)."""
    out = []
    uv, f = unit_mesh
    while len(out) < n:
        c = rng.uniform(-1, 1, 3) * SHELL_RADII[3] * margin
        rc = np.linalg.norm(c)
        if rc > SHELL_RADII[3] * margin:
            continue
        if rc > 0 and rc >= margin * brain_radius(c / rc, unit_mesh=brain_mesh)[0]:
            continue
        axes = rng.uniform(axes_lo, axes_hi, 3)
        rot = random_rotation(rng)
        out.append(_finish(ellipsoid(uv, axes, rot, c), f, first_label + len(out),
                           c, "ellipsoid"))
    return out


def config_c1():
    """One icosphere (subdiv 3, 1280 triangles, R = 80 mm), 32^3-cell lattice."""
    uv, f = _unit_icosphere(3)
    s = _finish(uv * 80.0, f, 1, (0.0, 0.0, 0.0), "sphere")
    lat = Lattice(origin=(-100.0, -100.0, -100.0), h=6.25, cells=(32, 32, 32))
    return Config("c1", [s], lattice=lat, precision="fp64")


def config_c2(cells=100):
    """Four SH-perturbed shells on icosphere subdiv 5 (4 x 20480 triangles),
    2 mm lattice over [-100, 100]^3 (100^3 cells, 6M centroids)."""
    shells = head_shells(_unit_icosphere(5))
    h = 200.0 / cells
    lat = Lattice(origin=(-100.0, -100.0, -100.0), h=h, cells=(cells,) * 3)
    return Config("c2", shells, lattice=lat, precision="fp32")


def config_c3(cells=200, shell_subdiv=6, ell_subdiv=4, n_ell=16, rounds=2):
    """Four shells at subdiv 6 plus 16 ellipsoids (semi-axes U[5, 20] mm) at
    subdiv 4, 1 mm lattice, two refine-and-relabel rounds."""
    shells = head_shells(_unit_icosphere(shell_subdiv))
    rng = _rng(3, 0)
    ells = deep_ellipsoids(rng, n_ell, _unit_icosphere(ell_subdiv), 5.0, 20.0, 5,
                           _unit_icosphere(shell_subdiv))
    h = 200.0 / cells
    lat = Lattice(origin=(-100.0, -100.0, -100.0), h=h, cells=(cells,) * 3)
    return Config("c3", shells + ells, lattice=lat, rounds=rounds, precision="fp32")


def c4_instance(i, t_lo=2e3, t_hi=1e5, n_lo=1e4, n_hi=2e6):
    """One batched-labeling instance: 1-8 surfaces (perturbed spheres or
    ellipsoids) with log-uniform triangle counts, log-uniform point count."""
    rng = _rng(4, i)
    n_surf = int(rng.integers(1, 9))
    surfs = []
    for k in range(n_surf):
        t = np.exp(rng.uniform(np.log(t_lo), np.log(t_hi)))
        nu = max(1, int(round(np.sqrt(t / 20.0))))
        uv, f = _unit_geodesic(nu)
        if rng.uniform() < 0.5:
            r = rng.uniform(20.0, 95.0)
            c = rng.uniform(-10.0, 10.0, 3)
            coeffs = rng.standard_normal(N_SH)
            surfs.append(_finish(sh_shell(uv, r, coeffs, center=c), f, k + 1, c, "sphere"))
        else:
            axes = rng.uniform(5.0, 40.0, 3)
            c = rng.uniform(-50.0, 50.0, 3)
            rot = random_rotation(rng)
            surfs.append(_finish(ellipsoid(uv, axes, rot, c), f, k + 1, c, "ellipsoid"))
    n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
    pts = uniform_box(rng, n, -100.0, 100.0)
    return surfs, pts


def config_c4(n_inst=64, **kw):
    """64 independent instances (list of (surfaces, points))."""
    return [c4_instance(i, **kw) for i in range(n_inst)]


def config_c5(nu=122, n_near=20_000_000, h=0.5, with_lattice=True):
    """Eight ~300k-triangle compartments (4 shells + 4 ellipsoids, geodesic
    frequency nu), a 0.5 mm lattice restricted to the outer shell's bounding
    box, and n_near points offset U[-0.5, 0.5] mm along triangle normals."""
    um = _unit_geodesic(nu)
    shells = head_shells(um)
    rng = _rng(5, 0)
    ells = deep_ellipsoids(rng, 4, um, 10.0, 30.0, 5, um)
    surfs = shells + ells
    lat = None
    if with_lattice:
        lo = surfs[0].v.min(0).astype(np.float64)
        hi = surfs[0].v.max(0).astype(np.float64)
        i0 = np.floor((lo + 100.0) / h).astype(int)
        i1 = np.ceil((hi + 100.0) / h).astype(int)
        lat = Lattice(origin=tuple(float(-100.0 + h * i) for i in i0), h=h,
                      cells=tuple(int(x) for x in (i1 - i0)))
    pts = near_surface_points(_rng(5, 1), surfs, n_near, 0.5) if n_near else None
    return Config("c5", surfs, lattice=lat, points=pts, precision="fp32")


def config_small(kind="shells", cells=24, subdiv=3, seed_item=0):
    """Small workloads for tests: same structure as the full configs, sizes the
    oracle finishes in seconds."""
    if kind == "sphere":
        uv, f = _unit_icosphere(subdiv)
        s = _finish(uv * 80.0, f, 1, (0.0, 0.0, 0.0), "sphere")
        surfs = [s]
    elif kind == "shells":
        surfs = head_shells(_unit_icosphere(subdiv))
    elif kind == "head":
        surfs = head_shells(_unit_icosphere(subdiv))
        rng = _rng(9, seed_item)
        surfs += deep_ellipsoids(rng, 4, _unit_icosphere(max(1, subdiv - 1)), 5.0, 20.0, 5,
                                 _unit_icosphere(subdiv))
    else:
        raise ValueError(kind)
    h = 200.0 / cells
    lat = Lattice(origin=(-100.0, -100.0, -100.0), h=h, cells=(cells,) * 3)
    return Config("small-" + kind, surfs, lattice=lat, precision="fp32")
