"""Inflation (paper section 2.2.2) on the device, through the C ABI, against
the oracle run on its own conforming mesh of the same surfaces: the crossing
arithmetic is the same sequence of double operations on both sides, so the
moved positions are bit-identical."""
import numpy as np
import pytest

import oracle
import synth
from oracle import conform, inflate, kuhn, smooth

torch = pytest.importorskip("torch")
import paper_2203_10000_amd as sal  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sal.Context(0)


def _oracle_mesh(cfg, rounds):
    leaves, _ = kuhn.refine_relabel(cfg.lattice, lambda p: oracle.label(p, cfg.surfaces), rounds)
    t, lab, _ = conform.conforming_mesh(leaves.keys, leaves.labels, cfg.lattice.cells)
    nodes, inv = np.unique(t.reshape(-1), return_inverse=True)
    lat = cfg.lattice
    xyz = (np.asarray(lat.origin)[None, :]
           + (lat.h / kuhn._FINE) * conform.unkey(nodes).astype(np.float64)).astype(np.float32)
    return nodes, inv.reshape(-1, 4), lab, xyz


def _device(ctx, cfg, rounds):
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    mesh.refine_relabel(ss, rounds)
    mesh.conform()
    return mesh, ss


@pytest.mark.parametrize("kind,cells,subdiv,rounds", [("sphere", 6, 2, 2), ("head", 8, 2, 2)])
def test_inflation_equals_the_oracle(ctx, kind, cells, subdiv, rounds):
    cfg = synth.config_small(kind, cells=cells, subdiv=subdiv)
    nodes, ids, lab, xyz0 = _oracle_mesh(cfg, rounds)
    e, surf = smooth.edges(ids, lab)
    mv = np.zeros(len(nodes), bool)
    mv[e[surf].reshape(-1)] = True
    mv &= ~smooth.on_box(nodes, cfg.lattice.cells)
    want, chosen, _ = inflate.inflate(xyz0.astype(np.float64), e, mv, nodes,
                                      inflate.triangles(cfg.surfaces), 0.05)
    mesh, ss = _device(ctx, cfg, rounds)
    info = mesh.inflate(ss, 0.05)
    out = mesh.export_conforming()
    torch.cuda.synchronize()
    print(kind, info, flush=True)
    assert np.array_equal(out["node_keys"].cpu().numpy(), nodes)
    got = out["xyz"].cpu().numpy()
    assert info["n_candidates"] == mv.sum()
    assert info["n_moved"] == np.sum(chosen >= 0)
    assert info["n_triangles"] == sum(len(s.f) for s in cfg.surfaces)
    bad = np.nonzero(np.any(got != want.astype(np.float32), axis=1))[0]
    assert len(bad) == 0, (len(bad), bad[:5], got[bad[:5]], want[bad[:5]])
    assert np.array_equal(got[~mv], xyz0[~mv])


def test_zero_zeta_moves_nothing_and_arguments_are_checked(ctx):
    cfg = synth.config_small("sphere", cells=4, subdiv=1)
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    mesh.refine_relabel(ss, 1)
    with pytest.raises(sal.SalError):
        mesh.inflate(ss)
    mesh.conform()
    before = mesh.export_conforming()["xyz"].cpu().numpy()
    info = mesh.inflate(ss, 0.0)
    assert info["n_moved"] > 0
    assert np.array_equal(mesh.export_conforming()["xyz"].cpu().numpy(), before)
    for z in (-0.1, 1.0, float("nan")):
        with pytest.raises(sal.SalError):
            mesh.inflate(ss, z)


def test_smoothing_then_inflation_matches_the_oracle_pipeline(ctx):
    """Section 2.2 order: smoothing, then inflation.  The smoothed positions
    differ from the oracle's by float32 rounding, so a node whose nearest
    crossing is a near tie may pick another edge; all others agree to the
    rounding bound of the smoothing test plus the inflation step."""
    cfg = synth.config_small("sphere", cells=6, subdiv=2)
    nodes, ids, lab, xyz0 = _oracle_mesh(cfg, 2)
    box = smooth.on_box(nodes, cfg.lattice.cells)
    sm, _ = smooth.smooth_mesh(ids, lab, xyz0.astype(np.float64), box)
    e, surf = smooth.edges(ids, lab)
    mv = np.zeros(len(nodes), bool)
    mv[e[surf].reshape(-1)] = True
    mv &= ~box
    want, _, _ = inflate.inflate(sm, e, mv, nodes, inflate.triangles(cfg.surfaces), 0.05)
    mesh, ss = _device(ctx, cfg, 2)
    mesh.smooth()
    mesh.inflate(ss, 0.05)
    got = mesh.export_conforming()["xyz"].cpu().numpy().astype(np.float64)
    err = np.abs(got - want).max(axis=1)
    tol = 2.0 ** -24 * np.abs(want).max() * 8
    print("max err %.3g, nodes above %.3g: %d of %d" % (err.max(), tol, np.sum(err > tol), len(err)))
    assert np.sum(err > tol) <= max(1, len(err) // 1000)


def test_mesh_without_an_interface(ctx):
    """A lattice that the surface does not reach: every label is 0, the mesh
    stays the Kuhn lattice, the surface phase of the smoothing has nothing to
    move (no iteration), the volume phase leaves the symmetric interior where
    it is, and inflation has no candidate."""
    surfaces = synth.config_small("sphere", cells=4, subdiv=1).surfaces
    lat = synth.Lattice(origin=(150.0, 150.0, 150.0), h=25.0, cells=(4, 5, 3))
    cfg = synth.Config("outside", surfaces, lattice=lat, precision="fp32")
    nodes, ids, lab, xyz0 = _oracle_mesh(cfg, 2)
    assert not np.any(lab)
    box = smooth.on_box(nodes, lat.cells)
    want, winfo = smooth.smooth_mesh(ids, lab, xyz0.astype(np.float64), box)
    assert winfo["iters_surface"] == 0 and winfo["n_surface_edges"] == 0
    mesh, ss = _device(ctx, cfg, 2)
    out = mesh.export_conforming()
    assert np.array_equal(out["node_keys"].cpu().numpy(), nodes)
    assert np.array_equal(out["xyz"].cpu().numpy(), xyz0)
    sinfo = mesh.smooth()
    print(sinfo, flush=True)
    for k in ("n_edges", "n_surface_edges", "n_surface_nodes", "n_volume_nodes",
              "iters_surface", "iters_volume"):
        assert sinfo[k] == winfo[k], k
    got = mesh.export_conforming()["xyz"].cpu().numpy().astype(np.float64)
    assert np.abs(got - want).max() <= 2.0 ** -24 * np.abs(want).max() * 8
    info = mesh.inflate(ss, 0.05)
    assert info["n_candidates"] == 0 and info["n_moved"] == 0
    assert np.array_equal(mesh.export_conforming()["xyz"].cpu().numpy().astype(np.float64), got)


def test_inflation_on_a_lattice_with_uneven_axes(ctx):
    """Different cell counts per axis, the box cutting through the sphere: the
    triangle bins and the box test are numbered per axis, so a mix-up of the
    axes changes the moved positions."""
    surfaces = synth.config_small("sphere", cells=4, subdiv=2).surfaces
    lat = synth.Lattice(origin=(-100.0, -90.0, -75.0), h=25.0, cells=(8, 7, 6))
    cfg = synth.Config("uneven-sphere", surfaces, lattice=lat, precision="fp32")
    nodes, ids, lab, xyz0 = _oracle_mesh(cfg, 2)
    e, surf = smooth.edges(ids, lab)
    mv = np.zeros(len(nodes), bool)
    mv[e[surf].reshape(-1)] = True
    mv &= ~smooth.on_box(nodes, lat.cells)
    want, chosen, _ = inflate.inflate(xyz0.astype(np.float64), e, mv, nodes,
                                      inflate.triangles(surfaces), 0.05)
    mesh, ss = _device(ctx, cfg, 2)
    info = mesh.inflate(ss, 0.05)
    out = mesh.export_conforming()
    assert np.array_equal(out["node_keys"].cpu().numpy(), nodes)
    assert info["n_candidates"] == mv.sum() and info["n_moved"] == np.sum(chosen >= 0)
    assert info["n_moved"] > 0
    got = out["xyz"].cpu().numpy()
    bad = np.nonzero(np.any(got != want.astype(np.float32), axis=1))[0]
    assert len(bad) == 0, (len(bad), bad[:5])
