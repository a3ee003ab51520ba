"""Conforming transition refinement (paper section 2.1.2, Fig. 2c-e) on the
device, through the C ABI, against the oracle: the same tetrahedra (as sets
of node keys) with the same labels, bit-exact, on leaf sets the oracle builds
by itself from the same surfaces."""
import numpy as np
import pytest

import oracle
import synth
from oracle import conform, kuhn

torch = pytest.importorskip("torch")
import paper_2203_10000_amd as sal  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sal.Context(0)


def _canonical(tets, labels):
    """Rows sorted within and then across, labels carried along."""
    t = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
    order = np.lexsort(t.T[::-1])
    return t[order], np.asarray(labels)[order]


def _device_conform(ctx, cfg, rounds, rule):
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh.refine_relabel(ss, rounds, rule=rule)
    info = mesh.conform()
    e = mesh.export_conforming()
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in e.items()}
    return mesh, ss, info, out


CASES = {
    "head_centroid": ("head", 8, 2, 2, "centroid"),
    "sphere_three_rounds": ("sphere", 6, 2, 3, "centroid"),
    "head_four_nodes": ("head", 8, 2, 2, "four_nodes"),
    # a different cell count on each axis, the box cutting through the sphere:
    # any mix-up of the axes in cell numbering changes the mesh
    "sphere_uneven_box": ("sphere", (8, 7, 6), 2, 3, "centroid"),
}


def _config(kind, cells, subdiv):
    if isinstance(cells, tuple):
        surfaces = synth.config_small(kind, cells=4, subdiv=subdiv).surfaces
        lat = synth.Lattice(origin=(-100.0, -90.0, -75.0), h=25.0, cells=cells)
        return synth.Config("uneven-" + kind, surfaces, lattice=lat, precision="fp32")
    return synth.config_small(kind, cells=cells, subdiv=subdiv)


def _oracle_leaves(cfg, rounds, rule):
    if rule == "centroid":
        leaves, _ = kuhn.refine_relabel(cfg.lattice, lambda p: oracle.label(p, cfg.surfaces),
                                        rounds)
    else:
        leaves, _ = kuhn.refine_relabel_nodes(
            cfg.lattice, lambda p: oracle.enclosure(p, cfg.surfaces),
            lambda m: oracle.mask_label(m, cfg.surfaces), rounds)
    return leaves


@pytest.mark.parametrize("case", list(CASES))
def test_conforming_mesh_equals_the_oracle(ctx, case):
    kind, cells, subdiv, rounds, rule = CASES[case]
    cfg = _config(kind, cells, subdiv)
    leaves = _oracle_leaves(cfg, rounds, rule)
    want_t, want_l, want_rounds = conform.conforming_mesh(leaves.keys, leaves.labels,
                                                          cfg.lattice.cells)
    mesh, _, info, out = _device_conform(ctx, cfg, rounds, rule)
    keys = out["node_keys"]
    ids = out["tets"]
    print(case, info, flush=True)
    assert info["n_tets"] == len(want_t) and info["closure_rounds"] == want_rounds
    # nodes: distinct, ascending, exactly the corners used
    assert np.all(np.diff(keys) > 0)
    assert ids.min() >= 0 and ids.max() < len(keys)
    assert np.array_equal(np.unique(ids), np.arange(len(keys)))
    got_t = keys[ids]
    # the same tetrahedra with the same labels
    gt, gl = _canonical(got_t, out["labels"])
    wt, wl = _canonical(want_t, want_l)
    assert np.array_equal(gt, wt)
    assert np.array_equal(gl, wl)
    # positively oriented, conforming, filling the box exactly
    v6 = conform.volumes6(got_t)
    assert np.all(v6 > 0)
    assert v6.sum() == 6 * np.prod(np.array(cfg.lattice.cells, dtype=np.int64) * kuhn._FINE)
    assert conform.faces_shared_once(got_t, cfg.lattice.cells) == 0
    # pieces per leaf add up
    p = info["n_by_pieces"]
    assert sum(p) == info["n_leaves"]
    assert p[0] + 2 * p[1] + 3 * p[2] + 4 * p[3] == info["n_tets"]
    # node coordinates: origin + key coordinates x h/8, rounded once
    lat = cfg.lattice
    want_xyz = (np.asarray(lat.origin, dtype=np.float64)[None, :]
                + (float(lat.h) / kuhn._FINE) * conform.unkey(keys).astype(np.float64))
    assert np.array_equal(out["xyz"], want_xyz.astype(np.float32))
    # the closure's leaves are the mesh's leaves now
    n_leaves, _ = mesh.size()
    assert n_leaves == info["n_leaves"]


def test_unrefined_lattice_is_its_own_conforming_mesh(ctx):
    cfg = synth.config_small("sphere", cells=3, subdiv=1)
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh.refine_relabel(ss, 0)
    info = mesh.conform()
    assert info["closure_rounds"] == 0
    assert info["n_tets"] == lat.n_points and info["n_by_pieces"][0] == lat.n_points
    out = mesh.export_conforming()
    torch.cuda.synchronize()
    keys = out["node_keys"].cpu().numpy()
    got = np.sort(keys[out["tets"].cpu().numpy()], axis=1)
    want = np.sort(kuhn.node_keys(kuhn.vertices_units(kuhn.level0_keys(lat.cells))), axis=1)
    assert np.array_equal(np.sort(got, axis=0), np.sort(want, axis=0))
    assert len(keys) == np.prod(np.array(lat.cells) + 1)


def test_conforming_mesh_cannot_be_refined_or_conformed_again(ctx):
    cfg = synth.config_small("sphere", cells=4, subdiv=1)
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    fresh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    with pytest.raises(sal.SalError):
        fresh.conform_info = {"n_tets": 0, "n_nodes": 0}
        fresh.export_conforming()
    mesh.refine_relabel(ss, 1)
    mesh.conform()
    with pytest.raises(sal.SalError):
        mesh.refine_relabel(ss, 1)
    with pytest.raises(sal.SalError):
        mesh.conform()
