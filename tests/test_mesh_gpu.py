"""Kuhn lattice, refine-and-relabel and export (HIP, through the C ABI)
against the oracle: leaf keys and labels bit-exact."""
import numpy as np
import pytest

import oracle
import synth
from oracle import kuhn

torch = pytest.importorskip("torch")
import paper_2203_10000_amd as sal  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sal.Context(0)


def export_np(mesh):
    e = mesh.export()
    torch.cuda.synchronize()
    keys = e["keys"].cpu().numpy().view(np.uint64)
    return keys, e["labels"].cpu().numpy(), e["centroids"].cpu().numpy()


def test_lattice_keys_and_centroids(ctx):
    lat = synth.config_c1().lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    keys, labels, cen = export_np(mesh)
    assert np.array_equal(keys, kuhn.level0_keys(lat.cells))
    assert np.array_equal(cen, kuhn.centroids_mm(keys, lat.origin, lat.h))
    assert np.all(labels == -2)                          # not labeled yet
    assert mesh.size() == (lat.n_points, 0)


def test_lattice_with_non_dyadic_spacing(ctx):
    lat = synth.Lattice(origin=(-100.0, -100.0, -100.0), h=200.0 / 24, cells=(24, 23, 22))
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    keys, _, cen = export_np(mesh)
    assert np.array_equal(cen, kuhn.centroids_mm(keys, lat.origin, lat.h))


def test_c1_full_lattice_plain_fp64(ctx):
    """One icosphere (1280 triangles), 32^3 cells x 6 = 196,608 centroids."""
    cfg = synth.config_c1()
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    st = mesh.refine_relabel(ss, 0, precision="fp64")
    keys, labels, cen = export_np(mesh)
    pts = kuhn.centroids_mm(keys, lat.origin, lat.h)
    want, w_ref = oracle.label(pts, cfg.surfaces, want_w=True)
    assert np.array_equal(labels, want)
    assert st[0]["n_labeled"] == 196608 and st[0]["n_pairs"] == 196608 * 1280
    # the FP64 winding number of every centroid, through sal_label_points
    dev = torch.from_numpy(pts).to("cuda:0").contiguous()
    lab2, w, _ = sal.label_points(ctx, ss, dev, precision="fp64", winding="f64")
    torch.cuda.synchronize()
    assert np.array_equal(lab2.cpu().numpy(), want)
    assert np.abs(w.cpu().numpy() - w_ref).max() < 1e-12


def _refine_case(ctx, precision, cells=16, rounds=2):
    cfg = synth.config_small("head", cells=cells, subdiv=3)
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    stats = mesh.refine_relabel(ss, rounds, precision=precision)
    keys, labels, _ = export_np(mesh)
    return cfg, keys, labels, stats, mesh


@pytest.fixture(scope="module")
def refine_oracle():
    cfg = synth.config_small("head", cells=16, subdiv=3)
    leaves, st = kuhn.refine_relabel(cfg.lattice, lambda p: oracle.label(p, cfg.surfaces), 2)
    return leaves, st


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_refine_relabel_two_rounds(ctx, refine_oracle, precision):
    leaves, ost = refine_oracle
    cfg, keys, labels, stats, mesh = _refine_case(ctx, precision)
    order = np.argsort(keys)
    assert np.array_equal(keys[order], leaves.keys)
    assert np.array_equal(labels[order], leaves.labels)
    for r in range(1, 3):
        assert stats[r]["n_boundary"] == ost[r]["boundary"]
        assert stats[r]["n_labeled"] == ost[r]["children"]
        assert stats[r]["n_leaves"] == ost[r]["leaves"]
    n0 = cfg.lattice.n_points
    assert mesh.size()[0] == n0 + 7 * sum(s["n_boundary"] for s in stats)
    # export is ordered by level
    lv = kuhn.decode(keys)[0]
    assert np.all(np.diff(lv) >= 0) and mesh.size()[1] == 2


def test_refine_in_two_calls_equals_one(ctx):
    cfg = synth.config_small("head", cells=12, subdiv=3)
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    a = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    a.refine_relabel(ss, 2)
    b = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    b.refine_relabel(ss, 1)
    b.refine_relabel(ss, 1)
    ka, la, _ = export_np(a)
    kb, lb, _ = export_np(b)
    assert np.array_equal(ka, kb) and np.array_equal(la, lb)


def test_refinement_depth_limit(ctx):
    cfg = synth.config_small("sphere", cells=8, subdiv=2)
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    with pytest.raises(sal.SalError) as e:
        mesh.refine_relabel(ss, 4)
    assert e.value.status == 6       # SAL_ERR_CAPACITY
    mesh.refine_relabel(ss, 3)       # three levels are allowed
    assert mesh.size()[1] == 3


def test_c2_full_size_sampled(ctx):
    """The benchmark workload: four 20,480-triangle shells, 6M lattice
    centroids, FP32 + recheck.  Labels checked against the oracle on a sample
    of uniform indices plus points within 1 mm of a shell."""
    cfg = synth.config_c2()
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    st = mesh.refine_relabel(ss, 0, precision="fp32")
    keys, labels, cen = export_np(mesh)
    assert len(keys) == 6_000_000 and np.all(labels >= 0)
    rng = np.random.default_rng(12)
    r = np.linalg.norm(cen.astype(np.float64), axis=0)
    near = np.nonzero(np.min(np.abs(r[:, None] - np.array([92, 86, 80, 76.0])), axis=1) < 6.0)[0]
    idx = np.unique(np.concatenate([rng.choice(len(keys), 20000, replace=False),
                                    rng.choice(near, 20000, replace=False)]))
    want = oracle.label(np.ascontiguousarray(cen[:, idx]), cfg.surfaces)
    assert np.array_equal(labels[idx], want)
    assert st[0]["n_recheck_pairs"] < 0.01 * len(keys)


# ------------------------------------------------------- four-node rule
@pytest.fixture(scope="module")
def node_oracle():
    cfg = synth.config_small("head", cells=12, subdiv=3)
    leaves, st = kuhn.refine_relabel_nodes(
        cfg.lattice, lambda p: oracle.enclosure(p, cfg.surfaces),
        lambda m: oracle.mask_label(m, cfg.surfaces), 2)
    return cfg, leaves, st


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_four_node_rule_two_rounds(ctx, node_oracle, precision):
    """Section 2.1.3 read literally: nodes labeled, a tetrahedron enclosed by
    a surface when its four nodes are, new nodes only after each split."""
    cfg, leaves, ost = node_oracle
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    st = mesh.refine_relabel(ss, 2, precision=precision, rule="four_nodes")
    keys, labels, _ = export_np(mesh)
    order = np.argsort(keys)
    assert np.array_equal(keys[order], leaves.keys)
    assert np.array_equal(labels[order], leaves.labels)
    n_nodes = (lat.cells[0] + 1) * (lat.cells[1] + 1) * (lat.cells[2] + 1)
    assert st[0]["n_labeled"] == n_nodes
    for r in (1, 2):
        assert st[r]["n_boundary"] == ost[r]["boundary"]
        assert st[r]["n_leaves"] == ost[r]["leaves"]
        assert st[r]["n_labeled"] == ost[r]["nodes"]   # each new node labeled once


def test_four_node_rule_rejects_the_round_graph(ctx, node_oracle):
    """use_graph applies to the centroid rule: with the four-node rule the call
    fails before anything is labeled."""
    cfg, _, _ = node_oracle
    lat = cfg.lattice
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    with pytest.raises(sal.SalError) as e:
        mesh.refine_relabel(ss, 2, rule="four_nodes", use_graph=True)
    assert e.value.status == 1
    _, labels, _ = export_np(mesh)
    assert np.all(labels == -2) and mesh.size() == (lat.n_points, 0)


@pytest.mark.parametrize("rule", ["centroid", "four_nodes"])
def test_converging_recursion_matches_the_oracle(ctx, rule):
    """Section 2.1.3 item 2 / Fig. 3: steps repeat until no boundary leaf
    coarser than the finest level is left; leaves, labels and the per-step
    counts equal the oracle's."""
    cfg = synth.config_small("head", cells=10, subdiv=3)
    lat = cfg.lattice
    if rule == "centroid":
        want, ost = kuhn.refine_relabel(lat, lambda p: oracle.label(p, cfg.surfaces), 2,
                                        converge=True)
    else:
        want, ost = kuhn.refine_relabel_nodes(lat, lambda p: oracle.enclosure(p, cfg.surfaces),
                                              lambda m: oracle.mask_label(m, cfg.surfaces), 2,
                                              converge=True)
    assert len(ost) - 1 > 2                      # the recursion goes past two steps
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    st, conv = mesh.refine_converge(ss, 2, max_steps=16, rule=rule)
    assert conv and len(st) == len(ost)
    keys, labels, _ = export_np(mesh)
    order = np.argsort(keys)
    assert np.array_equal(keys[order], want.keys)
    assert np.array_equal(labels[order], want.labels)
    for r in range(1, len(st)):
        assert st[r]["n_boundary"] == ost[r]["boundary"]
        assert st[r]["n_leaves"] == ost[r]["leaves"]
        assert st[r]["n_labeled"] == ost[r]["labeled" if rule == "centroid" else "nodes"]
    # a second call finds nothing to split; a cap of one step reports no convergence
    st2, conv2 = mesh.refine_converge(ss, 2, rule=rule)
    assert conv2 and len(st2) == 1 and mesh.size()[0] == len(want.keys)
    other = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    st3, conv3 = other.refine_converge(ss, 2, max_steps=1, rule=rule)
    assert not conv3 and len(st3) == 2


def test_element_rule_is_fixed_by_the_first_labeling(ctx):
    cfg = synth.config_small("sphere", cells=6, subdiv=2)
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    mesh.refine_relabel(ss, 1)
    with pytest.raises(sal.SalError) as e:
        mesh.refine_relabel(ss, 1, rule="four_nodes")
    assert e.value.status == 1
    other = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    other.refine_relabel(ss, 1, rule="four_nodes")
    other.refine_relabel(ss, 1, rule="four_nodes")
    assert other.size()[1] == 2
