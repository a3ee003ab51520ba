"""Refine-and-relabel rounds run as launches of one captured round graph
(sal_refine_relabel with use_graph): the same leaves, order and labels as the
host-driven rounds and as the oracle, across replays and capacity stops."""
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
    return e["keys"].cpu().numpy().view(np.uint64), e["labels"].cpu().numpy()


def _mesh(ctx, cfg):
    lat = cfg.lattice
    return sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_rounds_match_the_oracle(ctx, precision):
    cfg = synth.config_small("head", cells=16, subdiv=3)
    leaves, ost = kuhn.refine_relabel(cfg.lattice, lambda p: oracle.label(p, cfg.surfaces), 2)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh = _mesh(ctx, cfg)
    stats = mesh.refine_relabel(ss, 2, precision=precision, use_graph=True)
    keys, labels = export_np(mesh)
    order = np.argsort(keys)
    assert np.array_equal(keys[order], leaves.keys)
    assert np.array_equal(labels[order], leaves.labels)
    assert stats[0]["graph"] == 0                       # the lattice is labeled host-driven
    for r in (1, 2):
        assert stats[r]["graph"] in (1, 2)
        assert stats[r]["n_boundary"] == ost[r]["boundary"]
        assert stats[r]["n_labeled"] == ost[r]["children"]
        assert stats[r]["n_leaves"] == ost[r]["leaves"]
    assert mesh.size() == (len(leaves.keys), 2)


def test_graph_replays_across_calls_match_host_driven_rounds(ctx):
    """Three one-round calls: the first captures, the next two replay the
    kept graph, with other labeling work and synchronisations in between;
    after every call the mesh equals the host-driven one."""
    cfg = synth.config_small("head", cells=12, subdiv=3)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    a = _mesh(ctx, cfg)
    b = _mesh(ctx, cfg)
    a.refine_relabel(ss, 0)
    b.refine_relabel(ss, 0)
    rng = np.random.default_rng(3)
    pts = torch.from_numpy(synth.uniform_box(rng, 20000, -100, 100)).to("cuda:0")
    want_pts = oracle.label(pts.cpu().numpy(), cfg.surfaces)
    kinds = []
    for call in range(3):
        sa = a.refine_relabel(ss, 1)
        sb = b.refine_relabel(ss, 1, use_graph=True)
        kinds.append(sb[1]["graph"])
        ka, la = export_np(a)
        kb, lb = export_np(b)
        assert np.array_equal(ka, kb) and np.array_equal(la, lb), call
        for f in ("n_leaves", "n_boundary", "n_labeled", "n_pairs"):
            assert sa[1][f] == sb[1][f], (call, f)
        lab, _, _ = sal.label_points(ctx, ss, pts)          # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(lab.cpu().numpy(), want_pts)
    assert kinds == [1, 2, 2]


def test_graph_round_that_does_not_fit_runs_host_driven(ctx, monkeypatch):
    """Children reserved for round 1's count only (scratch capacity below 2x
    that): round 2 has 5.7x as many children, so the device-side plan stops it
    before it changes the mesh; it runs host-driven and the result is
    unchanged."""
    cfg = synth.config_small("head", cells=12, subdiv=3)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    ref = _mesh(ctx, cfg)
    sr = ref.refine_relabel(ss, 2)
    k1, k2 = sr[1]["n_labeled"], sr[2]["n_labeled"]
    assert k2 > 2 * k1 + 1024
    monkeypatch.setenv("SAL_REFINE_GRAPH_BUDGET", str(k1))
    m = _mesh(ctx, cfg)
    st = m.refine_relabel(ss, 2, use_graph=True)
    assert st[1]["graph"] in (1, 2) and st[2]["graph"] == 0
    k0, l0 = export_np(ref)
    k1, l1 = export_np(m)
    assert np.array_equal(k0, k1) and np.array_equal(l0, l1)
    for r in (1, 2):
        assert st[r]["n_leaves"] == sr[r]["n_leaves"]


def test_graph_rounds_respect_the_depth_limit(ctx):
    cfg = synth.config_small("sphere", cells=8, subdiv=2)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    a = _mesh(ctx, cfg)
    b = _mesh(ctx, cfg)
    a.refine_relabel(ss, 3)
    st = b.refine_relabel(ss, 3, use_graph=True)
    assert all(s["graph"] in (1, 2) for s in st[1:])
    ka, la = export_np(a)
    kb, lb = export_np(b)
    assert np.array_equal(ka, kb) and np.array_equal(la, lb)
    with pytest.raises(sal.SalError) as e:
        b.refine_relabel(ss, 1, use_graph=True)
    assert e.value.status == 6
