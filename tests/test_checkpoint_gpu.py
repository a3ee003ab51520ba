"""Checkpoint / resume through sal_tet_mesh_export and sal_tet_mesh_import:
a refined mesh rebuilt from its exported leaves has the same leaves and
labels, refines on exactly as the original (and as the oracle), and leaf sets
that are not a nested refinement of the lattice are rejected."""
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


def _leaves(mesh):
    e = mesh.export(keys=True, labels=True, centroids=False)
    torch.cuda.synchronize()
    keys = e["keys"].cpu().numpy().view(np.uint64)
    labels = e["labels"].cpu().numpy()
    order = np.argsort(keys)
    return keys[order], labels[order]


def _dev(keys, labels):
    return (torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).to("cuda:0"),
            torch.from_numpy(np.ascontiguousarray(labels, dtype=np.int32)).to("cuda:0"))


def test_export_import_resume_equals_uninterrupted_run(ctx):
    cfg = synth.config_small("head", cells=12, subdiv=3)
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    a = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    a.refine_relabel(ss, 2)
    keys, labels = _leaves(a)
    rng = np.random.default_rng(81)
    perm = rng.permutation(len(keys))                        # any order is accepted
    b = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    b.import_leaves(*_dev(keys[perm], labels[perm]))
    assert b.size() == a.size()
    kb, lb = _leaves(b)
    assert np.array_equal(kb, keys) and np.array_equal(lb, labels)
    # one more round on each: identical, and equal to the oracle's three rounds
    a.refine_relabel(ss, 1)
    b.refine_relabel(ss, 1)
    ka, la = _leaves(a)
    kb, lb = _leaves(b)
    assert np.array_equal(ka, kb) and np.array_equal(la, lb)
    want, _ = kuhn.refine_relabel(lat, lambda p: oracle.label(p, cfg.surfaces), 3)
    assert np.array_equal(ka, want.keys) and np.array_equal(la, want.labels)
    # the converging recursion also continues from a checkpoint
    c = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    c.import_leaves(*_dev(keys, labels))
    _, conv = c.refine_converge(ss, 3)
    d = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    d.refine_relabel(ss, 2)
    _, conv_d = d.refine_converge(ss, 3)
    assert conv and conv_d
    kc, lc = _leaves(c)
    kd, ld = _leaves(d)
    assert np.array_equal(kc, kd) and np.array_equal(lc, ld)


def test_import_rejects_what_is_not_a_nested_refinement(ctx):
    cfg = synth.config_small("sphere", cells=6, subdiv=2)
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    a = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    a.refine_relabel(ss, 2)
    keys, labels = _leaves(a)
    lv = kuhn.decode(keys)[0]
    deep = int(np.nonzero(lv == 2)[0][0])
    l1 = keys[lv == 1]                                        # level-1 leaves
    cases = {
        "a leaf missing": (np.delete(keys, deep), np.delete(labels, deep)),
        "a key twice": (np.append(keys, keys[0]), np.append(labels, labels[0])),
        "outside the lattice": (np.append(keys[1:], kuhn.encode(np.array([0]), np.array([0]),
                                                                 np.array([lat.cells[0]]),
                                                                 np.array([0]), np.array([0]))),
                                labels),
        "a negative label": (keys, np.where(np.arange(len(labels)) == 3, -1, labels)),
    }
    if len(l1):
        # a level-1 leaf plus its own 8 children: both a leaf and refined
        kids = kuhn.children(l1[:1], lat.cells).reshape(-1)
        cases["leaf and refined"] = (np.concatenate([keys, kids]),
                                     np.concatenate([labels, np.zeros(8, np.int32)]))
    for name, (k, l) in cases.items():
        m = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
        with pytest.raises(sal.SalError) as e:
            m.import_leaves(*_dev(k, l))
        assert e.value.status == 1, name
        assert m.size() == (lat.n_points, 0), name           # unchanged
        m.refine_relabel(ss, 0)                               # still usable
    # a labeled mesh cannot import
    with pytest.raises(sal.SalError):
        a.import_leaves(*_dev(keys, labels))
