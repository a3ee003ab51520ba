"""Parity at the full workload sizes (the benchmark's launch configurations),
on outputs the FP64 oracle can compute one by one: a uniform sample plus a
sample near the surfaces, where labels are hardest."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2203_10000_amd as sal  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sal.Context(0)


def _sample(rng, n_all, n, near_mask=None):
    idx = rng.choice(n_all, min(n, n_all), replace=False)
    if near_mask is not None and near_mask.any():
        near = np.nonzero(near_mask)[0]
        idx = np.concatenate([idx, rng.choice(near, min(n, len(near)), replace=False)])
    return np.unique(idx)


def test_c3_full_size_two_rounds(ctx):
    """20 compartments (409,600 triangles), 48M-centroid lattice, two
    refine-and-relabel rounds (1.06e8 leaves)."""
    cfg = synth.config_c3()
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    st = mesh.refine_relabel(ss, cfg.rounds, precision="fp32")
    n_leaves, level = mesh.size()
    assert level == 2
    assert n_leaves == lat.n_points + 7 * sum(r["n_boundary"] for r in st)
    assert all(r["n_boundary"] > 0 for r in st[1:])
    e = mesh.export(keys=False, labels=True, centroids=True)
    torch.cuda.synchronize()
    lab = e["labels"].cpu().numpy()
    cen = e["centroids"].cpu().numpy()
    del e
    assert np.all(lab >= 0)
    rng = np.random.default_rng(301)
    r = np.linalg.norm(cen.astype(np.float64), axis=0)
    near = np.min(np.abs(r[:, None] - np.array([92, 86, 80, 76.0])), axis=1) < 3.0
    idx = _sample(rng, len(lab), 2500, near)
    want = oracle.label(np.ascontiguousarray(cen[:, idx]), cfg.surfaces)
    assert np.array_equal(lab[idx], want)


def test_c4_full_size_batched(ctx):
    """64 instances: batched persistent launch (eager and hipGraph) equals the
    per-instance launches; a sample of every fourth instance against the oracle."""
    insts = synth.config_c4()
    dev = []
    for surfs, pts in insts:
        ss = sal.SurfaceSet(ctx, surfs)
        p = torch.from_numpy(pts).to("cuda:0")
        dev.append((ss, p, torch.empty(pts.shape[1], dtype=torch.int32, device="cuda:0")))
    per = []
    for ss, p, _ in dev:
        lab, _, _ = sal.label_points(ctx, ss, p)
        per.append(lab)
    sal.label_batch(ctx, dev)
    torch.cuda.synchronize()
    assert all(torch.equal(a, l) for a, (_, _, l) in zip(per, dev))
    for _ in range(2):
        for _, _, l in dev:
            l.fill_(-7)
        sal.label_batch(ctx, dev, use_graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(a, l) for a, (_, _, l) in zip(per, dev))
    rng = np.random.default_rng(401)
    for (surfs, pts), a in list(zip(insts, per))[::4]:
        idx = _sample(rng, pts.shape[1], 300)
        want = oracle.label(np.ascontiguousarray(pts[:, idx]), surfs)
        assert np.array_equal(a.cpu().numpy()[idx], want)


def test_c5_surfaces_near_surface_points(ctx):
    """The eight 297,680-triangle compartments with 2M points offset up to
    0.5 mm along face normals: labels against the oracle, and the recheck is
    driven by the conditioning flags alone."""
    cfg = synth.config_c5(n_near=2_000_000, with_lattice=False)
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    pts = torch.from_numpy(cfg.points).to("cuda:0")
    lab, _, st = sal.label_points(ctx, ss, pts, stats=True)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    assert st["n_recheck_points"] > 0 and st["n_band_flags"] == 0
    assert st["n_recheck_points"] < 0.05 * len(lab)
    rng = np.random.default_rng(501)
    idx = _sample(rng, len(lab), 1200)
    want = oracle.label(np.ascontiguousarray(cfg.points[:, idx]), cfg.surfaces)
    assert np.array_equal(lab[idx], want)
