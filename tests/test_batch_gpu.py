"""Batched persistent labeling (sal_label_batch) against per-instance calls and
the oracle; hipGraph capture and replay."""
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


def small_instances(n_inst=6, seed=0):
    """c4-like instances at test scale: 1-4 surfaces of 180-3,380 triangles,
    100-6,000 uniform points (one empty instance)."""
    out = []
    for i in range(n_inst):
        surfs, _ = synth.c4_instance(i, t_lo=180, t_hi=3500)
        surfs = surfs[:4]
        for k, s in enumerate(surfs):
            s.label = k + 1
        rng = np.random.default_rng(seed + i)
        n = 0 if i == 2 else int(rng.integers(100, 6000))
        out.append((surfs, synth.uniform_box(rng, n, -100, 100)))
    return out


def build(ctx, insts):
    dev = []
    for surfs, pts in insts:
        ss = sal.SurfaceSet(ctx, surfs)
        p = torch.from_numpy(np.ascontiguousarray(pts)).to("cuda:0")
        lab = torch.full((pts.shape[1],), -7, dtype=torch.int32, device="cuda:0")
        dev.append((ss, p, lab))
    return dev


def test_batch_equals_per_instance_and_oracle(ctx):
    insts = small_instances()
    dev = build(ctx, insts)
    st = sal.label_batch(ctx, dev, stats=True)
    torch.cuda.synchronize()
    for (surfs, pts), (ss, p, lab), s in zip(insts, dev, st):
        got = lab.cpu().numpy()
        single, _, _ = sal.label_points(ctx, ss, p)
        assert np.array_equal(got, single.cpu().numpy())
        assert np.array_equal(got, oracle.label(pts, surfs))
        assert s["n_points"] == pts.shape[1]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_splits_large_surfaces(ctx, precision):
    """Few points, large surfaces: the work list cuts surfaces into strip
    ranges whose partial sums are reduced in order."""
    cfg = synth.config_small("shells", subdiv=5)
    rng = np.random.default_rng(3)
    pts = np.concatenate([synth.uniform_box(rng, 200, -100, 100),
                          synth.near_surface_points(rng, cfg.surfaces, 200, 0.5)], 1)
    dev = build(ctx, [(cfg.surfaces, pts)])
    sal.label_batch(ctx, dev, precision=precision)
    torch.cuda.synchronize()
    assert np.array_equal(dev[0][2].cpu().numpy(), oracle.label(pts, cfg.surfaces))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_graph_replays(ctx, precision):
    insts = small_instances(4, seed=10)
    dev = build(ctx, insts)
    sal.label_batch(ctx, dev, use_graph=True, precision=precision)   # capture + launch
    torch.cuda.synchronize()
    first = [lab.clone() for _, _, lab in dev]
    for rep in range(3):
        # eager work on the same stream between replays
        for _, p, lab in dev:
            lab.fill_(-9)
        x = torch.randn(1000, device="cuda:0").sum()
        sal.label_batch(ctx, dev, use_graph=True, precision=precision)   # replay
        torch.cuda.synchronize()
        for f, (_, _, lab) in zip(first, dev):
            assert torch.equal(f, lab), rep
        del x
    # new coordinates in the same buffers: the replay sees them
    rng = np.random.default_rng(99)
    new = []
    for (surfs, pts), (ss, p, lab) in zip(insts, dev):
        q = synth.uniform_box(rng, pts.shape[1], -100, 100)
        p.copy_(torch.from_numpy(q))
        new.append((surfs, q))
    sal.label_batch(ctx, dev, use_graph=True, precision=precision)
    torch.cuda.synchronize()
    for (surfs, q), (_, _, lab) in zip(new, dev):
        assert np.array_equal(lab.cpu().numpy(), oracle.label(q, surfs))


def test_batch_work_list_reuse_and_graph_invalidation(ctx):
    """Eager calls on the same batch reuse the device work list; an eager call
    on another batch rewrites it, so a graph captured earlier must be captured
    again (not replayed on the other batch's work list)."""
    ia, ib = small_instances(3, seed=30), small_instances(4, seed=40)
    da, db = build(ctx, ia), build(ctx, ib)

    def check(insts, dev):
        torch.cuda.synchronize()
        for (surfs, pts), (_, _, lab) in zip(insts, dev):
            assert np.array_equal(lab.cpu().numpy(), oracle.label(pts, surfs))

    def clear(dev):
        for _, _, lab in dev:
            lab.fill_(-7)

    for step, (insts, dev, graph) in enumerate([(ia, da, True), (ib, db, False), (ia, da, True),
                                                (ia, da, False), (ia, da, False), (ib, db, False),
                                                (ia, da, False), (ia, da, True)]):
        clear(dev)
        sal.label_batch(ctx, dev, use_graph=graph)
        check(insts, dev)


def test_batch_fp64_form(ctx):
    """The persistent FP64 kernel: labels equal the per-point FP64 form's and
    the oracle's, points exactly on a triangle count as enclosed, and the
    exact-sign evaluations are counted per instance."""
    insts = small_instances(3, seed=20)
    # instance 0 also gets points exactly on its surfaces (vertices and
    # exactly representable edge midpoints)
    surfs0, pts0 = insts[0]
    on = np.concatenate([synth.face_centroids_on_surface(s, 50) for s in surfs0], 1)
    insts[0] = (surfs0, np.concatenate([pts0, on], 1))
    dev = build(ctx, insts)
    st = sal.label_batch(ctx, dev, precision="fp64", stats=True)
    torch.cuda.synchronize()
    for (surfs, pts), (ss, p, lab), s in zip(insts, dev, st):
        got = lab.cpu().numpy()
        single, _, one = sal.label_points(ctx, ss, p, precision="fp64", stats=True)
        assert np.array_equal(got, single.cpu().numpy())
        assert np.array_equal(got, oracle.label(pts, surfs))
        assert s["n_exact_fallbacks"] == one["n_exact_fallbacks"]
        assert s["n_recheck_points"] == 0
    assert st[0]["n_exact_fallbacks"] > 0


def test_batch_rejects_winding_and_nulls(ctx):
    with pytest.raises(sal.SalError):
        sal.label_batch(ctx, build(ctx, small_instances(1)), winding="f32")
