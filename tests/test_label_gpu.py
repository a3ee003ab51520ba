"""Parity of sal_label_points (HIP, through the C ABI) with the FP64 oracle.

Bar: labels bit-exact; winding numbers within 1e-5 absolute of the oracle's
(the float32 form) or 1e-12 (the plain FP64 form).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2203_10000_amd as sal  # noqa: E402

pytestmark = pytest.mark.gpu

W_TOL_F32 = 1e-5
W_TOL_F64 = 1e-12


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sal.Context(0)


def dev(pts):
    return torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).to("cuda:0")


def run(ctx, surfaces, pts, **kw):
    ss = sal.SurfaceSet(ctx, surfaces)
    lab, w, st = sal.label_points(ctx, ss, dev(pts), stats=True, **kw)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), (w.cpu().numpy().astype(np.float64) if w is not None else None), st


def mixed_points(cfg, n_uniform, n_near, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([synth.uniform_box(rng, n_uniform, -100, 100),
                           synth.near_surface_points(rng, cfg.surfaces, n_near, 0.5)], 1)


@pytest.fixture(scope="module")
def head_small():
    cfg = synth.config_small("head", subdiv=3)
    pts = mixed_points(cfg, 30000, 12000, 11)
    lab, w = oracle.label(pts, cfg.surfaces, want_w=True)
    return cfg, pts, lab, w


def test_plain_fp64_parity_one_sphere(ctx):
    cfg = synth.config_c1()
    pts = mixed_points(cfg, 20000, 8000, 1)
    want, w_ref = oracle.label(pts, cfg.surfaces, want_w=True)
    got, w, st = run(ctx, cfg.surfaces, pts, precision="fp64", winding="f64")
    assert np.array_equal(got, want)
    assert np.max(np.abs(w - w_ref)) < W_TOL_F64


def test_fp32_recheck_parity_head(ctx, head_small):
    cfg, pts, want, w_ref = head_small
    got, w, st = run(ctx, cfg.surfaces, pts, precision="fp32", winding="f64")
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:10]
    assert np.max(np.abs(w - w_ref)) < W_TOL_F32
    assert st["n_recheck_pairs"] > 0          # near-surface points were rechecked
    assert st["n_recheck_pairs"] < 0.2 * pts.shape[1]


def test_fp64_form_parity_head(ctx, head_small):
    cfg, pts, want, w_ref = head_small
    got, w, _ = run(ctx, cfg.surfaces, pts, precision="fp64", winding="f64")
    assert np.array_equal(got, want)
    assert np.max(np.abs(w - w_ref)) < W_TOL_F64


def test_precision_ladder(ctx):
    """Points at +-1e-9 .. 1e-3 mm from face interiors, edge midpoints and
    vertices: every label exact, and the float32 conditioning flag fires."""
    cfg = synth.config_small("shells", subdiv=4)
    rng = np.random.default_rng(5)
    pts = np.concatenate([synth.precision_ladder(s, rng, n_sites=24) for s in cfg.surfaces], 1)
    want, w_ref = oracle.label(pts, cfg.surfaces, want_w=True)
    got, w, st = run(ctx, cfg.surfaces, pts, precision="fp32", winding="f64")
    assert np.array_equal(got, want)
    assert np.max(np.abs(w - w_ref)) < W_TOL_F32
    assert st["n_cond_flags"] > 0


def test_points_on_the_surface_are_inside(ctx):
    cfg = synth.config_small("sphere", subdiv=3)
    s = cfg.surfaces[0]
    on = synth.face_centroids_on_surface(s)
    for prec in ("fp32", "fp64"):
        got, _, st = run(ctx, [s], on, precision=prec)
        assert np.all(got == s.label), prec
        assert st["n_exact_fallbacks"] > 0


def test_non_finite_points_get_minus_one(ctx):
    cfg = synth.config_small("sphere", subdiv=2)
    pts = np.array([[0, 0, 0], [np.nan, 0, 0], [0, np.inf, 0], [200, 0, 0], [0, 0, -np.inf]],
                   np.float32).T
    for prec in ("fp32", "fp64"):
        got, _, _ = run(ctx, cfg.surfaces, pts, precision=prec)
        assert list(got) == [1, -1, -1, 0, -1]


@pytest.mark.parametrize("n", [0, 1, 63, 65, 257, 1031])
def test_empty_and_ragged_sizes(ctx, head_small, n):
    cfg, pts, want, _ = head_small
    sub = np.ascontiguousarray(pts[:, :n])
    got, _, st = run(ctx, cfg.surfaces, sub, precision="fp32")
    assert got.shape == (n,) and np.array_equal(got, want[:n])


def test_every_tile_config_gives_the_same_labels(ctx, head_small):
    cfg, pts, want, w_ref = head_small
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    d = dev(pts)
    for ppl in (1, 2, 4):
        for bw in (1, 2, 4, 8):
            lab, w, _ = sal.label_points(ctx, ss, d, precision="fp32", winding="f64",
                                         points_per_lane=ppl, block_waves=bw)
            torch.cuda.synchronize()
            assert np.array_equal(lab.cpu().numpy(), want), (ppl, bw)
            assert np.max(np.abs(w.cpu().numpy() - w_ref)) < W_TOL_F32, (ppl, bw)


def test_runs_are_bit_identical(ctx, head_small):
    cfg, pts, _, _ = head_small
    a = run(ctx, cfg.surfaces, pts, precision="fp32", winding="f64")
    b = run(ctx, cfg.surfaces, pts, precision="fp32", winding="f64")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_band_recheck_path(ctx, head_small):
    """T = 0.9995 puts every enclosed pair inside the 1e-3 band, so the band
    path carries the labels through the FP64 recheck."""
    cfg, pts, _, _ = head_small
    sub = np.ascontiguousarray(pts[:, :6000])
    want = oracle.label(sub, cfg.surfaces, threshold=0.9995)
    got, _, st = run(ctx, cfg.surfaces, sub, precision="fp32", threshold=0.9995)
    assert np.array_equal(got, want)
    assert st["n_band_flags"] > 0


def test_winding_f32_output(ctx, head_small):
    cfg, pts, _, w_ref = head_small
    _, w, _ = run(ctx, cfg.surfaces, pts, precision="fp32", winding="f32")
    assert np.max(np.abs(w - w_ref)) < 2e-5


def test_tuner_picks_a_shape_and_caches_it(ctx, head_small, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SAL_TUNE_CACHE", str(cache))
    cfg, pts, want, _ = head_small
    sub = np.ascontiguousarray(pts[:, :3000])          # a point-count bucket no other test uses
    for prec in ("fp32", "fp64"):
        got, _, st = run(ctx, cfg.surfaces, sub, precision=prec)
        assert np.array_equal(got, want[:3000])
        assert st["points_per_lane"] in (1, 2, 4) and st["block_waves"] in (1, 2, 4, 8)
        got2, _, st2 = run(ctx, cfg.surfaces, sub, precision=prec)
        assert np.array_equal(got2, got)
        assert (st2["points_per_lane"], st2["block_waves"]) == (st["points_per_lane"], st["block_waves"])
    assert cache.exists() and len(cache.read_text().splitlines()) >= 2


# ---------------------------------------------------------------- validation
def _sphere(subdiv=2, r=50.0):
    v, f = synth.icosphere(subdiv)
    return (v * r).astype(np.float32), f.astype(np.int32)


def _status(ctx, surfaces, **kw):
    try:
        sal.SurfaceSet(ctx, surfaces, **kw)
        return 0
    except sal.SalError as e:
        return e.status


def test_surface_validation(ctx):
    v, f = _sphere()
    assert _status(ctx, [(v, f, 1)]) == 0
    assert _status(ctx, [(v, f[1:], 1)]) == 2                     # open
    rev = f[:, [0, 2, 1]].copy()
    assert _status(ctx, [(v, rev, 1)]) == 3                       # inward
    assert _status(ctx, [(v, rev, 1)], auto_orient=True) == 0
    bad = v.copy()
    bad[3, 1] = np.nan
    assert _status(ctx, [(bad, f, 1)]) == 1                       # NaN vertex
    ff = f.copy()
    ff[0, 0] = len(v) + 5
    assert _status(ctx, [(v, ff, 1)]) == 1                        # index out of range
    assert _status(ctx, [(v, f, 0)]) == 1                         # label must be > 0
    assert _status(ctx, [(v, f, 1)] * 65) == 1                    # too many surfaces


def test_auto_orient_gives_the_same_labels(ctx):
    v, f = _sphere(3)
    rng = np.random.default_rng(4)
    pts = synth.uniform_box(rng, 5000, -60, 60)
    ss1 = sal.SurfaceSet(ctx, [(v, f, 2)])
    ss2 = sal.SurfaceSet(ctx, [(v, f[:, [0, 2, 1]].copy(), 2)], auto_orient=True)
    a, _, _ = sal.label_points(ctx, ss1, dev(pts))
    b, _, _ = sal.label_points(ctx, ss2, dev(pts))
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bounding_box_culling_keeps_the_labels(ctx, precision):
    """cull_bounds skips a surface for wavefronts whose points all lie
    strictly outside its vertices' box (outside the convex hull, w = 0
    exactly) or inside a ball the surface does not cross (w = 1 or 0 exactly):
    labels still equal the oracle's, windings stay within the bar, and the
    skipped pairs are counted."""
    from oracle import kuhn
    cfg = synth.config_small("head", cells=24, subdiv=3)
    lat = cfg.lattice
    pts = kuhn.centroids_mm(kuhn.level0_keys(lat.cells), lat.origin, lat.h)
    want, w_ref = oracle.label(pts, cfg.surfaces, want_w=True)
    tol = W_TOL_F32 if precision == "fp32" else W_TOL_F64
    plain, w0, st0 = run(ctx, cfg.surfaces, pts, precision=precision, winding="f64")
    got, w, st = run(ctx, cfg.surfaces, pts, precision=precision, winding="f64", cull=True)
    assert np.array_equal(plain, want) and np.array_equal(got, want)
    assert np.max(np.abs(w - w_ref)) < tol
    assert st0["n_pairs_culled"] == 0
    assert 0.1 * st["n_pairs"] < st["n_pairs_culled"] < st["n_pairs"]
    # skipped pairs report exactly 0 or 1; the rest are the same computation
    same = (w != 0.0) & (w != 1.0)
    assert np.array_equal(w[same], w0[same])
    assert np.sum(w == 0.0) > 0 and np.sum(w == 1.0) > 0


def test_culling_in_refine_relabel_gives_the_same_mesh(ctx):
    cfg = synth.config_small("head", cells=12, subdiv=3)
    lat = cfg.lattice
    ss = sal.SurfaceSet(ctx, cfg.surfaces)
    out = []
    for cull in (False, True):
        for rule in ("centroid", "four_nodes"):
            mesh = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
            mesh.refine_relabel(ss, 2, rule=rule, cull=cull)
            e = mesh.export(keys=True, labels=True, centroids=False)
            torch.cuda.synchronize()
            out.append((e["keys"].cpu().numpy(), e["labels"].cpu().numpy()))
    for a, b in ((0, 2), (1, 3)):
        assert np.array_equal(out[a][0], out[b][0]) and np.array_equal(out[a][1], out[b][1])
