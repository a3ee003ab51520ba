"""Generators: closed, outward, star-shaped surfaces; seeded determinism;
the sizes the workloads state."""
import numpy as np

import synth
from synth.meshes import star_shaped_about


def test_icosphere_and_geodesic_counts():
    for s in range(5):
        v, f = synth.icosphere(s)
        assert f.shape[0] == 20 * 4 ** s and v.shape[0] == 10 * 4 ** s + 2
        assert synth.check_closed_oriented(f) and synth.signed_volume(v, f) > 0
    for nu in (1, 2, 5, 9):
        v, f = synth.geodesic_sphere(nu)
        assert f.shape[0] == 20 * nu * nu and v.shape[0] == 10 * nu * nu + 2
        assert synth.check_closed_oriented(f) and synth.signed_volume(v, f) > 0


def test_c1_c2_shapes():
    c1 = synth.config_c1()
    assert c1.n_tri == 1280 and c1.lattice.n_points == 196608
    c2 = synth.config_c2()
    assert [s.n_tri for s in c2.surfaces] == [20480] * 4 and c2.lattice.n_points == 6_000_000
    assert [s.label for s in c2.surfaces] == [1, 2, 3, 4]


def test_shell_perturbation_is_five_percent():
    c2 = synth.config_c2()
    for s, r in zip(c2.surfaces, (92, 86, 80, 76)):
        rad = np.linalg.norm(s.v.astype(np.float64), axis=1)
        assert abs(np.max(np.abs(rad - r)) - 0.05 * r) < 1e-4
        assert s.v.dtype == np.float32 and s.f.dtype == np.int32
        assert star_shaped_about(s.v.astype(np.float64), s.f, s.center) > 0


def test_seeded_determinism():
    a = synth.c4_instance(3)
    b = synth.c4_instance(3)
    assert np.array_equal(a[1], b[1])
    assert all(np.array_equal(x.v, y.v) for x, y in zip(a[0], b[0]))


def test_near_surface_offsets():
    cfg = synth.config_small("sphere", subdiv=3)
    rng = np.random.default_rng(0)
    p = synth.near_surface_points(rng, cfg.surfaces, 2000, 0.5).astype(np.float64)
    r = np.linalg.norm(p, axis=0)
    assert np.all(np.abs(r - 80.0) < 0.5 + 0.8)   # offset + sagitta of subdiv 3
