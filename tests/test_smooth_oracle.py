"""Pins of the Taubin smoothing oracle (paper section 2.2.1): closed forms on
a ring, exact invariants on Kuhn lattices, interfaces found by brute force."""
import numpy as np
import pytest

import oracle
import synth
from oracle import conform, kuhn, smooth


def _ring(n):
    return np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)


def _ring_case(n=64, k=5, amp=3.0, offset=(10.0, -4.0, 2.5)):
    th = 2 * np.pi * k / n
    x = np.tile(np.asarray(offset, dtype=np.float64), (n, 1))
    wave = amp * np.cos(th * np.arange(n))
    x[:, 0] += wave
    sigma = (2 * np.cos(th) - 2) / 3            # eigenvalue of (mean over i, i-1, i+1) - identity
    return x, wave, sigma


@pytest.mark.parametrize("lam,mu", [(0.4, 0.4), (0.33, 0.34), (0.6, 0.2)])
def test_ring_wave_is_scaled_by_the_taubin_transfer_function(lam, mu):
    """One iteration multiplies a wave by (1 + lam s)(1 - mu s), two by its
    square; constants do not move."""
    x, wave, s = _ring_case()
    adj = smooth.adjacency(len(x), _ring(len(x)))
    g = (1 + lam * s) * (1 - mu * s)
    mv = np.ones(len(x), bool)
    for it in (1, 2):
        y, n_it, _ = smooth.taubin(x, adj, mv, lam, mu, -1.0, it)
        assert n_it == it
        np.testing.assert_allclose(y[:, 0], x[:, 0] - wave + g ** it * wave, rtol=0, atol=1e-12)
        np.testing.assert_allclose(y[:, 1:], x[:, 1:], rtol=0, atol=1e-12)


def test_ring_ratios_and_stopping_rule():
    """Ratio of iteration k: |lam s| g^k ||wave|| / ||x0||; the phase stops at
    the first ratio <= xi."""
    lam = mu = 0.4
    x, wave, s = _ring_case()
    adj = smooth.adjacency(len(x), _ring(len(x)))
    g = (1 + lam * s) * (1 - mu * s)
    want = [abs(lam * s) * g ** k * np.linalg.norm(wave) / np.linalg.norm(x) for k in range(30)]
    _, n_it, r = smooth.taubin(x, adj, np.ones(len(x), bool), lam, mu, -1.0, 30)
    np.testing.assert_allclose(r, want, rtol=1e-10)
    xi = 0.5 * (want[6] + want[7])               # between iterations 7 and 8
    _, n_it, r = smooth.taubin(x, adj, np.ones(len(x), bool), lam, mu, xi, 30)
    assert n_it == 8
    _, n_it, _ = smooth.taubin(x, adj, np.ones(len(x), bool), lam, mu, 10.0, 30)
    assert n_it == 1


def test_translation_moves_the_result_by_the_same_vector():
    """The printed update (a sum of neighbour positions) would fail this."""
    x, _, _ = _ring_case()
    adj = smooth.adjacency(len(x), _ring(len(x)))
    mv = np.ones(len(x), bool)
    mv[::7] = False
    y0, _, _ = smooth.taubin(x, adj, mv, 0.4, 0.4, -1.0, 3)
    t = np.array([5.0, -7.0, 11.0])
    y1, _, _ = smooth.taubin(x + t, adj, mv, 0.4, 0.4, -1.0, 3)
    np.testing.assert_allclose(y1, y0 + t, rtol=0, atol=1e-11)
    assert np.array_equal(y0[~mv], x[~mv])


def _mesh_ids(tets_keys):
    nodes, inv = np.unique(tets_keys.reshape(-1), return_inverse=True)
    return nodes, inv.reshape(-1, 4)


def _xyz(nodes, lat):
    return (np.asarray(lat.origin)[None, :]
            + (lat.h / kuhn._FINE) * conform.unkey(nodes).astype(np.float64))


def test_unrefined_kuhn_lattice_interior_does_not_move():
    """Every interior node of a Kuhn lattice has a centrally symmetric set of
    14 neighbours, so the mean over it is the node itself."""
    lat = synth.Lattice(origin=(-3.0, 1.0, 0.5), h=1.25, cells=(5, 4, 6))
    keys = kuhn.level0_keys(lat.cells)
    t, lab, _ = conform.conforming_mesh(keys, np.ones(len(keys), np.int32), lat.cells)
    nodes, ids = _mesh_ids(t)
    xyz = _xyz(nodes, lat)
    box = smooth.on_box(nodes, lat.cells)
    e, _ = smooth.edges(ids, lab)
    deg = np.bincount(e.reshape(-1), minlength=len(nodes))
    assert np.all(deg[~box] == 14)
    y, info = smooth.smooth_mesh(ids, lab, xyz, box)
    np.testing.assert_allclose(y, xyz, rtol=0, atol=1e-12)
    assert info["n_surface_nodes"] == 0 and info["iters_volume"] == 1
    assert info["iters_surface"] == 0


def test_interface_of_two_labels_split_by_a_lattice_plane():
    """Labels by the side of the plane x = 0: the interface nodes are exactly
    the nodes on that plane, the interface edges exactly the edges in it."""
    lat = synth.Lattice(origin=(-4.0, -3.0, -3.0), h=1.0, cells=(8, 6, 6))
    keys = kuhn.level0_keys(lat.cells)
    cen = kuhn.centroids_mm(keys, lat.origin, lat.h)
    lab = (cen[0] > 0).astype(np.int32)
    t, tl, _ = conform.conforming_mesh(keys, lab, lat.cells)
    nodes, ids = _mesh_ids(t)
    xyz = _xyz(nodes, lat)
    e, surf = smooth.edges(ids, tl)
    on_plane = xyz[:, 0] == 0.0
    assert np.array_equal(surf, on_plane[e[:, 0]] & on_plane[e[:, 1]])
    interface = np.zeros(len(nodes), bool)
    interface[e[surf].reshape(-1)] = True
    assert np.array_equal(interface, on_plane)


@pytest.fixture(scope="module")
def refined_case():
    cfg = synth.config_small("head", cells=8, subdiv=2)
    leaves, _ = kuhn.refine_relabel(cfg.lattice, lambda p: oracle.label(p, cfg.surfaces), 2)
    t, tl, _ = conform.conforming_mesh(leaves.keys, leaves.labels, cfg.lattice.cells)
    nodes, ids = _mesh_ids(t)
    return cfg, nodes, ids, tl, _xyz(nodes, cfg.lattice)


def test_phases_move_only_their_own_nodes(refined_case):
    cfg, nodes, ids, tl, xyz = refined_case
    box = smooth.on_box(nodes, cfg.lattice.cells)
    e, surf = smooth.edges(ids, tl)
    interface = np.zeros(len(nodes), bool)
    interface[e[surf].reshape(-1)] = True
    only_surface, info = smooth.smooth_mesh(ids, tl, xyz, box, max_iter_volume=0)
    moved = np.any(only_surface != xyz, axis=1)
    assert moved.any() and not np.any(moved & ~interface) and not np.any(moved & box)
    both, info = smooth.smooth_mesh(ids, tl, xyz, box)
    assert np.array_equal(both[interface], only_surface[interface])
    assert np.array_equal(both[box], xyz[box])
    assert info["iters_surface"] >= 1 and info["iters_volume"] >= 1
    # refinement makes interior neighbour sets asymmetric: some volume nodes move
    assert np.any(np.any(both != only_surface, axis=1) & ~interface)


def test_surface_phase_uses_interface_edges_only():
    """Jittered mesh, interface nodes kept on the plane x = 0: smoothing them
    along interface edges (all in the plane) keeps them there, while the
    off-plane jitter of their other neighbours would pull them off it."""
    lat = synth.Lattice(origin=(-4.0, -3.0, -3.0), h=1.0, cells=(8, 6, 6))
    keys = kuhn.level0_keys(lat.cells)
    cen = kuhn.centroids_mm(keys, lat.origin, lat.h)
    t, tl, _ = conform.conforming_mesh(keys, (cen[0] > 0).astype(np.int32), lat.cells)
    nodes, ids = _mesh_ids(t)
    xyz = _xyz(nodes, lat)
    on_plane = xyz[:, 0] == 0.0
    xyz = xyz + np.random.default_rng(3).uniform(-0.1, 0.1, xyz.shape)
    xyz[on_plane, 0] = 0.0
    box = smooth.on_box(nodes, lat.cells)
    y, info = smooth.smooth_mesh(ids, tl, xyz, box, max_iter_volume=0)
    mv = on_plane & ~box
    assert info["n_surface_nodes"] == mv.sum() > 0
    assert np.all(y[mv, 0] == 0.0)
    assert np.all(np.any(y[mv, 1:] != xyz[mv, 1:], axis=1))
