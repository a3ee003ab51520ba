"""Pins of the conforming transition refinement oracle (paper section 2.1.2,
Fig. 2): exact invariants that a mistake anywhere in it would break."""
import numpy as np
import pytest

import oracle
import synth
from oracle import conform, kuhn


def _refined(kind, cells, subdiv, rounds=2):
    cfg = synth.config_small(kind, cells=cells, subdiv=subdiv)
    leaves, _ = kuhn.refine_relabel(cfg.lattice, lambda p: oracle.label(p, cfg.surfaces), rounds)
    return cfg, leaves


@pytest.fixture(scope="module")
def head_case():
    cfg, leaves = _refined("head", 8, 2)
    keys, labels, bits, rounds = conform.close(leaves.keys, leaves.labels, cfg.lattice.cells)
    tets, lab = conform.emit(keys, labels, bits)
    return cfg, leaves, keys, labels, bits, rounds, tets, lab


def test_every_face_is_shared_by_two_tetrahedra_or_lies_on_the_box(head_case):
    cfg, *_, tets, _ = head_case
    assert conform.faces_shared_once(tets, cfg.lattice.cells) == 0


def test_volumes_are_positive_and_fill_the_box_exactly(head_case):
    cfg, *_, tets, _ = head_case
    v6 = conform.volumes6(tets)
    assert np.all(v6 > 0)
    assert v6.sum() == 6 * np.prod(np.array(cfg.lattice.cells, dtype=np.int64) * 8)


def test_no_node_lies_inside_an_edge(head_case):
    *_, tets, _ = head_case
    nodes = np.unique(tets.reshape(-1))
    p = conform.unkey(tets)                          # [m, 4, 3]
    for i, j in conform.EDGES:
        s = p[:, i] + p[:, j]
        ok = np.all(s % 2 == 0, axis=1)
        mk = conform._key(s[ok] // 2)
        assert not np.isin(mk, nodes).any()


def test_labels_are_those_of_the_leaf_holding_each_tetrahedron(head_case):
    cfg, _, keys, labels, _, _, tets, lab = head_case
    # an interior point of each tetrahedron off every lattice facet
    w = np.array([0.4123, 0.2871, 0.1994, 0.1012])
    cen = np.einsum("v,mva->ma", w, conform.unkey(tets).astype(np.float64)) / 8.0
    owner = kuhn.containing_leaf(kuhn.LeafSet(keys, labels), cen, cfg.lattice.cells,
                                 kuhn.MAX_LEVEL)
    assert np.all(owner >= 0)
    assert np.array_equal(kuhn.LeafSet(keys, labels).labels[owner], lab)


def test_closure_leaves_only_the_patterns_of_the_paper(head_case):
    *_, bits, rounds, _, _ = head_case
    counts = np.bincount([bin(int(b)).count("1") for b in bits], minlength=7)
    assert counts[4:].sum() == 0
    assert all(conform.allowed(b) for b in bits)
    assert counts[1] > 0 and counts[2] > 0 and counts[3] > 0   # all three splits occur
    assert rounds >= 1


def test_unrefined_lattice_is_returned_as_is():
    cfg = synth.config_small("sphere", cells=3, subdiv=1)
    keys = kuhn.level0_keys(cfg.lattice.cells)
    tets, lab, rounds = conform.conforming_mesh(keys, np.ones(len(keys), np.int32),
                                                cfg.lattice.cells)
    assert rounds == 0 and len(tets) == len(keys)
    want = np.sort(kuhn.node_keys(kuhn.vertices_units(keys)), axis=1)
    assert np.array_equal(np.sort(np.sort(tets, axis=1), axis=0), np.sort(want, axis=0))


@pytest.fixture(scope="module")
def random_case():
    """Leaves from splitting random leaves (not label boundaries) twice: every
    hanging pattern occurs many times, two-edge splits included."""
    cells = (4, 4, 4)
    rng = np.random.default_rng(77)
    keys = kuhn.level0_keys(cells)
    for _ in range(2):
        pick = rng.random(len(keys)) < 0.15
        lv = kuhn.decode(keys[pick])[0]
        kids = [kuhn.children(keys[pick][lv == x], cells).reshape(-1) for x in np.unique(lv)]
        keys = np.concatenate([keys[~pick]] + kids)
    labels = rng.integers(0, 4, len(keys)).astype(np.int32)
    k, l, bits, rounds = conform.close(keys, labels, cells)
    return cells, k, l, bits


def test_random_leaf_sets_close_to_a_conforming_mesh(random_case):
    cells, k, l, bits = random_case
    counts = np.bincount([bin(int(b)).count("1") for b in bits], minlength=4)
    assert counts[1] > 100 and counts[3] > 100
    tets, _ = conform.emit(k, l, bits)
    assert conform.faces_shared_once(tets, cells) == 0
    assert conform.volumes6(tets).sum() == 6 * np.prod(np.array(cells, dtype=np.int64) * 8)


def _diagonal_pair(rule, kq, d_key):
    """The chosen diagonal as a set of two node keys."""
    return frozenset((kq["m1"], kq["c"]) if rule(kq, d_key) == "m1-c" else (kq["b"], kq["m2"]))


def test_the_quadrilateral_diagonal_is_a_property_of_the_face():
    """Both tetrahedra sharing a two-edge face see it with b and c (and m1,
    m2) swapped and with different fourth vertices; they must cut it along
    the same two nodes."""
    rng = np.random.default_rng(5)
    for _ in range(500):
        k = rng.choice(1 << 40, 6, replace=False)
        one = {"m1": k[0], "b": k[1], "c": k[2], "m2": k[3]}
        other = {"m1": k[3], "b": k[2], "c": k[1], "m2": k[0]}
        assert _diagonal_pair(conform.quad_diagonal, one, k[4]) == \
            _diagonal_pair(conform.quad_diagonal, other, k[5])


def test_a_diagonal_chosen_per_tetrahedron_fails_the_face_property():
    """Planted mistake: a rule that looks at the tetrahedron (its fourth
    vertex) instead of the face alone disagrees across the face."""
    def mutant(kq, d_key):
        return "m1-c" if d_key % 2 else "b-m2"
    rng = np.random.default_rng(6)
    disagree = 0
    for _ in range(200):
        k = rng.choice(1 << 40, 6, replace=False)
        one = {"m1": k[0], "b": k[1], "c": k[2], "m2": k[3]}
        other = {"m1": k[3], "b": k[2], "c": k[1], "m2": k[0]}
        disagree += _diagonal_pair(mutant, one, k[4]) != _diagonal_pair(mutant, other, k[5])
    assert disagree > 0
