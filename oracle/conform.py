"""Conforming transition refinement of a red-refined Kuhn leaf set -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper section 2.1.2 (Fig. 2): inside the refined region every element is
split into eight; an element outside it whose face toward the region has
one, two or three of its edges subdivided is split into two, three or four
tetrahedra.  Read on a leaf set from red refinement (levels may differ
across a face):

* a *hanging* edge of a leaf is one whose midpoint is a vertex of another
  leaf; an edge with a node at a quarter point sits next to a leaf two or
  more levels finer;
* the subdivision patterns of the paper are: one hanging edge (the leaf is
  bisected through its midpoint), two hanging edges of one face (three
  tetrahedra: the corner at their common vertex and the remaining
  quadrilateral cut along the diagonal through its smallest node key), or
  the three edges of one face (four tetrahedra over the midpoint split of
  that face);
* a leaf with any other hanging pattern, or with a quarter-point node, is
  split into its eight children (they keep its label) and the hanging edges
  are found again, until every leaf has an allowed pattern (closure);
* the output tetrahedra carry the label of the leaf they come from.

Nodes are integer points of the finest grid (kuhn.node_keys); tetrahedra are
returned as four node keys, positively oriented.
"""
import numpy as np

from . import kuhn

EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
FACES = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]


def _fine(v_units):
    return np.rint(np.asarray(v_units, dtype=np.float64) * kuhn._FINE).astype(np.int64)


def _key(f):
    return (f[..., 0] << 42) | (f[..., 1] << 21) | f[..., 2]


def unkey(keys):
    keys = np.asarray(keys, dtype=np.int64)
    m = (1 << 21) - 1
    return np.stack([(keys >> 42) & m, (keys >> 21) & m, keys & m], -1)


def hanging_pattern(keys, node_set):
    """Per leaf: bit e set when edge EDGES[e] has a node at its midpoint;
    `deep` when an edge has a node at a quarter point."""
    f = _fine(kuhn.vertices_units(keys))                # [n, 4, 3] on the finest grid
    bits = np.zeros(len(keys), dtype=np.int64)
    deep = np.zeros(len(keys), dtype=bool)
    for e, (i, j) in enumerate(EDGES):
        s = f[:, i] + f[:, j]
        mid_ok = np.all(s % 2 == 0, axis=1)
        mk = np.where(mid_ok, _key(s // 2), -1)
        bits |= (np.isin(mk, node_set) & mid_ok).astype(np.int64) << e
        for a, b in ((3, 1), (1, 3)):
            q = a * f[:, i] + b * f[:, j]
            q_ok = np.all(q % 4 == 0, axis=1)
            qk = np.where(q_ok, _key(q // 4), -1)
            deep |= np.isin(qk, node_set) & q_ok
    return bits, deep


def allowed(bits):
    """True for the patterns of Fig. 2c-e (and for no hanging edge)."""
    n = bin(int(bits)).count("1")
    if n <= 1:
        return True
    ed = [EDGES[e] for e in range(6) if bits >> e & 1]
    verts = set(v for e in ed for v in e)
    return (n == 2 and len(verts) == 3) or (n == 3 and len(verts) == 3)


def close(keys, labels, cells):
    """Splits leaves into their 8 children until every leaf's hanging edges
    form an allowed pattern.  Returns (keys, labels, bits, red_rounds)."""
    keys = np.asarray(keys, dtype=np.uint64)
    labels = np.asarray(labels, dtype=np.int32)
    rounds = 0
    while True:
        nodes = np.unique(_key(_fine(kuhn.vertices_units(keys)).reshape(-1, 3)))
        bits, deep = hanging_pattern(keys, nodes)
        red = deep | np.array([not allowed(b) for b in bits], dtype=bool)
        if not red.any():
            return keys, labels, bits, rounds
        rk = keys[red]
        lv = kuhn.decode(rk)[0]
        assert np.all(lv < kuhn.MAX_LEVEL), "closure beyond the deepest level"
        kids, klab = [], []
        for x in np.unique(lv):
            sel = lv == x
            c = kuhn.children(rk[sel], cells)
            kids.append(c.reshape(-1))
            klab.append(np.repeat(labels[red][sel], 8))
        keys = np.concatenate([keys[~red]] + kids)
        labels = np.concatenate([labels[~red]] + klab)
        rounds += 1


def _oriented(t):
    """t: [4, 3] integer points -> the same tetrahedron, positive volume."""
    d = np.linalg.det(np.array([t[1] - t[0], t[2] - t[0], t[3] - t[0]], dtype=np.float64))
    assert d != 0, "degenerate tetrahedron"
    return t if d > 0 else t[[1, 0, 2, 3]]


def quad_diagonal(kq, d_key):
    """The diagonal that cuts the quadrilateral (m1, b, c, m2) of a two-edge
    split: the one through its smallest node key, a choice made by the face
    alone so that both tetrahedra sharing it agree (d_key, the fourth vertex
    of the tetrahedron, is not used)."""
    low = min(kq, key=kq.get)
    return "m1-c" if low in ("m1", "c") else "b-m2"


def emit(keys, labels, bits):
    """The conforming tetrahedra: [m, 4] node keys and [m] labels."""
    f = _fine(kuhn.vertices_units(keys))
    out, lab = [], []
    for n in range(len(keys)):
        v = f[n]
        b = int(bits[n])
        ed = [EDGES[e] for e in range(6) if b >> e & 1]
        tets = []
        if not ed:
            tets.append(v)
        elif len(ed) == 1:
            i, j = ed[0]
            m = (v[i] + v[j]) // 2
            o = [x for x in range(4) if x not in (i, j)]
            tets += [np.array([v[i], m, v[o[0]], v[o[1]]]), np.array([m, v[j], v[o[0]], v[o[1]]])]
        elif len(ed) == 2:
            a = (set(ed[0]) & set(ed[1])).pop()
            b1 = ed[0][0] + ed[0][1] - a
            c1 = ed[1][0] + ed[1][1] - a
            d = ({0, 1, 2, 3} - {a, b1, c1}).pop()
            m1 = (v[a] + v[b1]) // 2
            m2 = (v[a] + v[c1]) // 2
            tets.append(np.array([v[a], m1, m2, v[d]]))
            quad = {"m1": m1, "b": v[b1], "c": v[c1], "m2": m2}
            kq = {k: int(_key(p)) for k, p in quad.items()}
            if quad_diagonal(kq, int(_key(v[d]))) == "m1-c":
                tets += [np.array([m1, v[b1], v[c1], v[d]]), np.array([m1, v[c1], m2, v[d]])]
            else:                            # diagonal b - m2
                tets += [np.array([m1, v[b1], m2, v[d]]), np.array([v[b1], v[c1], m2, v[d]])]
        else:
            fa = sorted(set(x for e in ed for x in e))
            d = ({0, 1, 2, 3} - set(fa)).pop()
            a, b_, c = fa
            mab, mbc, mca = (v[a] + v[b_]) // 2, (v[b_] + v[c]) // 2, (v[c] + v[a]) // 2
            tets += [np.array([v[a], mab, mca, v[d]]), np.array([mab, v[b_], mbc, v[d]]),
                     np.array([mca, mbc, v[c], v[d]]), np.array([mab, mbc, mca, v[d]])]
        for t in tets:
            out.append(_key(_oriented(t)))
            lab.append(labels[n])
    return np.array(out, dtype=np.int64).reshape(-1, 4), np.array(lab, dtype=np.int32)


def conforming_mesh(keys, labels, cells):
    """close() then emit(): (tets [m, 4] node keys, labels [m], red rounds)."""
    k, l, bits, rounds = close(keys, labels, cells)
    tets, lab = emit(k, l, bits)
    return tets, lab, rounds


def faces_shared_once(tets, cells):
    """Conformity check: every triangular face is shared by exactly two
    tetrahedra, or by one when it lies on the domain boundary.  Returns the
    number of faces that break this."""
    f = np.sort(np.concatenate([tets[:, list(fc)] for fc in FACES]), axis=1)
    uniq, counts = np.unique(f, axis=0, return_counts=True)
    pts = unkey(uniq)                                   # [F, 3, 3]
    lim = np.asarray(cells, dtype=np.int64) * kuhn._FINE
    on_box = np.zeros(len(uniq), dtype=bool)
    for a in range(3):
        on_box |= np.all(pts[:, :, a] == 0, axis=1) | np.all(pts[:, :, a] == lim[a], axis=1)
    bad = (counts > 2) | ((counts == 1) & ~on_box) | ((counts == 2) & on_box)
    return int(bad.sum())


def volumes6(tets):
    """Six times the volume of each tetrahedron, exactly, in finest-grid units."""
    p = unkey(tets).astype(np.int64)                    # [m, 4, 3]
    a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    return (a[:, 0] * (b[:, 1] * c[:, 2] - b[:, 2] * c[:, 1])
            - a[:, 1] * (b[:, 0] * c[:, 2] - b[:, 2] * c[:, 0])
            + a[:, 2] * (b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0]))
