"""Taubin smoothing of a conforming tetrahedral mesh -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper section 2.2.1 (smoothing), parameters in section 2.6.1 (lambda = mu = 0.4,
xi = 0.9 for the volume and 0.1 for the tissue boundaries).  The printed
update sums neighbour positions, which cannot be meant (it is not invariant
under translation); read as Taubin's method with the umbrella operator over
the index set N_i that holds node i and its neighbours:

    m_i(x)      = mean of x_j over j in N_i           (i itself included)
    x^(k+1/2)_i = x^(k)_i     + lambda (m_i(x^(k))     - x^(k)_i)
    x^(k+1)_i   = x^(k+1/2)_i - mu     (m_i(x^(k+1/2)) - x^(k+1/2)_i)

a forward (shrinking) step and a backward (inflating) one.  An iteration is
both half steps; after iteration k the phase stops when
||x^(k+1/2) - x^(k)||_2 / ||x^(0)||_2 <= xi (norms over the nodes the phase
moves, x^(0) their positions when the phase starts) or after max_iter
iterations.

Two phases, tissue boundaries first:
* surface: the nodes on an interface (an edge of the node joins tetrahedra
  of two or more labels), neighbours along interface edges only;
* volume: every other node, neighbours along all edges; interface nodes are
  held where the surface phase left them.
Nodes on the faces of the lattice box never move.

Written in float64 with scipy.sparse products, in the order of the
definitions above.
"""
import numpy as np
import scipy.sparse as sp

TET_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def edges(tets, labels):
    """Undirected edges of the mesh: [E, 2] node ids (a < b, ascending), and
    per edge whether the tetrahedra around it carry two or more labels."""
    tets = np.asarray(tets, dtype=np.int64)
    labels = np.asarray(labels, dtype=np.int64)
    e = np.concatenate([tets[:, [a, b]] for a, b in TET_EDGES])
    e = np.sort(e, axis=1)
    lab = np.tile(labels, len(TET_EDGES))
    uniq, inv = np.unique(e, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    lo = np.full(len(uniq), np.iinfo(np.int64).max)
    hi = np.full(len(uniq), np.iinfo(np.int64).min)
    np.minimum.at(lo, inv, lab)
    np.maximum.at(hi, inv, lab)
    return uniq, lo != hi


def adjacency(n, edge_list):
    """Symmetric 0/1 adjacency [n, n] of the given edges."""
    a, b = edge_list[:, 0], edge_list[:, 1]
    data = np.ones(2 * len(a))
    return sp.csr_matrix((data, (np.concatenate([a, b]), np.concatenate([b, a]))), shape=(n, n))


def umbrella_mean(x, adj):
    """m_i: mean of x over node i and its neighbours."""
    deg = np.asarray(adj.sum(axis=1)).reshape(-1)
    return (adj @ x + x) / (deg + 1.0)[:, None]


def taubin(x, adj, movable, lam, mu, xi, max_iter):
    """Runs the iterations on the nodes where `movable` is set.  Returns
    (positions, iterations run, ratio of each iteration)."""
    x = np.array(x, dtype=np.float64)
    mv = np.asarray(movable, dtype=bool)
    if not mv.any():
        return x, 0, []          # nothing to smooth: the phase runs no iteration
    norm0 = np.linalg.norm(x[mv])
    ratios = []
    for _ in range(max_iter):
        half = x.copy()
        half[mv] = x[mv] + lam * (umbrella_mean(x, adj)[mv] - x[mv])
        step = np.linalg.norm(half[mv] - x[mv])
        new = half.copy()
        new[mv] = half[mv] - mu * (umbrella_mean(half, adj)[mv] - half[mv])
        x = new
        ratios.append(step / norm0 if norm0 > 0 else 0.0)
        if ratios[-1] <= xi:
            break
    return x, len(ratios), ratios


def on_box(node_keys, cells, fine=8):
    """Nodes on a face of the lattice box (node keys on the finest grid)."""
    k = np.asarray(node_keys, dtype=np.int64)
    m = (1 << 21) - 1
    f = np.stack([(k >> 42) & m, (k >> 21) & m, k & m], -1)
    lim = np.asarray(cells, dtype=np.int64) * fine
    return np.any((f == 0) | (f == lim), axis=1)


def smooth_mesh(tets, labels, xyz, fixed, lam=0.4, mu=0.4, xi_surface=0.1, xi_volume=0.9,
                max_iter_surface=100, max_iter_volume=100):
    """Both phases.  tets [m, 4] node ids, labels [m], xyz [n, 3], fixed [n]
    (nodes that never move).  Returns (xyz, info)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    n = len(xyz)
    e, surf = edges(tets, labels)
    interface = np.zeros(n, dtype=bool)
    interface[e[surf].reshape(-1)] = True
    fixed = np.asarray(fixed, dtype=bool)
    s_mv = interface & ~fixed
    v_mv = ~interface & ~fixed
    x, it_s, r_s = taubin(xyz, adjacency(n, e[surf]), s_mv, lam, mu, xi_surface,
                          max_iter_surface)
    x, it_v, r_v = taubin(x, adjacency(n, e), v_mv, lam, mu, xi_volume, max_iter_volume)
    info = {"n_edges": len(e), "n_surface_edges": int(surf.sum()),
            "n_surface_nodes": int(s_mv.sum()), "n_volume_nodes": int(v_mv.sum()),
            "iters_surface": it_s, "iters_volume": it_v,
            "ratios_surface": r_s, "ratios_volume": r_v}
    return x, info
