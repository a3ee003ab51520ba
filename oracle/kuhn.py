"""Kuhn tetrahedral lattice, red refinement and recursive relabeling -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper section 2.1.1 lays a regular hexahedral lattice over the domain and
splits every hexahedron into tetrahedra; the workloads use the six-tetrahedron
split (Fig. 1c).  Section 2.1.2 refines an element into eight, and
section 2.1.3 (item 2, Fig. 3) re-labels only the elements adjacent to a
tissue boundary, recursively.

Everything here is point location in exact dyadic "lattice units" (one unit =
one level-0 cell edge, origin at the lattice corner):

* the cube [0,1]^3 of cell (i, j, k) is split by the permutation pi of the
  axes into {1 >= u[pi0] >= u[pi1] >= u[pi2] >= 0}; q indexes pi in the
  lexicographic list of permutations of (x, y, z);
* the tetrahedron containing a point is found from the floor of its
  coordinates and the descending order of their fractional parts;
* a child is a level-(l+1) tetrahedron whose centroid lies in the parent; a
  parent is the level-l tetrahedron containing the child's centroid;
* a leaf is on a label boundary when a leaf sharing a 2-D part of one of its
  faces has another label; the sharing leaves are found by locating points
  pushed just across every face, one per finest-level sub-triangle.

Keys: level << 60 | q << 57 | i << 38 | j << 19 | k (19 bits per index).
"""
import numpy as np

PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
_PERM_CODE = {p[0] * 9 + p[1] * 3 + p[2]: q for q, p in enumerate(PERMS)}
_CODE_TO_Q = np.full(27, -1, dtype=np.int64)
for _c, _q in _PERM_CODE.items():
    _CODE_TO_Q[_c] = _q
_PERM_ARR = np.array(PERMS, dtype=np.int64)


# ---------------------------------------------------------------- keys
def encode(level, q, i, j, k):
    level, q, i, j, k = (np.asarray(a, dtype=np.uint64) for a in (level, q, i, j, k))
    return ((level << np.uint64(60)) | (q << np.uint64(57)) | (i << np.uint64(38))
            | (j << np.uint64(19)) | k)


def decode(keys):
    keys = np.asarray(keys, dtype=np.uint64)
    m19 = np.uint64((1 << 19) - 1)
    level = (keys >> np.uint64(60)).astype(np.int64)
    q = ((keys >> np.uint64(57)) & np.uint64(7)).astype(np.int64)
    i = ((keys >> np.uint64(38)) & m19).astype(np.int64)
    j = ((keys >> np.uint64(19)) & m19).astype(np.int64)
    k = (keys & m19).astype(np.int64)
    return level, q, i, j, k


def level0_keys(cells):
    """All level-0 keys in point-index order ((k*ny + j)*nx + i)*6 + q."""
    nx, ny, nz = cells
    kk, jj, ii, qq = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), np.arange(6),
                                 indexing="ij")
    return encode(0, qq.ravel(), ii.ravel(), jj.ravel(), kk.ravel())


# ------------------------------------------------------------ geometry
def vertices_units(keys):
    """Vertices [n, 4, 3] in lattice units: x0 = cell corner, x1 = x0 + e_pi0,
    x2 = x1 + e_pi1, x3 = x0 + (1, 1, 1), all scaled by 2^-level."""
    level, q, i, j, k = decode(keys)
    n = level.size
    perm = _PERM_ARR[q]
    v = np.zeros((n, 4, 3), dtype=np.float64)
    v[:, 0] = np.stack([i, j, k], 1)
    v[:, 1] = v[:, 0]
    v[np.arange(n), 1, perm[:, 0]] += 1
    v[:, 2] = v[:, 1]
    v[np.arange(n), 2, perm[:, 1]] += 1
    v[:, 3] = v[:, 0] + 1
    return v * (2.0 ** -level)[:, None, None]


def centroid_units(keys):
    return vertices_units(keys).mean(axis=1)


def centroids_mm(keys, origin, h):
    """Centroids as float32 [3, n]: origin + (h 2^-level) (cell + c) in double,
    c[pi0] = 3/4, c[pi1] = 1/2, c[pi2] = 1/4, rounded once to float32."""
    level, q, i, j, k = decode(keys)
    perm = _PERM_ARR[q]
    n = level.size
    c = np.zeros((n, 3), dtype=np.float64)
    c[np.arange(n), perm[:, 0]] = 0.75
    c[np.arange(n), perm[:, 1]] = 0.5
    c[np.arange(n), perm[:, 2]] = 0.25
    cell = np.stack([i, j, k], 1).astype(np.float64)
    hl = float(h) * (2.0 ** -level.astype(np.float64))
    out = np.asarray(origin, dtype=np.float64)[None, :] + hl[:, None] * (cell + c)
    return out.T.astype(np.float32)


def locate(y, level, cells):
    """Key of the level-`level` tetrahedron containing each point y [n, 3]
    (lattice units), and a mask of points inside the domain.  Points must be
    strictly inside a tetrahedron."""
    u = np.asarray(y, dtype=np.float64) * (2.0 ** level)
    cell = np.floor(u)
    frac = u - cell
    cell = cell.astype(np.int64)
    lim = np.asarray(cells, dtype=np.int64) * (1 << level)
    inside = np.all((cell >= 0) & (cell < lim[None, :]), axis=1)
    order = np.argsort(-frac, axis=1, kind="stable")
    sf = np.take_along_axis(frac, order, axis=1)
    if inside.any():
        assert np.all(np.abs(sf[inside]) > 1e-12) and np.all(np.abs(np.diff(sf[inside], axis=1)) > 1e-12), \
            "sample point on a lattice facet"
    q = _CODE_TO_Q[order[:, 0] * 9 + order[:, 1] * 3 + order[:, 2]]
    cc = np.where(inside[:, None], cell, 0)
    keys = encode(np.full(len(q), level), q, cc[:, 0], cc[:, 1], cc[:, 2])
    return keys, inside


def children(keys, cells):
    """The 8 children of each key: [n, 8] keys, ordered by (sub-cell, q)."""
    level, q, i, j, k = decode(keys)
    n = level.size
    cand = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                for qq in range(6):
                    cand.append((dx, dy, dz, qq))
    cand = np.array(cand, dtype=np.int64)               # [48, 4]
    ck = encode(np.repeat(level + 1, 48), np.tile(cand[:, 3], n),
                (2 * np.repeat(i, 48) + np.tile(cand[:, 0], n)),
                (2 * np.repeat(j, 48) + np.tile(cand[:, 1], n)),
                (2 * np.repeat(k, 48) + np.tile(cand[:, 2], n)))
    cent = centroid_units(ck)
    lv = int(level[0]) if n else 0
    assert np.all(level == lv), "children(): one level per call"
    pk, _ = locate(cent, lv, cells)
    mine = pk == np.repeat(np.asarray(keys, dtype=np.uint64), 48)
    mine = mine.reshape(n, 48)
    assert np.all(mine.sum(1) == 8), "a Kuhn tetrahedron has 8 children"
    return ck.reshape(n, 48)[mine].reshape(n, 8)


def parent(keys, cells):
    level = decode(keys)[0]
    assert np.all(level >= 1)
    out = np.empty(len(keys), dtype=np.uint64)
    for lv in np.unique(level):
        m = level == lv
        out[m] = locate(centroid_units(np.asarray(keys)[m]), int(lv) - 1, cells)[0]
    return out


def _face_samples(tri, depth):
    """Interior points, one per sub-triangle of `depth` midpoint splits.
    tri: [n, 3, 3] -> [n, 4^depth, 3] with barycentric (1/2, 1/4, 1/4)."""
    t = tri[:, None]
    for _ in range(depth):
        a, b, c = t[:, :, 0], t[:, :, 1], t[:, :, 2]
        ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
        t = np.concatenate([np.stack(s, 2) for s in
                            ((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca))], 1)
    return (2 * t[:, :, 0] + t[:, :, 1] + t[:, :, 2]) / 4


class LeafSet:
    """Leaf keys with labels, searchable per level."""

    def __init__(self, keys, labels):
        order = np.argsort(keys)
        self.keys = np.asarray(keys, dtype=np.uint64)[order]
        self.labels = np.asarray(labels, dtype=np.int32)[order]

    def find(self, keys):
        pos = np.searchsorted(self.keys, keys)
        pos = np.minimum(pos, len(self.keys) - 1)
        hit = self.keys[pos] == keys
        return hit, pos


def containing_leaf(leaves, y, cells, max_level):
    """Index (into leaves.keys) of the leaf containing each point, -1 outside."""
    res = np.full(len(y), -1, dtype=np.int64)
    for lv in range(max_level + 1):
        keys, inside = locate(y, lv, cells)
        hit, pos = leaves.find(keys)
        take = inside & hit & (res < 0)
        res[take] = pos[take]
    return res


def boundary_mask(leaves, cells, max_level):
    """True for every leaf that shares a 2-D part of a face with a leaf of a
    different label (faces on the domain boundary are ignored)."""
    keys = leaves.keys
    level = decode(keys)[0]
    out = np.zeros(len(keys), dtype=bool)
    for lv in np.unique(level):
        sel = np.nonzero(level == lv)[0]
        depth = max_level - int(lv)
        v = vertices_units(keys[sel])                       # [n, 4, 3]
        for m in range(4):
            face = v[:, [x for x in range(4) if x != m]]    # [n, 3, 3]
            s = _face_samples(face, depth)                  # [n, S, 3]
            opp = v[:, m][:, None, :]
            eta = 2.0 ** -(depth + 8)
            y = (s + eta * (s - opp)).reshape(-1, 3)
            owner = np.repeat(sel, s.shape[1])
            other = containing_leaf(leaves, y, cells, max_level)
            ok = other >= 0
            diff = leaves.labels[other[ok]] != leaves.labels[owner[ok]]
            out[owner[ok][diff]] = True
    return out


def _split_marked(leaves, bmask, cells):
    """Children keys of the marked leaves (grouped by level)."""
    bkeys = leaves.keys[bmask]
    if not len(bkeys):
        return np.zeros(0, dtype=np.uint64)
    lv = decode(bkeys)[0]
    return np.concatenate([children(bkeys[lv == x], cells).reshape(-1) for x in np.unique(lv)])


def _steps(leaves, cells, rounds, converge, max_steps):
    """The marking of each recursion step (section 2.1.3 item 2): yields the
    boundary mask of the current leaves, to be split.  Fixed form: `rounds`
    steps.  Converging form (Fig. 3: repeat until the boundary between
    compartments no longer changes): `rounds` is the finest level; every
    step splits the boundary leaves coarser than it, and the recursion ends
    with the first step that finds none."""
    r = 0
    while converge or r < rounds:
        top = int(decode(leaves().keys)[0].max())
        bmask = boundary_mask(leaves(), cells, top)
        if converge:
            bmask &= decode(leaves().keys)[0] < rounds
            if not bmask.any():
                return
            if r == max_steps:
                raise RuntimeError("no convergence within %d steps" % max_steps)
        r += 1
        yield bmask


def refine_relabel(lattice, label_fn, rounds, converge=False, max_steps=64):
    """Paper section 2.1.3: label every level-0 centroid, then split each
    label-boundary leaf into its 8 children and label only the children:
    `rounds` times, or (converge=True) until no boundary leaf coarser than
    level `rounds` is left.  label_fn(points float32 [3, n]) -> int32 labels.

    Returns (LeafSet, stats) with stats[r] = dict(boundary, children, leaves)."""
    keys = level0_keys(lattice.cells)
    labels = label_fn(centroids_mm(keys, lattice.origin, lattice.h))
    state = [LeafSet(keys, labels)]
    stats = [dict(boundary=0, children=0, leaves=len(keys), labeled=len(keys))]
    for bmask in _steps(lambda: state[0], lattice.cells, rounds, converge, max_steps):
        leaves = state[0]
        kids = _split_marked(leaves, bmask, lattice.cells)
        klab = label_fn(centroids_mm(kids, lattice.origin, lattice.h)) if len(kids) else \
            np.zeros(0, dtype=np.int32)
        keep = ~bmask
        state[0] = LeafSet(np.concatenate([leaves.keys[keep], kids]),
                           np.concatenate([leaves.labels[keep], klab]))
        stats.append(dict(boundary=int(bmask.sum()), children=int(len(kids)),
                          leaves=int(len(state[0].keys)), labeled=int(len(kids))))
    return state[0], stats


# ------------------------------------------------- node-based labeling
# Section 2.1.3 as printed labels mesh nodes and calls a tetrahedron
# contained in a surface when its four nodes are; nodes are identified by
# integer coordinates on the finest grid any level can reach.
MAX_LEVEL = 3
_FINE = 1 << MAX_LEVEL


def lattice_nodes_units(cells):
    """All level-0 nodes [(nx+1)(ny+1)(nz+1), 3] in lattice units, x fastest."""
    nx, ny, nz = cells
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    return np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.float64)


def node_keys(v_units):
    """Keys of nodes given in lattice units (any shape [..., 3])."""
    f = np.rint(np.asarray(v_units, dtype=np.float64) * _FINE).astype(np.int64)
    assert np.all(np.abs(f / _FINE - v_units) == 0), "node off the finest grid"
    return (f[..., 0] << 42) | (f[..., 1] << 21) | f[..., 2]


def nodes_mm(v_units, origin, h):
    """Node positions as float32 [3, n]: origin + h u in double, rounded once."""
    u = np.asarray(v_units, dtype=np.float64).reshape(-1, 3)
    out = np.asarray(origin, dtype=np.float64)[None, :] + float(h) * u
    return out.T.astype(np.float32)


class NodeStore:
    """Enclosure masks of the labeled nodes, searchable by node key."""

    def __init__(self):
        self.keys = np.zeros(0, dtype=np.int64)
        self.masks = np.zeros(0, dtype=np.uint64)

    def add(self, keys, masks):
        k = np.concatenate([self.keys, keys])
        m = np.concatenate([self.masks, masks])
        order = np.argsort(k, kind="stable")
        self.keys, self.masks = k[order], m[order]

    def missing(self, keys):
        pos = np.minimum(np.searchsorted(self.keys, keys), max(len(self.keys) - 1, 0))
        return ~((len(self.keys) > 0) & (self.keys[pos] == keys))

    def get(self, keys):
        pos = np.searchsorted(self.keys, keys)
        assert np.all(self.keys[pos] == keys), "node not labeled"
        return self.masks[pos]


def element_masks(keys, store):
    """AND of the enclosure masks of each tetrahedron's four nodes."""
    nk = node_keys(vertices_units(keys))                # [n, 4]
    m = store.get(nk.reshape(-1)).reshape(-1, 4)
    return m[:, 0] & m[:, 1] & m[:, 2] & m[:, 3]


def refine_relabel_nodes(lattice, mask_fn, label_of_mask, rounds, converge=False, max_steps=64):
    """Section 2.1.3 read literally: the solid-angle test is applied to the
    nodes (item 1 labels every node of the lattice); a tetrahedron belongs to
    a surface when all four of its nodes are enclosed, and takes the label of
    the highest-priority such surface (else 0); then every label-boundary
    leaf is split into its 8 children and only nodes not labeled before are
    evaluated (item 2): `rounds` times, or (converge=True) until no boundary
    leaf coarser than level `rounds` is left.
    mask_fn(points float32 [3, n]) -> uint64 enclosure masks;
    label_of_mask(uint64 masks) -> int32 labels.

    Returns (LeafSet, stats) with stats[r] = dict(boundary, children, leaves,
    nodes = nodes labeled that round)."""
    store = NodeStore()
    nodes = lattice_nodes_units(lattice.cells)
    store.add(node_keys(nodes), mask_fn(nodes_mm(nodes, lattice.origin, lattice.h)))
    keys = level0_keys(lattice.cells)
    state = [LeafSet(keys, label_of_mask(element_masks(keys, store)))]
    stats = [dict(boundary=0, children=0, leaves=len(keys), nodes=len(nodes))]
    for bmask in _steps(lambda: state[0], lattice.cells, rounds, converge, max_steps):
        leaves = state[0]
        kids = _split_marked(leaves, bmask, lattice.cells)
        n_new = 0
        if len(kids):
            v = vertices_units(kids).reshape(-1, 3)
            nk, first = np.unique(node_keys(v), return_index=True)
            new = store.missing(nk)
            n_new = int(new.sum())
            if n_new:
                store.add(nk[new], mask_fn(nodes_mm(v[first[new]], lattice.origin, lattice.h)))
            klab = label_of_mask(element_masks(kids, store))
        else:
            klab = np.zeros(0, dtype=np.int32)
        keep = ~bmask
        state[0] = LeafSet(np.concatenate([leaves.keys[keep], kids]),
                           np.concatenate([leaves.labels[keep], klab]))
        stats.append(dict(boundary=int(bmask.sum()), children=int(len(kids)),
                          leaves=int(len(state[0].keys)), nodes=n_new))
    return state[0], stats
