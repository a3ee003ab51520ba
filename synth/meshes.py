"""Closed, outward-oriented triangle meshes built in float64.

Every mesh here is a radial graph (or an affine image of a sphere) around a
known centre, so it is star-shaped about that centre: the ray from the centre
through any point crosses the surface exactly once.  Triangles are ordered
counter-clockwise seen from outside, which makes the winding number +1 inside.
"""
import numpy as np
from scipy import special


def icosahedron():
    """Regular icosahedron inscribed in the unit sphere.

    Vertices are the cyclic permutations of (0, +-1, +-phi); faces are found as
    the vertex triples at mutual edge distance 2 and oriented so their normal
    points away from the origin.
    """
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    verts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            verts.append((0.0, s1, s2 * phi))
            verts.append((s1, s2 * phi, 0.0))
            verts.append((s2 * phi, 0.0, s1))
    v = np.array(verts, dtype=np.float64)
    faces = []
    n = len(v)
    d2 = ((v[:, None, :] - v[None, :, :]) ** 2).sum(-1)
    edge = np.abs(d2 - 4.0) < 1e-9
    for a in range(n):
        for b in range(a + 1, n):
            if not edge[a, b]:
                continue
            for c in range(b + 1, n):
                if edge[a, c] and edge[b, c]:
                    nrm = np.cross(v[b] - v[a], v[c] - v[a])
                    if np.dot(nrm, v[a] + v[b] + v[c]) > 0:
                        faces.append((a, b, c))
                    else:
                        faces.append((a, c, b))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(faces, dtype=np.int64)
    assert f.shape == (20, 3)
    return v, f


def icosphere(subdiv):
    """Unit icosphere: `subdiv` rounds of 4-way midpoint splits, 20*4^subdiv faces."""
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(subdiv):
        mid = {}
        new_faces = []

        def midpoint(i, j):
            key = (i, j) if i < j else (j, i)
            k = mid.get(key)
            if k is None:
                m = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
                m /= np.linalg.norm(m)
                k = len(verts)
                verts.append(tuple(m))
                mid[key] = k
            return k

        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            new_faces += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        f = np.array(new_faces, dtype=np.int64)
    return np.array(verts, dtype=np.float64), f


def geodesic_sphere(nu):
    """Unit geodesic sphere of frequency nu: 20*nu^2 faces, 10*nu^2+2 vertices.

    Each icosahedron face is cut into a triangular grid of nu^2 triangles; grid
    points shared between faces are merged through their integer barycentric
    weights on the icosahedron's vertices.
    """
    iv, ifc = icosahedron()
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nu + 1), indexing="ij")
    keep = ii + jj <= nu
    ii, jj = ii[keep], jj[keep]
    npf = ii.size
    local = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    local[ii, jj] = np.arange(npf)
    # integer weights of every grid point of every face on the 12 vertices
    w = np.zeros((20, npf, 12), dtype=np.int64)
    for fi, (A, B, C) in enumerate(ifc):
        w[fi, :, A] += nu - ii - jj
        w[fi, :, B] += ii
        w[fi, :, C] += jj
    w = w.reshape(-1, 12)
    uniq, inv = np.unique(w, axis=0, return_inverse=True)
    inv = inv.reshape(20, npf)
    p = uniq.astype(np.float64) @ iv / float(nu)
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    # up triangles (i,j),(i+1,j),(i,j+1); down (i+1,j),(i+1,j+1),(i,j+1)
    ui, uj = np.nonzero(np.add.outer(np.arange(nu), np.arange(nu)) < nu)
    di, dj = np.nonzero(np.add.outer(np.arange(nu), np.arange(nu)) + 1 < nu)
    up = np.stack([local[ui, uj], local[ui + 1, uj], local[ui, uj + 1]], 1)
    dn = np.stack([local[di + 1, dj], local[di + 1, dj + 1], local[di, dj + 1]], 1)
    tri_local = np.concatenate([up, dn])
    faces = np.concatenate([inv[fi][tri_local] for fi in range(20)])
    return p, faces.astype(np.int64)


def real_sph_harm(lmax, dirs):
    """Real orthonormal spherical harmonics Y_lm, l = 0..lmax, at unit vectors.

    Returns an array [(lmax+1)^2, n] ordered (l, m) with m = -l..l.
    """
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    out = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            ylm = special.sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                out.append(ylm.real)
            elif m > 0:
                out.append(np.sqrt(2.0) * (-1) ** m * ylm.real)
            else:
                out.append(np.sqrt(2.0) * (-1) ** m * ylm.imag)
    return np.array(out)


def sh_shell(unit_v, radius, coeffs, lmax=6, amp_frac=0.05, center=(0.0, 0.0, 0.0)):
    """Radially perturbed sphere r(u) = R + s * sum c_lm Y_lm(u).

    The scale s is chosen so that the largest |r - R| over the mesh vertices is
    exactly amp_frac * R.
    """
    f = coeffs @ real_sph_harm(lmax, unit_v)
    s = amp_frac * radius / np.max(np.abs(f))
    r = radius + s * f
    return np.asarray(center, dtype=np.float64) + unit_v * r[:, None]


def random_rotation(rng):
    """Rotation matrix from a normalised 4-D Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid(unit_v, semi_axes, rotation, center):
    """Affine image of a unit sphere mesh: centre + R diag(a, b, c) u."""
    scaled = unit_v * np.asarray(semi_axes, dtype=np.float64)[None, :]
    return np.asarray(center, dtype=np.float64) + scaled @ np.asarray(rotation).T


def signed_volume(v, f):
    """Enclosed volume by the divergence theorem (positive for outward faces)."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def check_closed_oriented(f):
    """True when every directed edge occurs once and its reverse once."""
    f = np.asarray(f, dtype=np.int64)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    m = int(f.max()) + 1
    fwd = np.sort(e[:, 0] * m + e[:, 1])
    if np.any(fwd[1:] == fwd[:-1]):
        return False
    rev = np.sort(e[:, 1] * m + e[:, 0])
    return bool(np.array_equal(fwd, rev))


def star_shaped_about(v, f, center):
    """Smallest signed volume of the cones (centre, v0, v1, v2); > 0 means every
    face is seen from the centre on its inner side."""
    c = np.asarray(center, dtype=np.float64)
    a, b, d = v[f[:, 0]] - c, v[f[:, 1]] - c, v[f[:, 2]] - c
    return float(np.einsum("ij,ij->i", a, np.cross(b, d)).min())
