"""Synthetic tetrahedral meshes shaped like the paper's verification and vascular cases.

* `cube_kuhn`: structured box, each hexahedron split into 6 tetrahedra along its
  main diagonal (Kuhn/Freudenthal split, conforming across cells).
* `tube`: straight circular pipe along z; a square cross-section grid mapped to
  the disc with the elliptical grid map (x sqrt(1 - y^2/2), y sqrt(1 - x^2/2)),
  extruded in layers and Kuhn-split, with seeded jitter of interior nodes and a
  seeded shuffle of vertex and element ids.
* `spheroid`: a prolate spheroidal chamber along x, truncated by two flat caps,
  built the same way with a radius that varies along the axis.

Every generator returns a `Mesh` (coords [nv][3] float64, tets [nt][4] int32,
bfaces [nb][3] int32, btags [nb] int32).  Random numbers come from splitmix64.
"""
from dataclasses import dataclass, field
import numpy as np

from .rng import uniform01, permutation

# Tags used by the generators.
CUBE_TAGS = {"x0": 1, "x1": 2, "y0": 3, "y1": 4, "z0": 5, "z1": 6}
TUBE_TAGS = {"inlet": 1, "outlet": 2, "wall": 3}
SPHEROID_TAGS = {"cap_lo": 1, "cap_hi": 2, "wall": 3}


@dataclass
class Mesh:
    coords: np.ndarray          # [nv][3] float64
    tets: np.ndarray            # [nt][4] int32
    bfaces: np.ndarray          # [nb][3] int32
    btags: np.ndarray           # [nb]    int32
    info: dict = field(default_factory=dict)

    @property
    def nv(self):
        return self.coords.shape[0]

    @property
    def nt(self):
        return self.tets.shape[0]


def _grid_ids(nx, ny, nz):
    return np.arange((nx + 1) * (ny + 1) * (nz + 1), dtype=np.int64).reshape(nz + 1, ny + 1, nx + 1)


def _kuhn_tets(nx, ny, nz, mirror_xy=False):
    """Kuhn split of an nx*ny*nz cell grid; vertex (i,j,k) has id i + (nx+1)(j + (ny+1)k).

    Cell corners c[dz][dy][dx]; for every permutation (p0,p1,p2) of the axes the
    tetrahedron is c000 -> c000+e_p0 -> c000+e_p0+e_p1 -> c111.  mirror_xy: cells
    in the lower half of x (of y) use the split reflected in x (in y), so the main
    diagonal of every cell points away from the grid centre; reflected splits
    meet conformingly on the mirror planes.  On a square grid mapped to a disc
    this splits each corner cell through its corner vertex instead of across it.
    """
    ids = _grid_ids(nx, ny, nz)
    c = {}
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                c[(dx, dy, dz)] = ids[dz:dz + nz, dy:dy + ny, dx:dx + nx].reshape(-1)
    if mirror_xy:
        ci = np.broadcast_to(np.arange(nx)[None, None, :], (nz, ny, nx)).reshape(-1)
        cj = np.broadcast_to(np.arange(ny)[None, :, None], (nz, ny, nx)).reshape(-1)
        fx, fy = ci < nx // 2, cj < ny // 2

        def corner(dx, dy, dz):
            a = np.where(fx, c[(1 - dx, dy, dz)], c[(dx, dy, dz)])
            b = np.where(fx, c[(1 - dx, 1 - dy, dz)], c[(dx, 1 - dy, dz)])
            return np.where(fy, b, a)
    else:
        def corner(dx, dy, dz):
            return c[(dx, dy, dz)]
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    out = []
    for p in perms:
        e = [0, 0, 0]
        path = [corner(0, 0, 0)]
        for ax in p[:2]:
            e[ax] = 1
            path.append(corner(*e))
        path.append(corner(1, 1, 1))
        out.append(np.stack(path, axis=1))
    # interleave so that the 6 tets of one cell are consecutive
    tets = np.stack(out, axis=1).reshape(-1, 4)
    return tets


def tet_signed_volumes(coords, tets):
    x0 = coords[tets[:, 0]]
    d1 = coords[tets[:, 1]] - x0
    d2 = coords[tets[:, 2]] - x0
    d3 = coords[tets[:, 3]] - x0
    return np.einsum("ij,ij->i", d1, np.cross(d2, d3)) / 6.0


def _orient_positive(coords, tets):
    vol = tet_signed_volumes(coords, tets)
    neg = vol < 0
    t = tets.copy()
    t[neg, 2], t[neg, 3] = tets[neg, 3], tets[neg, 2]
    return t


def boundary_faces(tets, nv):
    """Faces that belong to exactly one tetrahedron, as sorted vertex triples."""
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    f = np.sort(tets[:, loc].reshape(-1, 3).astype(np.int64), axis=1)
    key = (f[:, 0] * nv + f[:, 1]) * nv + f[:, 2]
    uniq, idx, cnt = np.unique(key, return_index=True, return_counts=True)
    return f[idx[cnt == 1]].astype(np.int32)


def tet_quality(coords, tets, sign=None):
    """Volume over cubed longest edge (0.118 for the regular tetrahedron); negative
    for inverted elements when sign gives the reference orientation."""
    vol = tet_signed_volumes(coords, tets)
    if sign is not None:
        vol = vol * sign
    X = coords[tets]
    lmax = np.zeros(len(tets))
    for a, b in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        lmax = np.maximum(lmax, np.linalg.norm(X[:, a] - X[:, b], axis=1))
    return vol / lmax ** 3


def _jitter_interior(coords, tets, interior, amp, seed):
    """Uniform jitter in [-amp, amp]^3 on interior nodes; the vertices of any tet
    whose quality (volume / longest edge^3) falls below half of its unjittered
    value, inverted ones included, get their jitter halved, repeatedly."""
    nv = coords.shape[0]
    r = uniform01(seed, 3 * nv).reshape(nv, 3) * 2.0 - 1.0
    jit = r * amp
    jit[~interior] = 0.0
    sign = np.sign(tet_signed_volumes(coords, tets))
    q0 = tet_quality(coords, tets, sign)
    for _ in range(60):
        bad = tet_quality(coords + jit, tets, sign) < 0.5 * q0
        if not bad.any():
            break
        vb = np.unique(tets[bad].reshape(-1))
        jit[vb] *= 0.5
    return coords + jit


def _shuffle(coords, tets, seed):
    nv, nt = coords.shape[0], tets.shape[0]
    pv = permutation(seed, nv, offset=0)           # new position -> old vertex
    inv = np.empty(nv, dtype=np.int64)
    inv[pv] = np.arange(nv)
    pe = permutation(seed, nt, offset=nv)
    return coords[pv], inv[tets[pe]].astype(np.int32), pv, pe


def cube_kuhn(n, length=1.0, origin=(0.0, 0.0, 0.0)):
    """Unit (or scaled) cube, n^3 hexahedra, 6n^3 tets, (n+1)^3 vertices.  Tags:
    x0=1, x1=2, y0=3, y1=4, z0=5, z1=6 (a face on an edge/corner takes the first
    matching tag in that order)."""
    g = np.linspace(0.0, length, n + 1)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + np.asarray(origin, float)
    tets = _orient_positive(coords, _kuhn_tets(n, n, n)).astype(np.int32)
    bf = boundary_faces(tets, coords.shape[0])
    cen = coords[bf].mean(axis=1) - np.asarray(origin, float)
    tol = 1e-9 * length
    tags = np.zeros(len(bf), dtype=np.int32)
    for ax, (lo, hi) in enumerate([(1, 2), (3, 4), (5, 6)]):
        tags[(tags == 0) & (np.abs(cen[:, ax]) < tol)] = lo
        tags[(tags == 0) & (np.abs(cen[:, ax] - length) < tol)] = hi
    # corner faces were assigned by axis order; re-derive exactly: a face lies on a
    # plane iff all its vertices do
    tags[:] = 0
    for ax, (lo, hi) in enumerate([(1, 2), (3, 4), (5, 6)]):
        v = coords[bf][:, :, ax] - origin[ax]
        tags[(tags == 0) & np.all(np.abs(v) < tol, axis=1)] = lo
        tags[(tags == 0) & np.all(np.abs(v - length) < tol, axis=1)] = hi
    assert (tags > 0).all()
    return Mesh(coords, tets, bf, tags, {"kind": "cube", "n": n, "h": length / n})


def _disc_map(sx, sy):
    """Elliptical grid map of the square [-1,1]^2 onto the unit disc."""
    return sx * np.sqrt(1.0 - 0.5 * sy * sy), sy * np.sqrt(1.0 - 0.5 * sx * sx)


def tube(nxy=32, nz=160, radius=1.0, length=10.0, jitter=0.1, seed=0, shuffle=True):
    """Straight tube along z with nxy^2 x nz hexahedra split into 6 tets each
    (Kuhn split mirrored about the axis planes, see _kuhn_tets).

    Interior nodes are jittered uniformly by up to jitter*h per coordinate with
    h = 2*radius/nxy, limited where it would halve an element's quality.  Tags:
    inlet (z=0) 1, outlet (z=length) 2, wall 3.
    """
    s = np.linspace(-1.0, 1.0, nxy + 1)
    zc = np.linspace(0.0, length, nz + 1)
    Z, SY, SX = np.meshgrid(zc, s, s, indexing="ij")
    X, Y = _disc_map(SX, SY)
    coords = np.stack([radius * X.ravel(), radius * Y.ravel(), Z.ravel()], axis=1)
    tets = _orient_positive(coords, _kuhn_tets(nxy, nxy, nz, mirror_xy=True)).astype(np.int32)
    h = 2.0 * radius / nxy
    on_wall = (np.abs(SX.ravel()) == 1.0) | (np.abs(SY.ravel()) == 1.0)
    on_cap = (Z.ravel() == 0.0) | (Z.ravel() == length)
    interior = ~(on_wall | on_cap)
    if jitter > 0:
        coords = _jitter_interior(coords, tets, interior, jitter * h, seed)
    if shuffle:
        coords, tets, _, _ = _shuffle(coords, tets, seed + 0x5EED)
    bf = boundary_faces(tets, coords.shape[0])
    zf = coords[bf][:, :, 2]
    tags = np.full(len(bf), TUBE_TAGS["wall"], dtype=np.int32)
    tags[np.all(np.abs(zf) < 1e-12, axis=1)] = TUBE_TAGS["inlet"]
    tags[np.all(np.abs(zf - length) < 1e-12, axis=1)] = TUBE_TAGS["outlet"]
    return Mesh(coords, tets, bf, tags, {"kind": "tube", "nxy": nxy, "nz": nz, "radius": radius,
                                         "length": length, "h": h, "seed": seed})


def tube_for_target(n_tets, seed=0, radius=1.0, length=10.0):
    """Tube of about n_tets tets keeping the aspect of the family: nxy = round((T/30)^(1/3))
    scaled to cross-section cells, nz from the remaining budget."""
    nr = max(2, int(round((n_tets / 30.0) ** (1.0 / 3.0))))
    nz = max(2, int(round(n_tets / (6.0 * nr * nr))))
    return tube(nxy=nr, nz=nz, radius=radius, length=length, seed=seed)


def spheroid(nyz=105, nx=121, semi=(4.0, 3.0, 3.0), xcut=3.5, jitter=0.1, seed=0, shuffle=True):
    """Prolate spheroidal chamber along x (semi-axes a,b,b), truncated at |x| = xcut.

    Cross-sections are discs of radius b*sqrt(1 - x^2/a^2) meshed by the mapped
    square grid.  Tags: cap x=-xcut 1, cap x=+xcut 2, wall 3.
    """
    a, b, _ = semi
    s = np.linspace(-1.0, 1.0, nyz + 1)
    xc = np.linspace(-xcut, xcut, nx + 1)
    XX, SZ, SY = np.meshgrid(xc, s, s, indexing="ij")
    U, V = _disc_map(SY, SZ)
    r = b * np.sqrt(1.0 - XX * XX / (a * a))
    coords = np.stack([XX.ravel(), (r * U).ravel(), (r * V).ravel()], axis=1)
    # index order (i fastest) is (sy, sz, x): build tets on that grid then they map through
    tets = _orient_positive(coords, _kuhn_tets(nyz, nyz, nx, mirror_xy=True)).astype(np.int32)
    h = 2.0 * b / nyz
    on_wall = (np.abs(SY.ravel()) == 1.0) | (np.abs(SZ.ravel()) == 1.0)
    on_cap = np.abs(np.abs(XX.ravel()) - xcut) < 1e-12
    interior = ~(on_wall | on_cap)
    if jitter > 0:
        coords = _jitter_interior(coords, tets, interior, jitter * h, seed)
    if shuffle:
        coords, tets, _, _ = _shuffle(coords, tets, seed + 0x5EED)
    bf = boundary_faces(tets, coords.shape[0])
    xf = coords[bf][:, :, 0]
    tags = np.full(len(bf), SPHEROID_TAGS["wall"], dtype=np.int32)
    tags[np.all(np.abs(xf + xcut) < 1e-12, axis=1)] = SPHEROID_TAGS["cap_lo"]
    tags[np.all(np.abs(xf - xcut) < 1e-12, axis=1)] = SPHEROID_TAGS["cap_hi"]
    return Mesh(coords, tets, bf, tags, {"kind": "spheroid", "nyz": nyz, "nx": nx, "semi": semi,
                                         "xcut": xcut, "h": h, "seed": seed})


def mesh_stats(mesh):
    """Mesh statistics in the style of the paper's mesh table: element and vertex
    counts, min/avg/max edge length and the average per-element edge ratio."""
    t = mesh.tets
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    L = np.stack([np.linalg.norm(mesh.coords[t[:, i]] - mesh.coords[t[:, j]], axis=1)
                  for i, j in pairs], axis=1)
    return {"elements": int(mesh.nt), "vertices": int(mesh.nv),
            "h_min": float(L.min()), "h_avg": float(L.mean()), "h_max": float(L.max()),
            "edge_ratio_avg": float((L.max(axis=1) / L.min(axis=1)).mean())}
