"""Seeded synthetic meshes and fields: the inputs both the GPU library and the oracle consume.

This module builds mesh geometry (face area vectors, centroids, volumes, interpolation weights) and
analytic input fields.  It holds none of the method's arithmetic: no interpolation, gradient,
flux, assembly or solve happens here.  The paper's meshes (OpenFOAM cases, patient geometry) are not
available, so every workload is a seeded stand-in with the shapes the method targets: jittered
unstructured tetrahedra (and extruded triangular prisms for 2D cases).

Conventions (the paper's static graph, Sec. "Structural isomorphism ... static graph construction"):
  owner[F], neighbour[Fi]   int32, internal faces first, then boundary faces grouped by patch
  Sf[F,3]                   face area vector pointing out of the owner
  Cf[F,3], C[Nc,3], V[Nc]   face centroids, cell centroids, cell volumes
  w[Fi]                     owner interpolation weight, w = S.(C_N - C_f) / S.(C_N - C_O)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# boundary-condition type codes shared with include/difvm.h (values are part of the ABI)
U_FIXED, U_ZEROGRAD, U_EMPTY = 0, 1, 2
P_ZEROGRAD, P_FIXED, P_WINDKESSEL, P_EMPTY = 0, 1, 2, 3


@dataclass
class Patch:
    name: str
    start: int          # first boundary face, in [Fi, Fi+Fb)
    size: int
    u_type: int
    p_type: int
    wk_id: int = -1


@dataclass
class Mesh:
    owner: np.ndarray
    neighbour: np.ndarray
    Sf: np.ndarray
    Cf: np.ndarray
    C: np.ndarray
    V: np.ndarray
    w: np.ndarray
    patches: list
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return int(self.V.shape[0])

    @property
    def n_internal_faces(self):
        return int(self.neighbour.shape[0])

    @property
    def n_faces(self):
        return int(self.owner.shape[0])

    @property
    def n_boundary_faces(self):
        return self.n_faces - self.n_internal_faces

    def patch(self, name):
        for p in self.patches:
            if p.name == name:
                return p
        raise KeyError(name)


# ----------------------------------------------------------------------------------------------
# geometry helpers (inputs only)
# ----------------------------------------------------------------------------------------------

def _tri_area_vec(a, b, c):
    return 0.5 * np.cross(b - a, c - a)


def _tet_faces(points, tets):
    """Faces of a conforming tet mesh. Returns (owner, neighbour, face_vertex_triples, internal_count)
    with internal faces first ordered by (owner, neighbour) and boundary faces ordered by owner."""
    nt = tets.shape[0]
    # face k of a tet is the triangle opposite vertex k
    opp = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    fv = tets[:, opp].reshape(-1, 3)                       # (4nt, 3)
    cell = np.repeat(np.arange(nt, dtype=np.int64), 4)
    key_sorted = np.sort(fv, axis=1).astype(np.int64)
    nv = int(points.shape[0])
    bits = max(1, int(nv - 1).bit_length())
    if 3 * bits > 62:
        raise ValueError("too many vertices for face keys")
    key = (key_sorted[:, 0] << (2 * bits)) | (key_sorted[:, 1] << bits) | key_sorted[:, 2]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same_next = np.zeros(ks.shape[0], dtype=bool)
    same_next[:-1] = ks[:-1] == ks[1:]
    if np.any(same_next[:-1] & same_next[1:]):
        raise ValueError("non-manifold mesh: a face shared by more than two cells")
    first = np.flatnonzero(same_next)                     # index of first of a pair
    is_pair_second = np.zeros(ks.shape[0], dtype=bool)
    is_pair_second[first + 1] = True
    single = np.flatnonzero(~same_next & ~is_pair_second)
    c0 = cell[order[first]]
    c1 = cell[order[first + 1]]
    own_i = np.minimum(c0, c1)
    nbr_i = np.maximum(c0, c1)
    # face vertices taken from the owner's copy
    tri_i = np.where((c0 <= c1)[:, None], fv[order[first]], fv[order[first + 1]])
    srt = np.lexsort((nbr_i, own_i))
    own_i, nbr_i, tri_i = own_i[srt], nbr_i[srt], tri_i[srt]
    own_b = cell[order[single]]
    tri_b = fv[order[single]]
    srt = np.argsort(own_b, kind="stable")
    return own_i, nbr_i, tri_i, own_b[srt], tri_b[srt]


def _orient_tets(points, tets):
    a, b, c, d = (points[tets[:, k]] for k in range(4))
    vol6 = np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))
    neg = vol6 < 0
    tets = tets.copy()
    tets[neg, 2], tets[neg, 3] = tets[neg, 3], tets[neg, 2].copy()
    return tets


def _weights(Sf_i, Cf_i, C, own, nbr):
    CN = C[nbr]
    CO = C[own]
    num = np.einsum("ij,ij->i", Sf_i, CN - Cf_i)
    den = np.einsum("ij,ij->i", Sf_i, CN - CO)
    return num / den


def tet_mesh(points, tets, classify, patch_specs, name=""):
    """Build a Mesh from a conforming tet mesh.

    classify(Cf_b, tri_points) -> integer patch index per boundary face (index into patch_specs).
    patch_specs: list of (name, u_type, p_type, wk_id).
    """
    points = np.ascontiguousarray(points, dtype=np.float64)
    tets = _orient_tets(points, np.asarray(tets, dtype=np.int64))
    own_i, nbr_i, tri_i, own_b, tri_b = _tet_faces(points, tets)
    C = points[tets].mean(axis=1)
    a, b, c, d = (points[tets[:, k]] for k in range(4))
    V = np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a)) / 6.0

    def geo(tri, own):
        p0, p1, p2 = points[tri[:, 0]], points[tri[:, 1]], points[tri[:, 2]]
        S = _tri_area_vec(p0, p1, p2)
        Cf = (p0 + p1 + p2) / 3.0
        flip = np.einsum("ij,ij->i", S, Cf - C[own]) < 0
        S[flip] *= -1.0
        return S, Cf

    S_i, Cf_i = geo(tri_i, own_i)
    S_b, Cf_b = geo(tri_b, own_b)
    pid = np.asarray(classify(Cf_b, points[tri_b]), dtype=np.int64)
    order = np.lexsort((np.arange(own_b.shape[0]), pid))  # group by patch, keep owner order
    own_b, S_b, Cf_b, pid = own_b[order], S_b[order], Cf_b[order], pid[order]
    Fi = own_i.shape[0]
    patches = []
    start = Fi
    for k, (pname, ut, pt, wk) in enumerate(patch_specs):
        n = int(np.count_nonzero(pid == k))
        patches.append(Patch(pname, start, n, ut, pt, wk))
        start += n
    if start != Fi + own_b.shape[0]:
        raise ValueError("boundary faces not covered by patches")
    w = _weights(S_i, Cf_i, C, own_i, nbr_i)
    return Mesh(owner=np.concatenate([own_i, own_b]).astype(np.int32),
                neighbour=nbr_i.astype(np.int32),
                Sf=np.ascontiguousarray(np.concatenate([S_i, S_b])),
                Cf=np.ascontiguousarray(np.concatenate([Cf_i, Cf_b])),
                C=np.ascontiguousarray(C), V=V, w=w, patches=patches, name=name,
                meta={"points": points, "tets": tets})


# ----------------------------------------------------------------------------------------------
# structured Kuhn (Freudenthal) cube
# ----------------------------------------------------------------------------------------------

_KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _kuhn_tets(nx, ny, nz):
    """Six tets per hex along the (0,0,0)->(1,1,1) diagonal, same rule in every hex (conforming)."""
    def vid(i, j, k):
        return (i * (ny + 1) + j) * (nz + 1) + k
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    out = []
    for perm in _KUHN_PERMS:
        cur = np.stack([I, J, K], axis=1)
        vs = [vid(cur[:, 0], cur[:, 1], cur[:, 2])]
        for ax in perm:
            cur = cur.copy()
            cur[:, ax] += 1
            vs.append(vid(cur[:, 0], cur[:, 1], cur[:, 2]))
        out.append(np.stack(vs, axis=1))
    # hex-major ordering: the 6 tets of a hex are consecutive
    return np.stack(out, axis=1).reshape(-1, 4)


def _box_points(nx, ny, nz, lo, hi, jitter, rng):
    xs = [np.linspace(lo[d], hi[d], n + 1) for d, n in enumerate((nx, ny, nz))]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter > 0:
        h = np.array([(hi[d] - lo[d]) / n for d, n in enumerate((nx, ny, nz))])
        idx = np.stack(np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                                   indexing="ij"), axis=-1).reshape(-1, 3)
        on_bnd = (idx == 0) | (idx == np.array([nx, ny, nz]))
        d = rng.uniform(-jitter, jitter, size=P.shape) * h
        d[on_bnd] = 0.0                      # boundary nodes move only tangentially
        P = P + d
    return P


def kuhn_cube(n, jitter=0.15, seed=2603002, patches="walls", lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
              nxyz=None):
    """Unit cube of n^3 hexes, each split into 6 Kuhn tets; interior nodes jittered by U[-j,j]*h.

    patches="walls": one fixedValue patch; "sides": six patches x0,x1,y0,y1,z0,z1;
    "channel": inlet x0 (U fixed), outlet x1 (U zeroGradient, Windkessel p), walls (rest).
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = (n, n, n) if nxyz is None else nxyz
    P = _box_points(nx, ny, nz, lo, hi, jitter, rng)
    T = _kuhn_tets(nx, ny, nz)
    lo_a, hi_a = np.asarray(lo, float), np.asarray(hi, float)
    tol = 1e-9 * float(np.max(hi_a - lo_a))

    def side_of(Cf):
        s = np.full(Cf.shape[0], -1, dtype=np.int64)
        for d in range(3):
            s[np.abs(Cf[:, d] - lo_a[d]) < tol] = 2 * d
            s[np.abs(Cf[:, d] - hi_a[d]) < tol] = 2 * d + 1
        if np.any(s < 0):
            raise ValueError("boundary face off the box surface")
        return s

    if patches == "walls":
        specs = [("walls", U_FIXED, P_FIXED, -1)]
        cls = lambda Cf, tri: np.zeros(Cf.shape[0], dtype=np.int64)
    elif patches == "sides":
        specs = [(nm, U_FIXED, P_FIXED, -1) for nm in ("x0", "x1", "y0", "y1", "z0", "z1")]
        cls = lambda Cf, tri: side_of(Cf)
    elif patches == "channel":
        specs = [("inlet", U_FIXED, P_ZEROGRAD, -1), ("outlet", U_ZEROGRAD, P_WINDKESSEL, 0),
                 ("walls", U_FIXED, P_ZEROGRAD, -1)]
        def cls(Cf, tri):
            s = side_of(Cf)
            return np.where(s == 0, 0, np.where(s == 1, 1, 2))
    elif patches == "channel_p0":
        specs = [("inlet", U_FIXED, P_ZEROGRAD, -1), ("outlet", U_ZEROGRAD, P_FIXED, -1),
                 ("walls", U_FIXED, P_ZEROGRAD, -1)]
        def cls(Cf, tri):
            s = side_of(Cf)
            return np.where(s == 0, 0, np.where(s == 1, 1, 2))
    else:
        raise ValueError(patches)
    return tet_mesh(P, T, cls, specs, name=f"kuhn{nx}x{ny}x{nz}")


# ----------------------------------------------------------------------------------------------
# extruded triangle meshes (2D cases, empty front/back)
# ----------------------------------------------------------------------------------------------

def extruded_triangles(pts2, tris, dz, classify_edge, patch_specs, name=""):
    """Prisms from a 2D triangulation extruded by dz along z.  Side quads are planar rectangles
    (exact geometry); front/back triangles form the last patch, which must be of empty type.

    classify_edge(mid_xy) -> patch index for boundary edges (front/back patch excluded).
    """
    pts2 = np.asarray(pts2, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    a, b, c = pts2[tris[:, 0]], pts2[tris[:, 1]], pts2[tris[:, 2]]
    cr = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    tris = tris.copy()
    neg = cr < 0
    tris[neg, 1], tris[neg, 2] = tris[neg, 2], tris[neg, 1].copy()
    a, b, c = pts2[tris[:, 0]], pts2[tris[:, 1]], pts2[tris[:, 2]]
    area = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    nt = tris.shape[0]
    cxy = (a + b + c) / 3.0
    C = np.concatenate([cxy, np.full((nt, 1), 0.5 * dz)], axis=1)
    V = area * dz
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    ecell = np.tile(np.arange(nt), 3)
    ek = np.sort(e, axis=1)
    key = ek[:, 0] * (pts2.shape[0] + 1) + ek[:, 1]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.zeros(ks.shape[0], dtype=bool)
    same[:-1] = ks[:-1] == ks[1:]
    second = np.zeros_like(same)
    second[np.flatnonzero(same) + 1] = True
    first = np.flatnonzero(same)
    single = np.flatnonzero(~same & ~second)
    c0, c1 = ecell[order[first]], ecell[order[first + 1]]
    own_i, nbr_i = np.minimum(c0, c1), np.maximum(c0, c1)
    ed_i = ek[order[first]]
    srt = np.lexsort((nbr_i, own_i))
    own_i, nbr_i, ed_i = own_i[srt], nbr_i[srt], ed_i[srt]
    own_b = ecell[order[single]]
    ed_b = ek[order[single]]

    def quad_geo(ed, own):
        p, q = pts2[ed[:, 0]], pts2[ed[:, 1]]
        t = q - p
        S = np.stack([t[:, 1] * dz, -t[:, 0] * dz, np.zeros(t.shape[0])], axis=1)
        mid = 0.5 * (p + q)
        Cf = np.concatenate([mid, np.full((t.shape[0], 1), 0.5 * dz)], axis=1)
        flip = np.einsum("ij,ij->i", S, Cf - C[own]) < 0
        S[flip] *= -1.0
        return S, Cf, mid

    S_i, Cf_i, _ = quad_geo(ed_i, own_i)
    S_b, Cf_b, mid_b = quad_geo(ed_b, own_b)
    pid = np.asarray(classify_edge(mid_b), dtype=np.int64)
    order = np.lexsort((own_b, pid))
    own_b, S_b, Cf_b, pid = own_b[order], S_b[order], Cf_b[order], pid[order]
    # front (z=0) and back (z=dz) triangles: empty patch
    cells = np.arange(nt)
    S_fb = np.concatenate([np.stack([np.zeros(nt), np.zeros(nt), -area], 1),
                           np.stack([np.zeros(nt), np.zeros(nt), area], 1)])
    Cf_fb = np.concatenate([np.concatenate([cxy, np.zeros((nt, 1))], 1),
                            np.concatenate([cxy, np.full((nt, 1), dz)], 1)])
    own_fb = np.concatenate([cells, cells])
    srt = np.argsort(own_fb, kind="stable")
    own_fb, S_fb, Cf_fb = own_fb[srt], S_fb[srt], Cf_fb[srt]
    Fi = own_i.shape[0]
    patches = []
    start = Fi
    for k, (pname, ut, pt, wk) in enumerate(patch_specs[:-1]):
        n = int(np.count_nonzero(pid == k))
        patches.append(Patch(pname, start, n, ut, pt, wk))
        start += n
    pname, ut, pt, wk = patch_specs[-1]
    patches.append(Patch(pname, start, 2 * nt, ut, pt, wk))
    w = _weights(S_i, Cf_i, C, own_i, nbr_i)
    return Mesh(owner=np.concatenate([own_i, own_b, own_fb]).astype(np.int32),
                neighbour=nbr_i.astype(np.int32),
                Sf=np.ascontiguousarray(np.concatenate([S_i, S_b, S_fb])),
                Cf=np.ascontiguousarray(np.concatenate([Cf_i, Cf_b, Cf_fb])),
                C=np.ascontiguousarray(C), V=V, w=w, patches=patches, name=name,
                meta={"points2": pts2, "tris": tris, "dz": dz})


def cavity(n=32, jitter=0.2, seed=2603001):
    """Lid-driven cavity [0,1]^2 x [0, 1/n]: (n+1)^2 nodes, interior jitter U[-j,j]h, edge nodes
    moved only along their edge, corners fixed; each quad split by its (i,j)-(i+1,j+1) diagonal."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    I, J = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    d = rng.uniform(-jitter, jitter, size=P.shape) * h
    d[(I == 0) | (I == n), 0] = 0.0
    d[(J == 0) | (J == n), 1] = 0.0
    P = P + d

    def vid(i, j):
        return i * (n + 1) + j
    qi, qj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()
    v00, v10, v11, v01 = vid(qi, qj), vid(qi + 1, qj), vid(qi + 1, qj + 1), vid(qi, qj + 1)
    tris = np.stack([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], 1).reshape(-1, 3)

    def cls(mid):
        return np.where(np.abs(mid[:, 1] - 1.0) < 1e-12, 0, 1)
    specs = [("lid", U_FIXED, P_ZEROGRAD, -1), ("walls", U_FIXED, P_ZEROGRAD, -1),
             ("frontAndBack", U_EMPTY, P_EMPTY, -1)]
    return extruded_triangles(P, tris, h, cls, specs, name=f"cavity{n}")


def channel2d(nx, ny, length=4.0, height=1.0, jitter=0.2, seed=2603005):
    """2D channel [0,L]x[0,H] of jittered triangles extruded one layer: inlet x=0, outlet x=L, walls."""
    rng = np.random.default_rng(seed)
    gx = np.linspace(0.0, length, nx + 1)
    gy = np.linspace(0.0, height, ny + 1)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    hx, hy = length / nx, height / ny
    d = rng.uniform(-jitter, jitter, size=P.shape) * np.array([hx, hy])
    d[(I == 0) | (I == nx), 0] = 0.0
    d[(J == 0) | (J == ny), 1] = 0.0
    P = P + d

    def vid(i, j):
        return i * (ny + 1) + j
    qi, qj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()
    v00, v10, v11, v01 = vid(qi, qj), vid(qi + 1, qj), vid(qi + 1, qj + 1), vid(qi, qj + 1)
    tris = np.stack([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], 1).reshape(-1, 3)

    def cls(mid):
        return np.where(np.abs(mid[:, 0]) < 1e-12, 0, np.where(np.abs(mid[:, 0] - length) < 1e-12, 1, 2))
    specs = [("inlet", U_FIXED, P_ZEROGRAD, -1), ("outlet", U_ZEROGRAD, P_FIXED, -1),
             ("walls", U_FIXED, P_ZEROGRAD, -1), ("frontAndBack", U_EMPTY, P_EMPTY, -1)]
    return extruded_triangles(P, tris, min(hx, hy), cls, specs, name=f"channel{nx}x{ny}")


def periodic_box2d(n, half=math.pi / 2, jitter=0.2, seed=2603006):
    """Square [-half,half]^2 of jittered triangles (one layer) with one fixedValue wall patch."""
    rng = np.random.default_rng(seed)
    h = 2 * half / n
    g = np.linspace(-half, half, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    I, J = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    d = rng.uniform(-jitter, jitter, size=P.shape) * h
    d[(I == 0) | (I == n), 0] = 0.0
    d[(J == 0) | (J == n), 1] = 0.0
    P = P + d

    def vid(i, j):
        return i * (n + 1) + j
    qi, qj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()
    v00, v10, v11, v01 = vid(qi, qj), vid(qi + 1, qj), vid(qi + 1, qj + 1), vid(qi, qj + 1)
    tris = np.stack([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], 1).reshape(-1, 3)
    specs = [("walls", U_FIXED, P_ZEROGRAD, -1), ("frontAndBack", U_EMPTY, P_EMPTY, -1)]
    return extruded_triangles(P, tris, h, lambda mid: np.zeros(mid.shape[0], dtype=np.int64), specs,
                              name=f"tgbox{n}")


# ----------------------------------------------------------------------------------------------
# circular tube: 5-block butterfly section, extruded, prisms split into 3 tets each
# ----------------------------------------------------------------------------------------------

def _butterfly_section(R, a, n, m):
    """Nodes and quads of an O-grid section of radius R: inner square [-a,a]^2 with n x n quads and
    four outer blocks with n x m quads. Returns (points2[N,2], quads[Q,4], on_wall[N])."""
    pts = {}
    order = []

    def node(p):
        key = (round(p[0] * 1e12), round(p[1] * 1e12))
        if key not in pts:
            pts[key] = len(order)
            order.append(p)
        return pts[key]

    quads = []
    s = np.linspace(-a, a, n + 1)
    inner = [[node((s[i], s[j])) for j in range(n + 1)] for i in range(n + 1)]
    for i in range(n):
        for j in range(n):
            quads.append((inner[i][j], inner[i + 1][j], inner[i + 1][j + 1], inner[i][j + 1]))
    # four sides: (square edge param, outward arc)
    for side in range(4):
        ids = []
        for i in range(n + 1):
            t = -1.0 + 2.0 * i / n                         # along the side
            if side == 0:
                sq = (a, a * t)
            elif side == 1:
                sq = (-a * t, a)
            elif side == 2:
                sq = (-a, -a * t)
            else:
                sq = (a * t, -a)
            ang = math.atan2(sq[1], sq[0])
            arc = (R * math.cos(ang), R * math.sin(ang))
            col = []
            for k in range(m + 1):
                r = k / m
                p = ((1 - r) * sq[0] + r * arc[0], (1 - r) * sq[1] + r * arc[1])
                col.append(node(p) if k < m else node(arc))
            ids.append(col)
        for i in range(n):
            for k in range(m):
                quads.append((ids[i][k], ids[i + 1][k], ids[i + 1][k + 1], ids[i][k + 1]))
    P = np.array(order, dtype=np.float64)
    on_wall = np.abs(np.hypot(P[:, 0], P[:, 1]) - R) < 1e-9
    return P, np.array(quads, dtype=np.int64), on_wall


def _prisms_to_tets(bot, top):
    """Split prisms (bottom a,b,c; top a',b',c' with every top id > every bottom id) into 3 tets each,
    cutting every quad face along the diagonal through its lowest global vertex id."""
    r = np.argmin(bot, axis=1)
    idx = (r[:, None] + np.arange(3)[None, :]) % 3
    B = np.take_along_axis(bot, idx, 1)
    T = np.take_along_axis(top, idx, 1)
    a, b, c = B[:, 0], B[:, 1], B[:, 2]
    a2, b2, c2 = T[:, 0], T[:, 1], T[:, 2]
    t0 = np.stack([a, a2, b2, c2], 1)
    bl = b < c
    t1 = np.where(bl[:, None], np.stack([a, b, c, c2], 1), np.stack([a, b, c, b2], 1))
    t2 = np.where(bl[:, None], np.stack([a, b, c2, b2], 1), np.stack([a, c, c2, b2], 1))
    return np.stack([t0, t1, t2], 1).reshape(-1, 4)


def tube(n=16, m=6, layers=521, R=0.5, L=10.0, jitter=0.1, seed=2603003, outlet="p0"):
    """Straight tube along x (radius R, length L): butterfly section with inner half-width R/2,
    quads split into triangles, extruded into `layers` prism layers, each prism split into 3 tets.
    Interior nodes jittered by U[-j,j]*h_local; wall nodes move only axially, end-plane nodes only
    in-plane.  Patches: inlet (x=0), outlet (x=L), wall.  The defaults give 2,000,640 tets (3,840
    per layer, axial spacing 0.0192): finer sections (n = 20, m = 8 or n = 24, m = 10) make the PISO
    step at Re 500, dt 1e-3 unstable near the outlet within 8 to 15 steps."""
    rng = np.random.default_rng(seed)
    P2, Q, on_wall = _butterfly_section(R, 0.5 * R, n, m)
    # quads -> triangles along the diagonal through the lower node id
    lo = np.argmin(Q, axis=1)
    Qr = np.take_along_axis(Q, (lo[:, None] + np.arange(4)[None, :]) % 4, 1)
    tris = np.concatenate([Qr[:, [0, 1, 2]], Qr[:, [0, 2, 3]]])
    ns = P2.shape[0]
    xs = np.linspace(0.0, L, layers + 1)
    # local spacing per section node: shortest incident quad edge
    e = np.concatenate([Q[:, [0, 1]], Q[:, [1, 2]], Q[:, [2, 3]], Q[:, [3, 0]]])
    el = np.linalg.norm(P2[e[:, 0]] - P2[e[:, 1]], axis=1)
    hsec = np.full(ns, np.inf)
    np.minimum.at(hsec, e[:, 0], el)
    np.minimum.at(hsec, e[:, 1], el)
    hx = L / layers
    npts = ns * (layers + 1)
    Pts = np.empty((npts, 3))
    for k in range(layers + 1):
        Pts[k * ns:(k + 1) * ns, 0] = xs[k]
        Pts[k * ns:(k + 1) * ns, 1:] = P2
    if jitter > 0:
        d = rng.uniform(-jitter, jitter, size=(npts, 3))
        h = np.minimum(np.tile(hsec, layers + 1), hx)
        d *= h[:, None]
        wall = np.tile(on_wall, layers + 1)
        layer = np.repeat(np.arange(layers + 1), ns)
        end = (layer == 0) | (layer == layers)
        d[wall, 1:] = 0.0
        d[end, 0] = 0.0
        Pts = Pts + d
    nt2 = tris.shape[0]
    lay = np.arange(layers)
    bot = (tris[None, :, :] + (lay * ns)[:, None, None]).reshape(-1, 3)
    top = bot + ns
    T = _prisms_to_tets(bot, top)

    def cls(Cf, tri):
        x = Cf[:, 0]
        return np.where(np.abs(x) < 1e-9, 0, np.where(np.abs(x - L) < 1e-9, 1, 2))
    if outlet == "p0":
        specs = [("inlet", U_FIXED, P_ZEROGRAD, -1), ("outlet", U_ZEROGRAD, P_FIXED, -1),
                 ("wall", U_FIXED, P_ZEROGRAD, -1)]
    else:
        specs = [("inlet", U_FIXED, P_ZEROGRAD, -1), ("outlet", U_ZEROGRAD, P_WINDKESSEL, 0),
                 ("wall", U_FIXED, P_ZEROGRAD, -1)]
    mesh = tet_mesh(Pts, T, cls, specs, name=f"tube{n}x{m}x{layers}")
    mesh.meta.update(R=R, L=L, nt2=nt2)
    return mesh


# ----------------------------------------------------------------------------------------------
# fields and boundary values (inputs)
# ----------------------------------------------------------------------------------------------

def sinusoid_field(seed, n_modes=8, kmax=3):
    """phi(x) = sum_m a_m sin(2 pi k_m.x + t_m), a_m ~ N(0,1)/sqrt(n), k_m in {-kmax..kmax}^3 \\ 0."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(n_modes) / math.sqrt(n_modes)
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    th = rng.uniform(0.0, 2 * math.pi, n_modes)

    def f(x):
        x = np.asarray(x, dtype=np.float64)
        return (a[None, :] * np.sin(2 * math.pi * x @ ks.T + th[None, :])).sum(axis=1)
    return f


def boundary_mask(mesh, kind):
    """Per-boundary-face code for a BC table: 'u' or 'p' -> 0 fixed, 1 zeroGradient, 2 empty."""
    Fb = mesh.n_boundary_faces
    Fi = mesh.n_internal_faces
    out = np.empty(Fb, dtype=np.int32)
    for p in mesh.patches:
        s = slice(p.start - Fi, p.start - Fi + p.size)
        if kind == "u":
            out[s] = {U_FIXED: 0, U_ZEROGRAD: 1, U_EMPTY: 2}[p.u_type]
        elif kind == "p":
            out[s] = {P_FIXED: 0, P_WINDKESSEL: 0, P_ZEROGRAD: 1, P_EMPTY: 2}[p.p_type]
        else:
            raise ValueError(kind)
    return out


def parabolic_inlet(Cf_b, axis_origin, R, umax, axis=0):
    """u = umax (1 - r^2/R^2) along +axis for points Cf_b (r from the axis through axis_origin)."""
    d = Cf_b - np.asarray(axis_origin, dtype=np.float64)[None, :]
    d[:, axis] = 0.0
    r2 = np.einsum("ij,ij->i", d, d)
    u = np.zeros_like(Cf_b)
    u[:, axis] = umax * np.clip(1.0 - r2 / (R * R), 0.0, None)
    return u


def check_mesh(mesh, tol=1e-10):
    """Validity: V > 0, S.d > 0 on every non-empty face, closed cells (sum of outward S = 0)."""
    Fi = mesh.n_internal_faces
    o, nb = mesh.owner, mesh.neighbour
    if np.any(mesh.V <= 0):
        raise ValueError("non-positive volume")
    d = mesh.C[nb] - mesh.C[o[:Fi]]
    if np.any(np.einsum("ij,ij->i", mesh.Sf[:Fi], d) <= 0):
        raise ValueError("internal face with S.d <= 0")
    db = mesh.Cf[Fi:] - mesh.C[o[Fi:]]
    if np.any(np.einsum("ij,ij->i", mesh.Sf[Fi:], db) <= 0):
        raise ValueError("boundary face with S.d <= 0")
    acc = np.zeros((mesh.n_cells, 3))
    np.add.at(acc, o, mesh.Sf)
    np.add.at(acc, nb, -mesh.Sf[:Fi])
    scale = np.abs(mesh.Sf).max()
    if np.abs(acc).max() > tol * scale * 10:
        raise ValueError(f"open cell: |sum S| = {np.abs(acc).max()}")
    if np.any(nb == o[:Fi]):
        raise ValueError("neighbour == owner")
    return True


# ----------------------------------------------------------------------------------------------
# structured hexahedra under an affine map (planar parallelogram faces, no skewness)
# ----------------------------------------------------------------------------------------------

def hex_box(nx, ny, nz, A=None, origin=(0.0, 0.0, 0.0), patches="walls"):
    """Hexes of the unit box mapped by x = origin + A xi (xi in [0,1]^3).  With a sheared A the faces
    are non-orthogonal (S not parallel to d) while the line between cell centroids still passes through
    the face centroid, so linear interpolation is exact at C_f."""
    A = np.eye(3) if A is None else np.asarray(A, dtype=np.float64)
    if np.linalg.det(A) <= 0:
        raise ValueError("map must preserve orientation")
    org = np.asarray(origin, dtype=np.float64)
    n = np.array([nx, ny, nz])

    def X(i, j, k):
        xi = np.stack([i / nx, j / ny, k / nz], axis=-1)
        return org + xi @ A.T

    def cid(i, j, k):
        return (i * ny + j) * nz + k
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    C = X(I + 0.5, J + 0.5, K + 0.5)
    V = np.full(I.shape[0], np.linalg.det(A) / (nx * ny * nz))
    units = np.eye(3, dtype=np.int64)

    def faces_dir(ax, idx_lo):
        # quad with corner idx (ax fixed) spanned by the two other axes
        a1, a2 = [d for d in range(3) if d != ax]
        e1, e2 = units[a1], units[a2]
        p0 = idx_lo
        pts = [p0, p0 + e1, p0 + e1 + e2, p0 + e2]
        P = [X(p[:, 0], p[:, 1], p[:, 2]) for p in pts]
        S = 0.5 * np.cross(P[2] - P[0], P[3] - P[1])
        Cf = 0.25 * (P[0] + P[1] + P[2] + P[3])
        return S, Cf

    own_i, nbr_i, S_i, Cf_i = [], [], [], []
    own_b, S_b, Cf_b, side_b = [], [], [], []
    for ax in range(3):
        rng_ = [np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1)]
        rng_[ax] = np.arange(n[ax] + 1)
        for d in range(3):
            if d != ax:
                rng_[d] = np.arange(n[d])
        G = np.stack(np.meshgrid(*rng_, indexing="ij"), axis=-1).reshape(-1, 3)
        S, Cf = faces_dir(ax, G)
        lo_cell = G.copy()
        lo_cell[:, ax] -= 1
        hi_cell = G
        inner = (G[:, ax] > 0) & (G[:, ax] < n[ax])
        o = cid(lo_cell[inner, 0], lo_cell[inner, 1], lo_cell[inner, 2])
        nb = cid(hi_cell[inner, 0], hi_cell[inner, 1], hi_cell[inner, 2])
        own_i.append(o); nbr_i.append(nb); S_i.append(S[inner]); Cf_i.append(Cf[inner])
        lo_side = G[:, ax] == 0
        hi_side = G[:, ax] == n[ax]
        own_b.append(cid(hi_cell[lo_side, 0], hi_cell[lo_side, 1], hi_cell[lo_side, 2]))
        S_b.append(-S[lo_side]); Cf_b.append(Cf[lo_side]); side_b.append(np.full(lo_side.sum(), 2 * ax))
        own_b.append(cid(lo_cell[hi_side, 0], lo_cell[hi_side, 1], lo_cell[hi_side, 2]))
        S_b.append(S[hi_side]); Cf_b.append(Cf[hi_side]); side_b.append(np.full(hi_side.sum(), 2 * ax + 1))
    own_i, nbr_i = np.concatenate(own_i), np.concatenate(nbr_i)
    S_i, Cf_i = np.concatenate(S_i), np.concatenate(Cf_i)
    srt = np.lexsort((nbr_i, own_i))
    own_i, nbr_i, S_i, Cf_i = own_i[srt], nbr_i[srt], S_i[srt], Cf_i[srt]
    own_b, S_b, Cf_b, side_b = map(np.concatenate, (own_b, S_b, Cf_b, side_b))
    # orient every area vector out of its owner
    S_i[np.einsum("ij,ij->i", S_i, Cf_i - C[own_i]) < 0] *= -1.0
    S_b[np.einsum("ij,ij->i", S_b, Cf_b - C[own_b]) < 0] *= -1.0
    if patches == "walls":
        pid = np.zeros(own_b.shape[0], dtype=np.int64)
        specs = [("walls", U_FIXED, P_FIXED, -1)]
    elif patches == "sides":
        pid = side_b
        specs = [(nm, U_FIXED, P_FIXED, -1) for nm in ("x0", "x1", "y0", "y1", "z0", "z1")]
    else:
        # dict: side name (x0..z1) -> (patch name, u_type, p_type, wk_id); sides sharing a patch
        # name are merged, patches ordered by first appearance in x0..z1
        specs, pid_of_side = [], []
        for nm in ("x0", "x1", "y0", "y1", "z0", "z1"):
            spec = tuple(patches[nm])
            names = [q[0] for q in specs]
            if spec[0] in names:
                pid_of_side.append(names.index(spec[0]))
            else:
                specs.append(spec)
                pid_of_side.append(len(specs) - 1)
        pid = np.asarray(pid_of_side, dtype=np.int64)[side_b]
    order = np.lexsort((own_b, pid))
    own_b, S_b, Cf_b, pid = own_b[order], S_b[order], Cf_b[order], pid[order]
    Fi = own_i.shape[0]
    plist = []
    start = Fi
    for k, (pname, ut, pt, wk) in enumerate(specs):
        cnt = int(np.count_nonzero(pid == k))
        plist.append(Patch(pname, start, cnt, ut, pt, wk))
        start += cnt
    w = _weights(S_i, Cf_i, C, own_i, nbr_i)
    return Mesh(owner=np.concatenate([own_i, own_b]).astype(np.int32), neighbour=nbr_i.astype(np.int32),
                Sf=np.ascontiguousarray(np.concatenate([S_i, S_b])),
                Cf=np.ascontiguousarray(np.concatenate([Cf_i, Cf_b])), C=np.ascontiguousarray(C), V=V, w=w,
                patches=plist, name=f"hex{nx}x{ny}x{nz}")


def quad_channel(nx, ny, length, height=1.0, inlet=True):
    """2D box of orthogonal quads (one hex layer, empty front/back): inlet x0 (U fixed), outlet x1
    (U zeroGradient, p fixed), walls y0/y1 (U fixed).  inlet=False makes x0/x1 fixed-U walls too."""
    dz = min(length / nx, height / ny)
    A = np.diag([length, height, dz])
    e = ("frontAndBack", U_EMPTY, P_EMPTY, -1)
    if inlet:
        sides = {"x0": ("inlet", U_FIXED, P_ZEROGRAD, -1), "x1": ("outlet", U_ZEROGRAD, P_FIXED, -1),
                 "y0": ("walls", U_FIXED, P_ZEROGRAD, -1), "y1": ("walls", U_FIXED, P_ZEROGRAD, -1),
                 "z0": e, "z1": e}
    else:
        w = ("walls", U_FIXED, P_ZEROGRAD, -1)
        sides = {"x0": w, "x1": w, "y0": w, "y1": w, "z0": e, "z1": e}
    return hex_box(nx, ny, 1, A=A, patches=sides)


# ----------------------------------------------------------------------------------------------
# two-level bifurcating tube (voxelised union of swept tubes, Kuhn-split voxels)
# ----------------------------------------------------------------------------------------------

def _smoothstep(t):
    t = np.clip(t, 0.0, 1.0)
    return t * t * (3.0 - 2.0 * t)


def ybif_segments(r0=0.5):
    """Centre lines y(x) (z = 0) and radii: parent on [0,3]; branches A (up) and B (down) with
    lateral offsets +-1 reached over 2 length units by a smoothstep; at x = 6 branch A splits into
    A1/A2 (offsets +-0.6).  Radii follow r_child = r_parent / 2^(1/3).  All outlets lie on x = 10."""
    rA = r0 / 2 ** (1 / 3)
    rA1 = rA / 2 ** (1 / 3)
    yA = lambda x: 1.0 * _smoothstep((x - 3.0) / 2.0)
    yB = lambda x: -1.0 * _smoothstep((x - 3.0) / 2.0)
    yA1 = lambda x: 1.0 + 0.6 * _smoothstep((x - 6.0) / 2.0)
    yA2 = lambda x: 1.0 - 0.6 * _smoothstep((x - 6.0) / 2.0)
    # (name, x range, centre line, radius); ranges overlap a little so the union is connected
    return [("parent", (0.0, 3.4), lambda x: 0.0 * x, r0), ("A", (3.0, 6.3), yA, rA), ("B", (3.0, 10.0), yB, rA),
            ("A1", (6.0, 10.0), yA1, rA1), ("A2", (6.0, 10.0), yA2, rA1)]


def ybif(h=None, target_cells=400_000, jitter=0.15, seed=2603004, L=10.0):
    """Bifurcating tube: voxels of size h whose centre lies in the union of the swept tubes, each
    voxel split into 6 Kuhn tets, largest connected component kept; interior nodes jittered by
    U[-j,j]h.  Patches: inlet (x=0), outlets A1, A2, B (x=L, Windkessel 0,1,2), wall (staircase)."""
    from scipy import ndimage
    segs = ybif_segments()
    lo = np.array([0.0, -1.6, -0.55])
    hi = np.array([L, 1.9, 0.55])

    def mask_for(hh):
        n = np.maximum(1, np.round((hi - lo) / hh).astype(int))
        hx = (hi - lo) / n
        xc = lo[0] + (np.arange(n[0]) + 0.5) * hx[0]
        yc = lo[1] + (np.arange(n[1]) + 0.5) * hx[1]
        zc = lo[2] + (np.arange(n[2]) + 0.5) * hx[2]
        X, Y, Z = np.meshgrid(xc, yc, zc, indexing="ij")
        inside = np.zeros(X.shape, dtype=bool)
        for _, (x0, x1), yfun, r in segs:
            sel = (X >= x0) & (X <= x1)
            inside |= sel & ((Y - yfun(X)) ** 2 + Z ** 2 <= r * r)
        lab, nl = ndimage.label(inside)
        if nl > 1:
            sizes = ndimage.sum(inside, lab, index=np.arange(1, nl + 1))
            inside = lab == (1 + int(np.argmax(sizes)))
        return inside, n, hx

    if h is None:
        # bisection on h for the target cell count (6 tets per voxel)
        a, b = 0.01, 0.2
        for _ in range(30):
            mid = 0.5 * (a + b)
            cnt = 6 * int(mask_for(mid)[0].sum())
            if cnt > target_cells:
                a = mid
            else:
                b = mid
        h = b
    inside, n, hx = mask_for(h)
    idx = np.argwhere(inside)
    # nodes of kept voxels
    def vid(i, j, k):
        return (i * (n[1] + 1) + j) * (n[2] + 1) + k
    corners = []
    for perm in _KUHN_PERMS:
        cur = idx.copy()
        vs = [vid(cur[:, 0], cur[:, 1], cur[:, 2])]
        for ax in perm:
            cur = cur.copy()
            cur[:, ax] += 1
            vs.append(vid(cur[:, 0], cur[:, 1], cur[:, 2]))
        corners.append(np.stack(vs, axis=1))
    T = np.stack(corners, axis=1).reshape(-1, 4)
    used, Tc = np.unique(T, return_inverse=True)
    Tc = Tc.reshape(T.shape)
    I = used // ((n[1] + 1) * (n[2] + 1))
    J = (used // (n[2] + 1)) % (n[1] + 1)
    K = used % (n[2] + 1)
    P = lo[None, :] + np.stack([I, J, K], 1) * hx[None, :]
    # boundary nodes: nodes of faces with one adjacent kept voxel -> find via face extraction on the
    # un-jittered mesh; jitter only the others
    own_i, nbr_i, tri_i, own_b, tri_b = _tet_faces(P, Tc)
    on_bnd = np.zeros(P.shape[0], dtype=bool)
    on_bnd[np.unique(tri_b)] = True
    rng = np.random.default_rng(seed)
    d = rng.uniform(-jitter, jitter, size=P.shape) * hx[None, :]
    d[on_bnd] = 0.0
    P = P + d
    tol = 1e-9 * L

    def cls(Cf, tri):
        x, y = Cf[:, 0], Cf[:, 1]
        out = np.full(Cf.shape[0], 4, dtype=np.int64)          # wall
        out[np.abs(x) < tol] = 0                                # inlet
        at_out = np.abs(x - L) < tol
        out[at_out & (y > 1.3)] = 1                             # A1 (centre y = 1.6)
        out[at_out & (y <= 1.3) & (y > -0.2)] = 2               # A2 (centre y = 0.4)
        out[at_out & (y <= -0.2)] = 3                           # B  (centre y = -1.0)
        return out
    specs = [("inlet", U_FIXED, P_ZEROGRAD, -1), ("A1", U_ZEROGRAD, P_WINDKESSEL, 0),
             ("A2", U_ZEROGRAD, P_WINDKESSEL, 1), ("B", U_ZEROGRAD, P_WINDKESSEL, 2),
             ("wall", U_FIXED, P_ZEROGRAD, -1)]
    mesh = tet_mesh(P, Tc, cls, specs, name=f"ybif_h{h:.4f}")
    mesh.meta.update(h=float(h), L=L, R=0.5, segments=[(s[0], s[3]) for s in segs])
    return mesh


def windkessel_nominal(mesh, q_in, tau=0.1, outlets=("A1", "A2", "B")):
    """Nominal RCR per outlet: flow split by outlet area, Rd = 1/Q_ref, Rp = Rd/9, C = tau/Rd."""
    areas = np.array([np.linalg.norm(mesh.Sf[mesh.patch(o).start:mesh.patch(o).start + mesh.patch(o).size], axis=1).sum()
                      for o in outlets])
    q = q_in * areas / areas.sum()
    Rd = 1.0 / q
    return np.stack([Rd / 9.0, tau / Rd, Rd], 1)


# ----------------------------------------------------------------------------------------------
# batched form: several meshes packed block-diagonally into one
# ----------------------------------------------------------------------------------------------

def pack(meshes, name="packed"):
    """One mesh holding the given meshes side by side: cells and internal faces concatenated, then
    every member's boundary block in member order (its patches keep their order, named "k/name",
    Windkessel ids shifted past the previous members').  Returns (mesh, seg_cell_start) with
    seg_cell_start[k] the first cell of member k and seg_cell_start[-1] = total cells; the offsets of
    each member's cells, internal faces, boundary faces and Windkessel ids are in mesh.meta["members"]."""
    nc = [m.n_cells for m in meshes]
    nfi = [m.n_internal_faces for m in meshes]
    nfb = [m.n_boundary_faces for m in meshes]
    c0 = np.concatenate([[0], np.cumsum(nc)]).astype(np.int64)
    fi0 = np.concatenate([[0], np.cumsum(nfi)]).astype(np.int64)
    fb0 = np.concatenate([[0], np.cumsum(nfb)]).astype(np.int64)
    Fi = int(fi0[-1])
    own_i, nbr, own_b, S_i, S_b, Cf_i, Cf_b, w, patches, members = [], [], [], [], [], [], [], [], [], []
    wk0 = 0
    for k, m in enumerate(meshes):
        fi = m.n_internal_faces
        own_i.append(m.owner[:fi] + c0[k])
        nbr.append(m.neighbour + c0[k])
        own_b.append(m.owner[fi:] + c0[k])
        S_i.append(m.Sf[:fi])
        S_b.append(m.Sf[fi:])
        Cf_i.append(m.Cf[:fi])
        Cf_b.append(m.Cf[fi:])
        w.append(m.w)
        n_wk = 0
        for p in m.patches:
            wk = p.wk_id + wk0 if p.wk_id >= 0 else -1
            n_wk = max(n_wk, p.wk_id + 1)
            patches.append(Patch(f"{k}/{p.name}", Fi + int(fb0[k]) + (p.start - fi), p.size, p.u_type, p.p_type, wk))
        members.append(dict(cell_start=int(c0[k]), n_cells=nc[k], face_start=int(fi0[k]), n_internal_faces=fi,
                            bface_start=Fi + int(fb0[k]), n_boundary_faces=nfb[k], wk_start=wk0, n_windkessel=n_wk))
        wk0 += n_wk
    out = Mesh(owner=np.concatenate(own_i + own_b).astype(np.int32), neighbour=np.concatenate(nbr).astype(np.int32),
               Sf=np.concatenate(S_i + S_b), Cf=np.concatenate(Cf_i + Cf_b), C=np.concatenate([m.C for m in meshes]),
               V=np.concatenate([m.V for m in meshes]), w=np.concatenate(w), patches=patches, name=name,
               meta=dict(members=members))
    return out, c0.astype(np.int32)


def member_faces(packed, k):
    """Face indices (in the packed mesh) of member k, in the member's own face order."""
    mb = packed.meta["members"][k]
    return np.concatenate([np.arange(mb["face_start"], mb["face_start"] + mb["n_internal_faces"]),
                           np.arange(mb["bface_start"], mb["bface_start"] + mb["n_boundary_faces"])])


def inlet_flow(mesh, Ub, patch="inlet"):
    """Volume flow entering through a patch for boundary velocities Ub[Fb, 3] (positive inwards)."""
    p = mesh.patch(patch)
    s = slice(p.start - mesh.n_internal_faces, p.start - mesh.n_internal_faces + p.size)
    return -float((Ub[s] * mesh.Sf[p.start:p.start + p.size]).sum())


def box_channel_inlet(mesh, umax=1.0):
    """Ub with u_x = 16 umax y(1-y) z(1-z) on the inlet of a unit-box channel, zero elsewhere."""
    Ub = np.zeros((mesh.n_boundary_faces, 3))
    p = mesh.patch("inlet")
    c = mesh.Cf[p.start:p.start + p.size]
    Ub[p.start - mesh.n_internal_faces:p.start - mesh.n_internal_faces + p.size, 0] = \
        16 * umax * c[:, 1] * (1 - c[:, 1]) * c[:, 2] * (1 - c[:, 2])
    return Ub


def batch_members(n_members=64, seed0=2603100, n_lo=2e4, n_hi=3e5):
    """Members of the many-mesh batch.  Member k draws from seed seed0+k: a target size
    N = exp(U[ln n_lo, ln n_hi]) cells, a Reynolds number U[100, 800] and Windkessel factors
    U[0.5, 2]^3 on the nominal RCR.  Even k: a straight tube (butterfly section 8 x 4, 1152 tets per
    layer, axial spacing 0.05, parabolic inlet u_max = 1, Re on the mean velocity and D = 1); odd k: a
    unit-box Kuhn channel (inlet 16 y(1-y) z(1-z), Re on u_max and the unit length).  Each has one
    Windkessel outlet.  Returns dicts with mesh, nu, Ub, wk [1, 3], pc0 [1]."""
    out = []
    for k in range(n_members):
        rng = np.random.default_rng(seed0 + k)
        N = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        Re = float(rng.uniform(100.0, 800.0))
        fac = rng.uniform(0.5, 2.0, 3)
        if k % 2 == 0:
            layers = max(4, int(round(N / 1152)))
            m = tube(n=8, m=4, layers=layers, R=0.5, L=0.05 * layers, seed=seed0 + k, outlet="wk")
            Ub = np.zeros((m.n_boundary_faces, 3))
            p = m.patch("inlet")
            s = slice(p.start - m.n_internal_faces, p.start - m.n_internal_faces + p.size)
            Ub[s] = parabolic_inlet(m.Cf[p.start:p.start + p.size], (0.0, 0.0, 0.0), 0.5, 1.0)
            nu = 0.5 * 1.0 / Re
        else:
            nb = max(4, int(round((N / 6.0) ** (1.0 / 3.0))))
            m = kuhn_cube(nb, jitter=0.15, patches="channel", seed=seed0 + k)
            Ub = box_channel_inlet(m)
            nu = 1.0 / Re
        wk = windkessel_nominal(m, inlet_flow(m, Ub), outlets=("outlet",)) * fac[None, :]
        m.name = f"member{k}:{m.name}"
        out.append(dict(mesh=m, nu=nu, Ub=Ub, wk=wk, pc0=np.zeros(1), Re=Re))
    return out


# ----------------------------------------------------------------------------------------------
# manufactured Poisson solution on the unit cube (inputs of the Poisson verification workload)
# ----------------------------------------------------------------------------------------------

def poisson_mms_solution(x):
    """phi(x) = 2 sin(pi x) (y^4 - y) sin(2 pi z) + 10 (the paper's 3D Poisson verification field)."""
    return 2 * np.sin(math.pi * x[:, 0]) * (x[:, 1] ** 4 - x[:, 1]) * np.sin(2 * math.pi * x[:, 2]) + 10.0


def poisson_mms_source(x):
    """f = lap(phi) of poisson_mms_solution."""
    s = np.sin(math.pi * x[:, 0]) * np.sin(2 * math.pi * x[:, 2])
    return -10 * math.pi ** 2 * s * (x[:, 1] ** 4 - x[:, 1]) + 24 * s * x[:, 1] ** 2


def poisson_mms_gradient(x):
    """grad(phi) of poisson_mms_solution, [n, 3]."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    pi = math.pi
    return np.stack([2 * pi * np.cos(pi * X) * (Y ** 4 - Y) * np.sin(2 * pi * Z),
                     2 * np.sin(pi * X) * (4 * Y ** 3 - 1) * np.sin(2 * pi * Z),
                     4 * pi * np.sin(pi * X) * (Y ** 4 - Y) * np.cos(2 * pi * Z)], 1)
