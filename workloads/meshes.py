"""Seeded simplex meshes for the plane channel and the straight pipe.

Conventions shared by every consumer of these meshes:

* ``xyz``   float64 [nv, d]       vertex coordinates (locality-ordered).
* ``cells`` int32   [nc, d+1]     linear simplices (orientation arbitrary).
* ``bfaces`` int32  [nf, d]       boundary facets, ordered so the facet normal
  points out of the domain: in 2D the domain lies to the left of a->b; in 3D
  (b-a) x (c-a) points outward.
* ``btags`` int32   [nf]          1 = inlet, 2 = outlet, 3 = wall.
* ``curved_edges`` int32 [ncv, 2] and ``curved_xyz`` float64 [ncv, d]: wall
  edges whose quadratic midside node is moved onto the true curved boundary
  (the straight midpoint projected radially); every other edge keeps its
  midpoint. Both arrays are empty for straight-walled domains.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import Delaunay
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import reverse_cuthill_mckee

INLET, OUTLET, WALL = 1, 2, 3


@dataclass
class Mesh:
    dim: int
    xyz: np.ndarray
    cells: np.ndarray
    bfaces: np.ndarray
    btags: np.ndarray
    curved_edges: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    curved_xyz: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    name: str = ""

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nc(self) -> int:
        return int(self.cells.shape[0])


def channel_mesh(nx: int = 32, ny: int = 8, length: float = 4.0, height: float = 1.0) -> Mesh:
    """Structured channel [0,length]x[0,height]; each quad split along the
    (i,j)->(i+1,j+1) diagonal. Vertex v = j*(nx+1) + i."""
    xs = np.linspace(0.0, length, nx + 1)
    ys = np.linspace(0.0, height, ny + 1)
    X, Y = np.meshgrid(xs, ys)  # [ny+1, nx+1]
    xyz = np.stack([X.ravel(), Y.ravel()], 1).astype(np.float64)
    vid = np.arange((nx + 1) * (ny + 1), dtype=np.int64).reshape(ny + 1, nx + 1)
    v00 = vid[:-1, :-1].ravel()
    v10 = vid[:-1, 1:].ravel()
    v01 = vid[1:, :-1].ravel()
    v11 = vid[1:, 1:].ravel()
    tri = np.empty((2 * nx * ny, 3), np.int64)
    tri[0::2] = np.stack([v00, v10, v11], 1)
    tri[1::2] = np.stack([v00, v11, v01], 1)
    faces, tags = [], []
    for i in range(nx):  # bottom wall, left to right
        faces.append((vid[0, i], vid[0, i + 1])); tags.append(WALL)
    for j in range(ny):  # outlet x = length, upward
        faces.append((vid[j, nx], vid[j + 1, nx])); tags.append(OUTLET)
    for i in range(nx, 0, -1):  # top wall, right to left
        faces.append((vid[ny, i], vid[ny, i - 1])); tags.append(WALL)
    for j in range(ny, 0, -1):  # inlet x = 0, downward
        faces.append((vid[j, 0], vid[j - 1, 0])); tags.append(INLET)
    return Mesh(2, xyz, tri.astype(np.int32), np.array(faces, np.int32),
                np.array(tags, np.int32), np.zeros((0, 2), np.int32), np.zeros((0, 2)),
                name=f"channel{nx}x{ny}")


def _disk_points(h: float, radius: float, rng: np.random.Generator) -> np.ndarray:
    """Concentric rings of spacing ~h with seeded angular offsets and a small
    radial jitter on interior rings; the outer ring lies exactly on r=radius."""
    nr = max(1, int(round(radius / h)))
    pts = [np.zeros((1, 2))]
    for i in range(1, nr + 1):
        r = radius * i / nr
        n = max(6, int(round(2.0 * np.pi * r / h)))
        th = rng.uniform(0.0, 2.0 * np.pi / n) + 2.0 * np.pi * np.arange(n) / n
        if i < nr:
            r = r + rng.uniform(-0.12, 0.12, n) * (radius / nr)
            th = th + rng.uniform(-0.12, 0.12, n) * (2.0 * np.pi / n)
        else:
            r = np.full(n, radius)
        pts.append(np.stack([r * np.cos(th), r * np.sin(th)], 1))
    return np.concatenate(pts, 0)


# Prism (bottom 0,1,2; top 3,4,5 with 3 above 0) relabelings that move any
# vertex to position 0 while keeping the vertical pairs.
_PRISM_ROT = np.array([[0, 1, 2, 3, 4, 5], [1, 2, 0, 4, 5, 3], [2, 0, 1, 5, 3, 4],
                       [3, 5, 4, 0, 2, 1], [4, 3, 5, 1, 0, 2], [5, 4, 3, 2, 1, 0]])


def _split_prisms(P: np.ndarray) -> np.ndarray:
    """Split prisms [n,6] into 3 tets each. Every quadrilateral side is cut
    along the diagonal through its smallest global vertex index, so prisms
    that share a side cut it the same way (conforming tetrahedralization)."""
    m = np.argmin(P, 1)
    V = np.take_along_axis(P, _PRISM_ROT[m], 1)
    use15 = np.minimum(V[:, 1], V[:, 5]) < np.minimum(V[:, 2], V[:, 4])
    t = np.empty((P.shape[0], 3, 4), P.dtype)
    a = [[0, 1, 2, 5], [0, 1, 5, 4], [0, 4, 5, 3]]
    b = [[0, 1, 2, 4], [0, 4, 2, 5], [0, 4, 5, 3]]
    for k in range(3):
        t[:, k] = np.where(use15[:, None], V[:, a[k]], V[:, b[k]])
    return t.reshape(-1, 4)


def _boundary_faces_3d(cells: np.ndarray, xyz: np.ndarray):
    """Facets used by exactly one tet, oriented outward."""
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    f = cells[:, loc].reshape(-1, 3).astype(np.int64)
    opp = cells[:, [0, 1, 2, 3]].reshape(-1)
    fs = np.sort(f, 1)
    nv = xyz.shape[0]
    key = (fs[:, 0] * nv + fs[:, 1]) * nv + fs[:, 2]
    _, idx, cnt = np.unique(key, return_index=True, return_counts=True)
    sel = idx[cnt == 1]
    F = f[sel]
    o = opp[sel]
    a, b, c = xyz[F[:, 0]], xyz[F[:, 1]], xyz[F[:, 2]]
    nrm = np.cross(b - a, c - a)
    inward = np.einsum("ij,ij->i", nrm, xyz[o] - a) > 0
    F[inward] = F[inward][:, [0, 2, 1]]
    return F


def pipe_mesh(h: float, radius: float = 1.0, length: float = 10.0, seed: int = 102,
              curved: bool = True) -> Mesh:
    """Straight pipe along z, r <= radius, 0 <= z <= length.

    The cross-section is a seeded 2D Delaunay triangulation of jittered
    concentric rings (outer ring exactly on the circle), extruded through
    seeded layers; each prism is split into 3 tets. Vertices are numbered
    layer by layer, with the in-layer order from reverse Cuthill-McKee, so
    that P2 neighbours sit close in memory."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = _disk_points(h, radius, rng)
    tri = Delaunay(pts).simplices.astype(np.int64)
    # locality order inside one layer
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [0, 2]]], 0)
    n2 = pts.shape[0]
    adj = coo_matrix((np.ones(e.shape[0]), (e[:, 0], e[:, 1])), shape=(n2, n2)).tocsr()
    adj = adj + adj.T
    perm = reverse_cuthill_mckee(adj.tocsr(), symmetric_mode=True)
    inv = np.empty(n2, np.int64)
    inv[perm] = np.arange(n2)
    pts = pts[perm]
    tri = inv[tri]
    nz = max(1, int(round(length / h)))
    z = length * np.arange(nz + 1) / nz
    if nz > 1:
        z[1:-1] += rng.uniform(-0.15, 0.15, nz - 1) * (length / nz)
    xyz = np.concatenate([np.concatenate([pts, np.full((n2, 1), zk)], 1) for zk in z], 0)
    prisms = []
    for k in range(nz):
        lo, hi = k * n2, (k + 1) * n2
        prisms.append(np.concatenate([tri + lo, tri + hi], 1))
    P = np.concatenate(prisms, 0)
    cells = _split_prisms(P)
    F = _boundary_faces_3d(cells, xyz)
    zf = xyz[F][:, :, 2]
    tags = np.full(F.shape[0], WALL, np.int32)
    tags[np.all(zf == 0.0, 1)] = INLET
    tags[np.all(zf == length, 1)] = OUTLET
    ce = np.zeros((0, 2), np.int32)
    cx = np.zeros((0, 3))
    if curved:
        W = F[tags == WALL]
        we = np.concatenate([W[:, [0, 1]], W[:, [1, 2]], W[:, [0, 2]]], 0)
        we = np.unique(np.sort(we, 1), axis=0)
        mid = 0.5 * (xyz[we[:, 0]] + xyz[we[:, 1]])
        r = np.hypot(mid[:, 0], mid[:, 1])
        mid[:, :2] *= (radius / r)[:, None]
        ce = we.astype(np.int32)
        cx = mid
    return Mesh(3, xyz, cells.astype(np.int32), F.astype(np.int32), tags, ce, cx,
                name=f"pipe_h{h:g}_L{length:g}")


def pipe_tet_count(h: float, radius: float = 1.0, length: float = 10.0, seed: int = 102) -> int:
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = _disk_points(h, radius, rng)
    ntri = Delaunay(pts).simplices.shape[0]
    return 3 * ntri * max(1, int(round(length / h)))


def pipe_mesh_for_tets(n_tets: int, radius: float = 1.0, length: float = 10.0,
                       seed: int = 102, curved: bool = True) -> Mesh:
    """Pipe mesh whose tet count is the closest found to ``n_tets``."""
    lo, hi = 0.01, 2.0
    for _ in range(40):
        mid = np.sqrt(lo * hi)
        if pipe_tet_count(mid, radius, length, seed) > n_tets:
            lo = mid
        else:
            hi = mid
    best = min((lo, hi), key=lambda hh: abs(pipe_tet_count(hh, radius, length, seed) - n_tets))
    return pipe_mesh(best, radius, length, seed, curved)


def p2_node_coords(mesh: Mesh, edges: np.ndarray) -> np.ndarray:
    """Coordinates of all quadratic nodes given a canonical edge list: vertices
    first, then one node per edge (curved override or straight midpoint)."""
    mid = 0.5 * (mesh.xyz[edges[:, 0]] + mesh.xyz[edges[:, 1]])
    if mesh.curved_edges.shape[0]:
        nv = mesh.nv
        key = edges[:, 0].astype(np.int64) * nv + edges[:, 1]
        ck = np.sort(mesh.curved_edges, 1).astype(np.int64)
        ckey = ck[:, 0] * nv + ck[:, 1]
        pos = np.searchsorted(key, ckey)
        assert np.all(key[pos] == ckey)
        mid[pos] = mesh.curved_xyz
    return np.concatenate([mesh.xyz, mid], 0)
