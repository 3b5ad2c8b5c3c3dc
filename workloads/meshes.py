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


# ---- vessel networks: unions of cylinders, voxelized and split into tets ----

def _capped_cylinder_sdf(P: np.ndarray, a: np.ndarray, b: np.ndarray, r: float) -> np.ndarray:
    """Negative inside the finite cylinder with axis a->b, radius r and flat caps."""
    ab = b - a
    L = float(np.linalg.norm(ab))
    u = ab / L
    t = (P - a) @ u
    radial = np.linalg.norm(P - a - t[:, None] * u, axis=1)
    return np.maximum(radial - r, np.maximum(-t, t - L))


# the six tets of the Kuhn split of a hex (corner bits x=1, y=2, z=4): every hex
# uses the same 0-7 diagonal, so neighbouring hexes split their shared faces alike
_KUHN = []
for _p in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
    _c0, _c1 = 1 << _p[0], (1 << _p[0]) | (1 << _p[1])
    _KUHN.append((0, _c0, _c1, 7))
_KUHN = np.array(_KUHN)


def _inside_grid(segments, h: float):
    """Boolean grid of the cubes (side h) whose centre lies inside the union of
    capped cylinders and junction spheres; returns (inside, origin). Each
    segment is evaluated only on the sub-grid of its own bounding box."""
    lo = np.min([np.minimum(s["a"], s["b"]) - s["r"] for s in segments], 0) - h
    hi = np.max([np.maximum(s["a"], s["b"]) + s["r"] for s in segments], 0) + h
    lo[2] = 0.0  # the inlet starts on z = 0
    n = np.ceil((hi - lo) / h).astype(int)
    inside = np.zeros(n, bool)
    for s in segments:
        a, b, r = np.asarray(s["a"], float), np.asarray(s["b"], float), float(s["r"])
        shapes = [("cyl", a, b)]
        for end, pt in (("a", a), ("b", b)):
            if s.get(end + "_role", "inner") == "inner":
                shapes.append(("sph", pt, pt))
        for kind, p0, p1 in shapes:
            blo = np.maximum(np.floor((np.minimum(p0, p1) - r - lo) / h).astype(int) - 1, 0)
            bhi = np.minimum(np.ceil((np.maximum(p0, p1) + r - lo) / h).astype(int) + 1, n)
            if np.any(bhi <= blo):
                continue
            ax = [lo[d] + h * (np.arange(blo[d], bhi[d]) + 0.5) for d in range(3)]
            X, Y, Z = np.meshgrid(*ax, indexing="ij")
            P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
            if kind == "cyl":
                f = _capped_cylinder_sdf(P, p0, p1, r)
            else:
                f = np.linalg.norm(P - p0, axis=1) - r
            sub = inside[blo[0]:bhi[0], blo[1]:bhi[1], blo[2]:bhi[2]]
            sub |= (f < 0.0).reshape(sub.shape)
    return inside, lo


# cube faces in corner bits (x=1, y=2, z=4): (axis, side, the four corners in the order
# min, a, max, b around the face). With the Kuhn split every face is cut along its
# min-max diagonal, so its two boundary triangles are (min, a, max) and (min, max, b).
_CUBE_FACES = []
for _ax in range(3):
    _o = [d for d in range(3) if d != _ax]
    for _side in (0, 1):
        _base = _side << _ax
        _c = [_base, _base | (1 << _o[0]), _base | (1 << _o[0]) | (1 << _o[1]), _base | (1 << _o[1])]
        _CUBE_FACES.append((_ax, _side, _c))


def _morton3(i, j, k) -> np.ndarray:
    """Z-order (Morton) keys of non-negative 3D grid indices below 2^21: the
    bits of i, j and k interleaved, i's bit b going to bit 3b + 2."""
    i, j, k = (np.asarray(a, np.int64) for a in (i, j, k))
    key = np.zeros(i.shape, np.int64)
    for b in range(21):
        key |= (((i >> b) & 1) << (3 * b + 2)) | (((j >> b) & 1) << (3 * b + 1)) | (((k >> b) & 1) << (3 * b))
    return key


def vessel_mesh(segments, h: float, name: str, order: str = "morton"):
    """Tet mesh of a union of cylinders. ``segments`` is a list of dicts with
    keys a, b (axis end points), r (radius) and role ('inlet', 'outlet' or
    'inner'); inner end points get a junction sphere of the segment's radius.

    The bounding box is cut into cubes of side h (the plane z = 0 is a grid
    plane, so an inlet segment starting on it has a flat inlet); a cube is kept
    when its centre lies inside the union, only the largest face-connected set
    of cubes is kept, and each cube is split into six tets along one diagonal,
    which makes the mesh conforming. The boundary facets are the cube faces
    between a kept and a dropped cube, two triangles each, along the diagonal
    the split uses. Tags: 1 = inlet (facets on the inlet segment's start
    plane), 2 + k = outlet of the k-th outlet segment (facets within one cube
    of its end plane), 3 is never used for outlets; walls are tag 3 and
    outlets are numbered from 4 when there are several.

    ``order`` numbers cubes (hence cells) and vertices: "morton" along the
    Z-order curve of their grid indices, so that consecutive vertex (and edge)
    numbers lie close together in space, as a mesh renumbering pass would
    leave them; "lex" in lexicographic grid order."""
    from scipy.ndimage import label
    inside, pts_lo = _inside_grid(segments, h)
    n = np.array(inside.shape)
    lab, nlab = label(inside)  # face connectivity (6-neighbourhood)
    sizes = np.bincount(lab.ravel())
    sizes[0] = 0
    keep = lab == np.argmax(sizes)
    del lab
    hi, hj, hk = np.nonzero(keep)
    if order == "morton":  # cubes along the Z-order curve of their grid index
        o = np.argsort(_morton3(hi, hj, hk), kind="stable")
        hi, hj, hk = hi[o], hj[o], hk[o]
    # corner vertex ids on the (n+1)^3 grid, compacted
    nn = n + 1
    corners = np.stack([((hi + ((c >> 0) & 1)) * nn[1] + hj + ((c >> 1) & 1)) * nn[2] + hk + ((c >> 2) & 1)
                        for c in range(8)], 1).astype(np.int64)
    used, inv = np.unique(corners, return_inverse=True)
    gi = used // (nn[1] * nn[2])
    gj = (used // nn[2]) % nn[1]
    gk = used % nn[2]
    if order == "morton":  # renumber the vertices along the same curve
        o = np.argsort(_morton3(gi, gj, gk), kind="stable")
        rank = np.empty_like(o)
        rank[o] = np.arange(o.size)
        inv = rank[inv]
        gi, gj, gk = gi[o], gj[o], gk[o]
    corners = inv.reshape(corners.shape)
    xyz = pts_lo + h * np.stack([gi, gj, gk], 1).astype(float)
    cells = corners[:, _KUHN].reshape(-1, 4)
    # boundary facets: faces towards a dropped (or outside) cube, oriented outward
    pad = np.zeros(n + 2, bool)
    pad[1:-1, 1:-1, 1:-1] = keep
    F = []
    for ax, side, c in _CUBE_FACES:
        off = [0, 0, 0]
        off[ax] = 1 if side else -1
        nb = pad[1 + off[0] + hi, 1 + off[1] + hj, 1 + off[2] + hk]
        sel = ~nb
        q = corners[sel][:, c]  # [m, 4]: min, a, max, b
        t1 = q[:, [0, 1, 2]]
        t2 = q[:, [0, 2, 3]]
        F.append(np.concatenate([t1, t2], 0))
    F = np.concatenate(F, 0)
    # outward orientation from the geometry (the cube centre lies inside)
    a, b, cc = xyz[F[:, 0]], xyz[F[:, 1]], xyz[F[:, 2]]
    nrm = np.cross(b - a, cc - a)
    mid = (a + b + cc) / 3.0
    # the cube a facet came from: its centre is half a cube behind the facet
    cen_all = []
    for ax, side, c in _CUBE_FACES:
        off = np.zeros(3)
        off[ax] = 1 if side else -1
        nb = pad[1 + int(off[0]) + hi, 1 + int(off[1]) + hj, 1 + int(off[2]) + hk]
        m = int(np.count_nonzero(~nb))
        cen_all.append(np.repeat(-off[None, :], 2 * m, 0))
    back = np.concatenate(cen_all, 0)  # points from the facet into its cube
    inward = np.einsum("ij,ij->i", nrm, back) > 0
    F[inward] = F[inward][:, [0, 2, 1]]
    tags = np.full(F.shape[0], WALL, np.int32)
    fx = xyz[F]  # [nf, 3, 3]
    outs = [s for s in segments if s["role"] == "outlet"]
    for k, s in enumerate(outs):
        a, b = np.asarray(s["a"], float), np.asarray(s["b"], float)
        u = (b - a) / np.linalg.norm(b - a)
        t = (fx - b) @ u
        radial = np.linalg.norm(fx - b - t[..., None] * u, axis=2)
        sel = np.all(t >= -h, 1) & np.all(radial <= s["r"] + h, 1)
        tags[sel] = OUTLET if len(outs) == 1 else 4 + k
    inl = [s for s in segments if s["role"] == "inlet"][0]
    tags[np.all(fx[:, :, 2] == 0.0, 1) & np.all(np.hypot(fx[:, :, 0] - inl["a"][0], fx[:, :, 1] - inl["a"][1])
                                                <= inl["r"] + h, 1)] = INLET
    return Mesh(3, xyz, cells.astype(np.int32), F.astype(np.int32), tags, name=name)


def _rot(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation matrix about a unit axis (Rodrigues)."""
    ax = axis / np.linalg.norm(axis)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


def vessel_tree_segments(generations: int, radius: float = 1.0, ratio: float = 1.0 / np.sqrt(2.0),
                         half_angle: float = np.pi / 6, length_factor: float = 6.0):
    """Segments of a symmetric bifurcating tree rooted at the origin along +z.
    Each segment is length_factor times its radius long; daughters leave at
    +-half_angle from the parent axis (the angle between them is 2 half_angle),
    in a plane turned 90 degrees about the parent axis at every generation;
    daughter radius = parent radius * ratio. generations = 1 is a Y-bifurcation."""
    segs = []
    root = dict(a=np.zeros(3), b=np.array([0.0, 0.0, length_factor * radius]), r=radius)
    root["a_role"] = "inlet"
    frontier = [(root, np.array([1.0, 0.0, 0.0]))]  # segment and the normal of its branching plane
    segs.append(root)
    for g in range(generations):
        nxt = []
        for s, nrm in frontier:
            u = (s["b"] - s["a"]) / np.linalg.norm(s["b"] - s["a"])
            r = s["r"] * ratio
            bend = np.cross(nrm, u)  # in-plane direction perpendicular to the axis
            for sign in (1.0, -1.0):
                d = _rot(np.cross(u, bend), sign * half_angle) @ u
                c = dict(a=s["b"].copy(), b=s["b"] + length_factor * r * d, r=r)
                segs.append(c)
                nxt.append((c, _rot(d, np.pi / 2) @ nrm))
        frontier = nxt
    children = {id(s): False for s in segs}
    for s in segs:
        for t in segs:
            if t is not s and np.allclose(t["a"], s["b"]):
                children[id(s)] = True
    for s in segs:
        if s.get("a_role") == "inlet":
            s["role"] = "inlet"
        elif not children[id(s)]:
            s["role"] = "outlet"
            s["b_role"] = "outlet"
        else:
            s["role"] = "inner"
        if s["role"] == "inlet":
            s["b_role"] = "inner"
    return segs


def y_bifurcation_mesh(h: float, radii=(1.0, 0.7, 0.7)) -> Mesh:
    """Y-bifurcation: root radius radii[0], daughters radii[1], radii[2], 60 degrees between them."""
    segs = vessel_tree_segments(1, radii[0], 1.0)
    for s, r in zip(segs[1:], radii[1:]):
        u = (s["b"] - s["a"]) / np.linalg.norm(s["b"] - s["a"])
        s["r"] = r
        s["b"] = s["a"] + 6.0 * r * u
    return vessel_mesh(segs, h, f"ybif_h{h:g}")


def vessel_tree_mesh(h: float, generations: int = 3) -> Mesh:
    return vessel_mesh(vessel_tree_segments(generations), h, f"tree{generations}_h{h:g}")


def _h_for_tets(make, n_tets: int, h0: float) -> float:
    """Cube side h for about n_tets tets: one trial mesh at h0, then the count
    scales as h^-3 (the domain volume is fixed)."""
    trial = make(h0)
    return h0 * (trial.nc / float(n_tets)) ** (1.0 / 3.0)


def y_bifurcation_mesh_for_tets(n_tets: int) -> Mesh:
    """Y-bifurcation (radii 1.0/0.7/0.7) with about n_tets tets."""
    h = _h_for_tets(y_bifurcation_mesh, n_tets, 0.1)
    m = y_bifurcation_mesh(h)
    m.name = f"ybif_{m.nc}"
    return m


def vessel_tree_mesh_for_tets(n_tets: int, generations: int = 3) -> Mesh:
    """Bifurcating tree with about n_tets tets."""
    h = _h_for_tets(lambda hh: vessel_tree_mesh(hh, generations), n_tets, 0.08)
    m = vessel_tree_mesh(h, generations)
    m.name = f"tree{generations}_{m.nc}"
    return m
