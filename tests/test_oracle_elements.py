"""Pins for the oracle's element integrals and boundary loads.

Closed forms: the quadratic-triangle and quadratic-tet mass matrices
(textbook values from exact barycentric integration), partition-of-unity
and linear-reproduction identities, and the divergence theorem."""
import numpy as np
import pytest

from oracle.assemble import assemble, boundary_loads
from workloads import Mesh, channel_mesh, pipe_mesh


def _single(d, seed=0):
    rng = np.random.default_rng(seed)
    if d == 2:
        xyz = np.array([[0.1, 0.2], [1.3, 0.1], [0.4, 1.1]]) + 0.1 * rng.standard_normal((3, 2))
        cells = np.array([[0, 1, 2]], np.int32)
        faces = np.array([[0, 1], [1, 2], [2, 0]], np.int32)
    else:
        xyz = np.array([[0.0, 0.0, 0.0], [1.2, 0.1, 0.0], [0.2, 1.0, 0.1], [0.1, 0.3, 0.9]])
        xyz = xyz + 0.1 * rng.standard_normal((4, 3))
        cells = np.array([[0, 1, 2, 3]], np.int32)
        faces = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], np.int32)
    return Mesh(d, xyz, cells, faces, np.ones(faces.shape[0], np.int32))


def _dense(asm, vals):
    rp, col = asm["S2"]
    n2 = asm["n2"]
    A = np.zeros((n2, n2))
    for a in range(n2):
        A[a, col[rp[a]:rp[a + 1]]] = vals[rp[a]:rp[a + 1]]
    return A


def test_p2_triangle_mass_closed_form():
    m = _single(2)
    asm = assemble(m)
    x = m.xyz
    u, v = x[1] - x[0], x[2] - x[0]
    area = 0.5 * abs(u[0] * v[1] - u[1] * v[0])
    M = _dense(asm, asm["M"])
    # local order: v0 v1 v2 e01 e12 e02 ; global edges sorted (01,02,12) -> ids 3,4,5
    e = {(0, 1): 3, (0, 2): 4, (1, 2): 5}
    ref = np.zeros((6, 6))
    for i in range(3):
        ref[i, i] = 6
        for j in range(3):
            if j != i:
                ref[i, j] = -1
    for (a, b), k in e.items():
        opp = 3 - a - b
        ref[opp, k] = ref[k, opp] = -4
        for (a2, b2), k2 in e.items():
            ref[k, k2] = 32 if k == k2 else 16
    assert np.allclose(M, area / 180.0 * ref, rtol=0, atol=1e-15)


def test_p2_tet_mass_closed_form():
    m = _single(3)
    asm = assemble(m)
    x = m.xyz
    vol = abs(np.dot(np.cross(x[1] - x[0], x[2] - x[0]), x[3] - x[0])) / 6.0
    M = _dense(asm, asm["M"])
    edges = [tuple(e) for e in asm["edges"]]
    ref = np.zeros((10, 10))
    for i in range(4):
        for j in range(4):
            ref[i, j] = 6 if i == j else 1
    for k, (a, b) in enumerate(edges):
        K = 4 + k
        for v in range(4):
            ref[v, K] = ref[K, v] = -4 if v in (a, b) else -6
        for k2, (a2, b2) in enumerate(edges):
            K2 = 4 + k2
            ref[K, K2] = 32 if K == K2 else (16 if len({a, b} & {a2, b2}) == 1 else 8)
    assert np.allclose(M, vol / 420.0 * ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("which", ["channel", "pipe_curved", "pipe_straight"])
def test_global_identities(which):
    if which == "channel":
        m = channel_mesh(8, 4)
    else:
        m = pipe_mesh(0.6, length=2.0, curved=(which == "pipe_curved"))
    asm = assemble(m)
    d, n2, nv = m.dim, asm["n2"], asm["nv"]
    Ks = _dense(asm, asm["Ks"])
    M = _dense(asm, asm["M"])
    X = asm["node_xyz"]
    vol = M.sum()
    # constants are in the space: stiffness rows sum to zero
    assert np.abs(Ks.sum(1)).max() < 1e-12
    # coordinates are in the (isoparametric) space: int |grad x_c|^2 = |Omega|
    for c in range(d):
        assert abs(X[:, c] @ Ks @ X[:, c] - vol) < 1e-11 * vol
        assert abs(X[:, c] @ M @ np.ones(n2) - np.sum(M @ X[:, c])) < 1e-12
    if which != "pipe_curved":
        exact = 4.0 * 1.0 if which == "channel" else None
        if exact is not None:
            assert abs(vol - exact) < 1e-12
    # lumped pressure mass sums to the volume
    assert abs(asm["Mp"].sum() - vol) < 1e-12 * vol
    rp21, col21 = asm["C21"]
    rows = np.repeat(np.arange(n2), np.diff(rp21))
    for c in range(d):
        G = np.zeros((n2, nv))
        G[rows, col21] = asm["G"][c]
        # sum_A G^c_Av = -int d_c(1) N_v = 0
        assert np.abs(G.sum(0)).max() < 1e-12
        # sum_A x^c'_A G^c_Av = -delta_cc' int N_v
        for c2 in range(d):
            val = X[:, c2] @ G
            ref = -asm["Mp"] if c == c2 else 0.0
            assert np.abs(val - ref).max() < 1e-12


def test_facet_loads_flat_closed_form():
    """Quadratic facet basis integrals: segment L/6, L/6, 2L/3; triangle 0,0,0,
    |F|/3 x3. Summed over a closed boundary, int n dGamma vanishes."""
    m = _single(2)
    asm = assemble(m)
    lo = boundary_loads(m, asm, [1])[0]
    x = m.xyz
    for a, b in m.bfaces:
        t = x[b] - x[a]
        n = np.array([t[1], -t[0]])
        e = 3 + {(0, 1): 0, (0, 2): 1, (1, 2): 2}[tuple(sorted((a, b)))]
        assert np.allclose(lo[e], 2.0 / 3.0 * n)
    assert np.allclose(lo.sum(0), 0.0, atol=1e-15)
    # outward: n points away from the centroid
    m3 = _single(3)
    asm3 = assemble(m3)
    lo3 = boundary_loads(m3, asm3, [1])[0]
    assert np.allclose(lo3[:4], 0.0, atol=1e-15)
    assert np.allclose(lo3.sum(0), 0.0, atol=1e-15)
    cen = m3.xyz.mean(0)
    for f in m3.bfaces:
        x0, x1, x2 = m3.xyz[f]
        nrm = np.cross(x1 - x0, x2 - x0)
        assert np.dot(nrm, x0 - cen) > 0


def test_pipe_loads_and_closed_surface():
    m = pipe_mesh(0.5, length=2.0)
    asm = assemble(m)
    lo = boundary_loads(m, asm, [1, 2, 3])
    inlet, outlet = lo[0].sum(0), lo[1].sum(0)
    # flat caps: int n = area * normal; the polygonal cap area is below pi
    assert inlet[2] < 0 and outlet[2] > 0 and abs(inlet[2] + outlet[2]) < 1e-12
    assert np.allclose(inlet[:2], 0, atol=1e-12)
    assert np.allclose(lo.sum((0, 1)), 0.0, atol=1e-12)
