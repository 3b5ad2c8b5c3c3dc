"""Pins for the oracle's quadratic numbering and sparsity patterns."""
import json
import os
from itertools import combinations

import numpy as np

from oracle.numbering import p2_numbering, s2_pattern, c21_pattern
from workloads import channel_mesh, pipe_mesh

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def test_paper_channel_counts():
    """Section 3.2 prints 882 quadratic triangles, 1,881 nodes and 4,262 DOF;
    a 49x9 split grid has exactly those counts (and 500 vertices)."""
    g = json.load(open(GOLD))["channel"]
    m = channel_mesh(49, 9, 49 / 9, 1.0)
    edges, c2n = p2_numbering(m.nv, m.cells)
    n2 = m.nv + edges.shape[0]
    assert m.nc == g["cells"] and n2 == g["nodes"] and 2 * n2 + m.nv == g["dof"]


def test_glenn_counts_consistent():
    """Glenn (section 3.5): DOF = 3 * nodes + vertices gives an integer vertex
    count below the node count, as the counting rule requires."""
    g = json.load(open(GOLD))["glenn"]
    nv = g["dof"] - 3 * g["nodes"]
    assert 0 < nv < g["nodes"]


def test_euler_2d():
    for nx, ny in [(32, 8), (5, 3)]:
        m = channel_mesh(nx, ny)
        edges, _ = p2_numbering(m.nv, m.cells)
        assert m.nv + edges.shape[0] == 2 * m.nv + m.nc - 1


def test_euler_3d_ball():
    m = pipe_mesh(0.5, length=2.0)
    edges, _ = p2_numbering(m.nv, m.cells)
    # V - E + F - T = 1 for a ball; F = (4T + Fb)/2
    F = (4 * m.nc + m.bfaces.shape[0]) // 2
    assert m.nv - edges.shape[0] + F - m.nc == 1


def test_config_channel_exact_counts():
    m = channel_mesh(32, 8)
    edges, c2n = p2_numbering(m.nv, m.cells)
    n2 = m.nv + edges.shape[0]
    rp, col = s2_pattern(c2n, n2)
    rp21, col21 = c21_pattern(c2n, m.cells, n2, m.nv)
    assert (m.nv, edges.shape[0], n2, 2 * n2 + m.nv) == (297, 808, 1105, 2507)
    assert (col.size, col21.size) == (12097, 5065)


def _brute(m):
    """Numbering and patterns by explicit loops over cells and node pairs."""
    d = m.dim
    le = [(0, 1), (1, 2), (0, 2)] if d == 2 else [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]
    es = sorted({tuple(sorted((int(c[i]), int(c[j])))) for c in m.cells for i, j in le})
    eid = {e: m.nv + k for k, e in enumerate(es)}
    c2n = [[int(v) for v in c] + [eid[tuple(sorted((int(c[i]), int(c[j]))))] for i, j in le]
           for c in m.cells]
    n2 = m.nv + len(es)
    s2 = [set() for _ in range(n2)]
    c21 = [set() for _ in range(n2)]
    for c, nodes in zip(m.cells, c2n):
        for a in nodes:
            s2[a].update(nodes)
            c21[a].update(int(v) for v in c)
    return np.array(es), np.array(c2n), [sorted(r) for r in s2], [sorted(r) for r in c21]


def test_brute_force_small_2d_3d():
    for m in [channel_mesh(4, 3), pipe_mesh(0.7, length=1.5)]:
        edges, c2n = p2_numbering(m.nv, m.cells)
        be, bc, bs2, bc21 = _brute(m)
        assert np.array_equal(edges, be) and np.array_equal(c2n, bc)
        n2 = m.nv + edges.shape[0]
        rp, col = s2_pattern(c2n, n2)
        rp21, col21 = c21_pattern(c2n, m.cells, n2, m.nv)
        for a in range(n2):
            assert list(col[rp[a]:rp[a + 1]]) == bs2[a]
            assert list(col21[rp21[a]:rp21[a + 1]]) == bc21[a]


def test_c21_is_vertex_prefix_of_s2():
    """Vertex ids precede edge ids, so each C21 row is the vertex part of the
    S2 row; and the S2 row of a vertex is its C21-transpose row."""
    m = pipe_mesh(0.6, length=2.0)
    edges, c2n = p2_numbering(m.nv, m.cells)
    n2 = m.nv + edges.shape[0]
    rp, col = s2_pattern(c2n, n2)
    rp21, col21 = c21_pattern(c2n, m.cells, n2, m.nv)
    for a in range(0, n2, 7):
        r = col[rp[a]:rp[a + 1]]
        assert np.array_equal(r[r < m.nv], col21[rp21[a]:rp21[a + 1]])
    rows21 = np.repeat(np.arange(n2), np.diff(rp21))
    for v in range(0, m.nv, 5):
        assert np.array_equal(np.sort(rows21[col21 == v]), col[rp[v]:rp[v + 1]])


def test_vessel_meshes_are_balls_with_tagged_openings():
    """The voxel vessel meshes are single balls (V - E + F - T = 1), every
    boundary facet is used by one tet, and every opening got its tag."""
    from workloads.meshes import INLET, WALL, vessel_tree_mesh, y_bifurcation_mesh
    for m, n_out in ((y_bifurcation_mesh(0.35), 2), (vessel_tree_mesh(0.25, 3), 8)):
        edges, _ = p2_numbering(m.nv, m.cells)
        F = (4 * m.nc + m.bfaces.shape[0]) // 2
        assert m.nv - edges.shape[0] + F - m.nc == 1, m.name
        tags = set(np.unique(m.btags).tolist())
        assert INLET in tags and WALL in tags
        assert len(tags - {INLET, WALL}) == n_out, (m.name, tags)
        vol = np.abs(np.einsum("ij,ij->i", np.cross(m.xyz[m.cells[:, 1]] - m.xyz[m.cells[:, 0]],
                                                   m.xyz[m.cells[:, 2]] - m.xyz[m.cells[:, 0]]),
                               m.xyz[m.cells[:, 3]] - m.xyz[m.cells[:, 0]])) / 6.0
        assert vol.min() > 0.0
