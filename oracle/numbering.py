"""Quadratic-node numbering and structural sparsity (oracle; test infrastructure only).

Section 2.3 (Eq. shape_fun) places quadratic velocity nodes at the simplex
vertices and edge midpoints and linear pressure nodes at the vertices; the
paper leaves the global numbering to its pre-processing script. The numbering
used throughout this project is:
* vertices keep their input index 0..nv-1;
* edges are the unique vertex pairs {a<b} of all cells, sorted
  lexicographically; edge e gets node id nv + e;
* cell-local node order: vertices, then edges (0,1),(1,2),(0,2) and in 3D
  also (0,3),(1,3),(2,3).
Patterns come from connectivity only: S2 holds every (A,B) of quadratic
nodes sharing a cell, C21 every (A, v) of a quadratic node and a vertex of a
cell containing it. Rows are sorted; explicit zeros are kept.
"""
from __future__ import annotations

import numpy as np

LOCAL_EDGES = {2: [(0, 1), (1, 2), (0, 2)],
               3: [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]}


def p2_numbering(nv: int, cells: np.ndarray):
    """Returns edges int64 [ne,2] (lexicographic) and c2n int64 [nc, 6|10]."""
    cells = np.asarray(cells, np.int64)
    d = cells.shape[1] - 1
    le = LOCAL_EDGES[d]
    a = np.stack([np.minimum(cells[:, i], cells[:, j]) for i, j in le], 1)
    b = np.stack([np.maximum(cells[:, i], cells[:, j]) for i, j in le], 1)
    key = a * nv + b
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    edges = np.stack([uniq // nv, uniq % nv], 1)
    c2n = np.concatenate([cells, nv + inv.reshape(cells.shape[0], len(le))], 1)
    return edges, c2n


def _pairs_to_csr(rows: np.ndarray, cols: np.ndarray, nrows: int, ncols: int):
    key = np.unique(rows.astype(np.int64) * ncols + cols)
    r = key // ncols
    c = key % ncols
    rowptr = np.zeros(nrows + 1, np.int64)
    np.add.at(rowptr, r + 1, 1)
    return np.cumsum(rowptr), c.astype(np.int64)


def s2_pattern(c2n: np.ndarray, n2: int):
    """CSR (rowptr int64 [n2+1], col int64) of quadratic node pairs sharing a cell."""
    nn = c2n.shape[1]
    rows = np.repeat(c2n, nn, axis=1).ravel()
    cols = np.tile(c2n, (1, nn)).ravel()
    return _pairs_to_csr(rows, cols, n2, n2)


def c21_pattern(c2n: np.ndarray, cells: np.ndarray, n2: int, nv: int):
    """CSR of (quadratic node, vertex) pairs sharing a cell."""
    nn = c2n.shape[1]
    nvl = cells.shape[1]
    rows = np.repeat(c2n, nvl, axis=1).ravel()
    cols = np.tile(np.asarray(cells, np.int64), (1, nn)).ravel()
    return _pairs_to_csr(rows, cols, n2, nv)
