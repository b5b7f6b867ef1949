"""Seeded synthetic problem generators (graphs, boundary terms, right-hand sides).

This module is the only code shared by the CPU oracle's tests and the GPU path's
tests and benchmark.  It builds the *problem data* of eq. (prob) in Section 1 of
the paper -- a connected graph with edge weights w_e, lower-order boundary terms
d_i on S_b and a right-hand side f -- and nothing of the method itself: no
assembly of A, no aggregation, no smoothing, no reduction.

Every generator returns a :class:`Graph` whose adjacency is stored in CSR form
with both directions of every edge, columns strictly increasing within a row and
no self loops, together with the per-vertex vector ``d``.

Mesh shapes follow the structured meshes of the paper's experiments (Section 4:
2D unit square with n^2 vertices, 3D unit cube with n^3 vertices); the random
geometric graphs stand in for "general graphs".  All randomness comes from
``numpy.random.default_rng`` (PCG64) with explicit seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 13076305


def seed_for(config: int, item: int = 0) -> int:
    """Seed convention: SEED_BASE + 100*config + item."""
    return SEED_BASE + 100 * config + item


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int32, n+1
    col: np.ndarray  # int32, nnz (both directions, sorted per row, no self loops)
    w: np.ndarray  # float64, nnz, symmetric (w_ij == w_ji)
    d: np.ndarray  # float64, n, >= 0, nonzero only on the boundary set S_b
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2


def csr_from_edges(n: int, ei: np.ndarray, ej: np.ndarray, we: np.ndarray | None = None):
    """Symmetric CSR (both directions, sorted columns, duplicates dropped) from an
    undirected edge list.  Duplicate edges keep the first weight seen."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    if we is None:
        we = np.ones(ei.shape[0], dtype=np.float64)
    keep = ei != ej
    ei, ej, we = ei[keep], ej[keep], np.asarray(we, dtype=np.float64)[keep]
    lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    ukey = lo * n + hi
    uorder = np.argsort(ukey, kind="stable")
    ufirst = np.ones(ukey.shape[0], dtype=bool)
    ufirst[1:] = ukey[uorder][1:] != ukey[uorder][:-1]
    sel = uorder[ufirst]
    ei, ej, we = lo[sel], hi[sel], we[sel]
    rows = np.concatenate([ei, ej])
    cols = np.concatenate([ej, ei])
    vals = np.concatenate([we, we])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, rows, cols, vals = key[order], rows[order], cols[order], vals[order]
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    rows, cols, vals = rows[first], cols[first], vals[first]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def grid2d(N: int, M: int | None = None) -> Graph:
    """Triangulated N x M grid of the unit square (M defaults to N).

    Vertex (r, c) has id r*M + c.  Edges: horizontal (r,c)-(r,c+1), vertical
    (r,c)-(r+1,c) and one diagonal per cell (r,c)-(r+1,c+1); all w_e = 1.
    d_i = 1 on the boundary vertices (any of r, c on the domain edge)."""
    M = N if M is None else M
    r, c = np.meshgrid(np.arange(N), np.arange(M), indexing="ij")
    vid = (r * M + c).astype(np.int64)
    ei, ej = [], []
    ei.append(vid[:, :-1].ravel()); ej.append(vid[:, 1:].ravel())
    ei.append(vid[:-1, :].ravel()); ej.append(vid[1:, :].ravel())
    ei.append(vid[:-1, :-1].ravel()); ej.append(vid[1:, 1:].ravel())
    n = N * M
    row_ptr, col, w = csr_from_edges(n, np.concatenate(ei), np.concatenate(ej))
    bnd = (r == 0) | (r == N - 1) | (c == 0) | (c == M - 1)
    d = bnd.ravel().astype(np.float64)
    return Graph(n, row_ptr, col, w, d, name=f"grid2d-{N}x{M}")


def tet3d(N: int) -> Graph:
    """N^3-vertex structured cube, each cell split into 6 tetrahedra sharing the
    (1,1,1) diagonal (Kuhn split).  Vertex (x,y,z) has id (z*N+y)*N+x.  Edge
    directions (1,0,0),(0,1,0),(0,0,1),(1,1,0),(1,0,1),(0,1,1),(1,1,1): interior
    degree 14.  w_e = 1; d_i = 1 on vertices with a coordinate in {0, N-1}."""
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    vid = ((z * N + y) * N + x).astype(np.int64)
    dirs = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]
    ei, ej = [], []
    for dx, dy, dz in dirs:
        src = vid[: N - dz, : N - dy, : N - dx]
        dst = vid[dz:, dy:, dx:]
        ei.append(src.ravel()); ej.append(dst.ravel())
    n = N ** 3
    row_ptr, col, w = csr_from_edges(n, np.concatenate(ei), np.concatenate(ej))
    bnd = (x == 0) | (x == N - 1) | (y == 0) | (y == N - 1) | (z == 0) | (z == N - 1)
    d = bnd.ravel().astype(np.float64)
    return Graph(n, row_ptr, col, w, d, name=f"tet3d-{N}")


def poisson2d(N: int, neumann: bool = True) -> Graph:
    """Linear finite elements for the Laplacian on the unit square with the
    structured right-triangle mesh of Section 4 (n = N^2): the stiffness matrix
    is the 5-point graph Laplacian (the diagonal edges of the triangles carry
    zero weight and are not stored), w_e = 1.  Neumann (d = 0) as in the
    paper's experiments, else d = 1 on the boundary."""
    r, c = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    vid = r * N + c
    ei = np.concatenate([vid[:, :-1].ravel(), vid[:-1, :].ravel()])
    ej = np.concatenate([vid[:, 1:].ravel(), vid[1:, :].ravel()])
    row_ptr, col, w = csr_from_edges(N * N, ei, ej)
    bnd = (r == 0) | (r == N - 1) | (c == 0) | (c == N - 1)
    d = np.zeros(N * N) if neumann else bnd.ravel().astype(np.float64)
    return Graph(N * N, row_ptr, col, w, d, name=f"poisson2d-{N}{'-neumann' if neumann else ''}")


def poisson3d(N: int, neumann: bool = True) -> Graph:
    """The same on the unit cube with the Kuhn 6-tetrahedra mesh (n = N^3): the
    stiffness matrix is the 7-point graph Laplacian (the face and body
    diagonals carry zero weight), w_e = 1, vertex id (z*N+y)*N+x."""
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    vid = ((z * N + y) * N + x).astype(np.int64)
    ei = np.concatenate([vid[:, :, :-1].ravel(), vid[:, :-1, :].ravel(), vid[:-1, :, :].ravel()])
    ej = np.concatenate([vid[:, :, 1:].ravel(), vid[:, 1:, :].ravel(), vid[1:, :, :].ravel()])
    n = N ** 3
    row_ptr, col, w = csr_from_edges(n, ei, ej)
    bnd = (x == 0) | (x == N - 1) | (y == 0) | (y == N - 1) | (z == 0) | (z == N - 1)
    d = np.zeros(n) if neumann else bnd.ravel().astype(np.float64)
    return Graph(n, row_ptr, col, w, d, name=f"poisson3d-{N}{'-neumann' if neumann else ''}")


def project_range(f: np.ndarray) -> np.ndarray:
    """f minus its mean: the right-hand side of a pure Neumann problem must be
    orthogonal to the constants (the kernel of A)."""
    f = np.asarray(f, dtype=np.float64)
    return f - f.mean()


def delaunay3d(N: int, seed: int, neumann: bool = False) -> Graph:
    """Unstructured mesh of the unit cube in the manner of Section 4's general
    graphs: the N^3 vertices of the structured grid (spacing h = 1/(N-1), id
    (z*N+y)*N+x) each moved by a random vector of length h/2 (direction uniform
    on the sphere), then the Delaunay tetrahedralization of the moved points
    (SciPy / Qhull); its edges with w_e = 1.  d_i = 1 on the vertices that lay
    on the cube's boundary before the move, or d = 0 (pure Neumann, as in the
    paper's runs)."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    grid = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)
    v = rng.standard_normal(grid.shape)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    h = 1.0 / (N - 1)
    pts = (grid + 0.5 * v) * h
    tet = Delaunay(pts).simplices.astype(np.int64)
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    ei = np.concatenate([tet[:, a] for a, _ in pairs])
    ej = np.concatenate([tet[:, b] for _, b in pairs])
    n = N ** 3
    row_ptr, col, w = csr_from_edges(n, ei, ej)
    if np.any(np.diff(row_ptr) == 0):
        raise ValueError("a vertex is in no tetrahedron")
    bnd = (x == 0) | (x == N - 1) | (y == 0) | (y == N - 1) | (z == 0) | (z == N - 1)
    d = np.zeros(n) if neumann else bnd.ravel().astype(np.float64)
    return Graph(n, row_ptr, col, w, d, name=f"delaunay3d-{N}-s{seed}{'-neumann' if neumann else ''}")


def _morton16(px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Interleave two 16-bit integer coordinates into a 32-bit Morton key."""

    def spread(v):
        v = v.astype(np.uint64) & 0xFFFF
        v = (v | (v << 8)) & 0x00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F
        v = (v | (v << 2)) & 0x33333333
        v = (v | (v << 1)) & 0x55555555
        return v

    return spread(px) | (spread(py) << np.uint64(1))


def rgg(n_points: int, seed: int, frac_bnd: float = 0.01, mean_degree: float = 6.0) -> Graph:
    """Random geometric graph: n_points uniform points in [0,1]^2, reordered by a
    16-bit-per-axis Morton key, connected when closer than r = sqrt(deg/(pi n)).
    Only the largest connected component is kept (relabelled in order); w_e = 1;
    d_i = 1 on max(1, ceil(frac_bnd * n)) distinct seeded vertices."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n_points, 2))
    q = np.minimum((pts * 65536.0).astype(np.int64), 65535)
    order = np.argsort(_morton16(q[:, 0], q[:, 1]), kind="stable")
    pts = pts[order]
    radius = math.sqrt(mean_degree / (math.pi * n_points))
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    ei, ej = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    adj = coo_matrix((np.ones(ei.shape[0]), (ei, ej)), shape=(n_points, n_points))
    _, lab = connected_components(adj, directed=False)
    big = np.argmax(np.bincount(lab))
    keep = lab == big
    newid = -np.ones(n_points, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    sel = keep[ei] & keep[ej]
    n = int(keep.sum())
    row_ptr, col, w = csr_from_edges(n, newid[ei[sel]], newid[ej[sel]])
    nb = max(1, int(math.ceil(frac_bnd * n)))
    d = np.zeros(n, dtype=np.float64)
    d[rng.permutation(n)[:nb]] = 1.0
    return Graph(n, row_ptr, col, w, d, name=f"rgg-{n_points}-s{seed}")


def rgg_batch_sizes(count: int, seed: int, lo: float = 1e3, hi: float = 2e5) -> np.ndarray:
    """Point counts log-uniform in [lo, hi] for a batch of random geometric graphs."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def rhs(n: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """Right-hand side: 'uniform' = U[-1,1], 'normal' = N(0,1), in vertex order."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, size=n)
    if kind == "normal":
        return rng.standard_normal(n)
    raise ValueError(kind)


def random_graph(n: int, p: float, seed: int, weighted: bool = False, dfrac: float = 0.2) -> Graph:
    """Small connected random graph (a random spanning path plus Erdos-Renyi edges)
    for brute-force and randomized tests.  Weighted variants draw w in [0.5, 2)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    ei = [perm[:-1]]
    ej = [perm[1:]]
    iu, ju = np.triu_indices(n, 1)
    pick = rng.random(iu.shape[0]) < p
    ei.append(iu[pick]); ej.append(ju[pick])
    ei = np.concatenate(ei); ej = np.concatenate(ej)
    we = rng.uniform(0.5, 2.0, size=ei.shape[0]) if weighted else None
    row_ptr, col, w = csr_from_edges(n, ei, ej, we)
    d = np.zeros(n)
    nb = max(1, int(round(dfrac * n)))
    d[rng.permutation(n)[:nb]] = rng.uniform(0.5, 2.0, size=nb) if weighted else 1.0
    return Graph(n, row_ptr, col, w, d, name=f"random-{n}-s{seed}")
