"""Pins for the oracle's operator assembly (eq. (prob), Section 1)."""
import numpy as np
import pytest

import inputs
import oracle
from oracle.level import bilinear_form


GRAPHS = [
    lambda: inputs.grid2d(9, 7),
    lambda: inputs.tet3d(5),
    lambda: inputs.delaunay3d(6, seed=7),
    lambda: inputs.random_graph(30, 0.15, seed=3, weighted=True),
    lambda: inputs.random_graph(25, 0.2, seed=4, weighted=False),
]


@pytest.mark.parametrize("make", GRAPHS)
def test_constants_map_to_d(make):
    """A 1 = d exactly: the constants span the kernel of the pure Laplacian."""
    g = make()
    lvl = oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)
    Au = oracle.apply_A(lvl, np.ones(g.n))
    if np.all(g.w == np.round(g.w)):
        assert np.array_equal(Au, g.d)
    else:
        np.testing.assert_allclose(Au, g.d, atol=1e-13)
    lvl0 = oracle.assemble(g.n, g.row_ptr, g.col, g.w, np.zeros(g.n))
    np.testing.assert_allclose(oracle.apply_A(lvl0, np.ones(g.n)), 0.0, atol=1e-13)


@pytest.mark.parametrize("make", GRAPHS)
def test_bilinear_form_matches_edge_sum(make):
    """(Au, v) equals the edge-by-edge sum of eq. (prob) and A is symmetric."""
    g = make()
    lvl = oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(g.n), rng.standard_normal(g.n)
    ref = bilinear_form(g.n, g.row_ptr, g.col, g.w, g.d, u, v)
    got = float(np.dot(oracle.apply_A(lvl, u), v))
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-12)
    A = lvl.dense()
    assert np.array_equal(A, A.T)
    assert np.all(np.linalg.eigvalsh(A) > 0)  # connected + some d_i > 0 => SPD


def test_diagonal_is_degree_plus_d():
    g = inputs.grid2d(6)
    lvl = oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)
    deg = np.diff(g.row_ptr)
    assert np.array_equal(lvl.D, deg + g.d)
    # interior vertex of the triangulated grid: 6 neighbours, no boundary term
    assert lvl.D[2 * 6 + 2] == 6.0
    # corners: (0,0) has 3 neighbours (right, down, diagonal) + d = 1
    assert lvl.D[0] == 4.0


def test_generators_shapes():
    g = inputs.grid2d(64)
    assert g.n == 4096 and g.nnz == 24066
    t = inputs.tet3d(6)
    deg = np.diff(t.row_ptr)
    assert deg.max() == 14
    inner = (2 * 6 + 2) * 6 + 2
    assert deg[inner] == 14


def test_delaunay_mesh():
    """Jittered-grid Delaunay mesh of the cube: valid symmetric CSR, every
    vertex in the mesh, connected, the boundary set of the structured grid, a
    reproducible draw, and the Euler characteristic of a tetrahedralized ball
    (V - E + F - T = 1) for the triangulation it came from."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import Delaunay

    N = 9
    g = inputs.delaunay3d(N, seed=11)
    assert g.n == N ** 3
    A = csr_matrix((g.w, g.col, g.row_ptr), shape=(g.n, g.n))
    assert (A != A.T).nnz == 0 and np.all(A.diagonal() == 0)
    for i in range(g.n):
        c = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    assert connected_components(A, directed=False)[0] == 1
    assert int(g.d.sum()) == N ** 3 - (N - 2) ** 3
    g2 = inputs.delaunay3d(N, seed=11)
    assert np.array_equal(g.col, g2.col) and np.array_equal(g.row_ptr, g2.row_ptr)
    assert not np.array_equal(inputs.delaunay3d(N, seed=12).col[:50], g.col[:50]) or \
        inputs.delaunay3d(N, seed=12).nnz != g.nnz
    # the same triangulation, rebuilt from the same draw, gives the Euler characteristic
    rng = np.random.default_rng(11)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    grid = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)
    v = rng.standard_normal(grid.shape)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    tet = Delaunay((grid + 0.5 * v) / (N - 1)).simplices
    faces = {tuple(sorted(f)) for t in tet for f in
             ((t[0], t[1], t[2]), (t[0], t[1], t[3]), (t[0], t[2], t[3]), (t[1], t[2], t[3]))}
    assert g.n - g.n_edges + len(faces) - len(tet) == 1
