"""Pins for the oracle's operator assembly (eq. (prob), Section 1)."""
import numpy as np
import pytest

import inputs
import oracle
from oracle.level import bilinear_form


GRAPHS = [
    lambda: inputs.grid2d(9, 7),
    lambda: inputs.tet3d(5),
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
