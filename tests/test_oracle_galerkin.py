"""Pins for the oracle's Galerkin operator A_H = P^T A P (Section 3) and the
quotient graph of Section 2."""
import numpy as np
import pytest

import inputs
import oracle
from oracle.spectral import prolongator


CASES = [
    (lambda: inputs.grid2d(16, 13), 2),
    (lambda: inputs.tet3d(6), 3),
    (lambda: inputs.random_graph(80, 0.05, seed=11, weighted=True), 2),
    (lambda: inputs.rgg(1500, seed=2), 3),
    (lambda: inputs.delaunay3d(8, seed=9), 3),
]


@pytest.mark.parametrize("make,passes", CASES)
def test_quotient_equals_dense_triple_product(make, passes):
    g = make()
    lvl = oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)
    agg, coarse = oracle.aggregate_level(lvl, passes)
    P = prolongator(agg, coarse.n)
    AH = P.T @ lvl.dense() @ P
    if np.all(g.w == np.round(g.w)) and np.all(g.d == np.round(g.d)):
        assert np.array_equal(coarse.dense(), AH)  # integer sums are exact
    else:
        np.testing.assert_allclose(coarse.dense(), AH, rtol=1e-13, atol=1e-13)
    # symmetric, row sums = d_H (zero on aggregates away from the boundary)
    Ad = coarse.dense()
    assert np.array_equal(Ad, Ad.T)
    np.testing.assert_allclose(Ad.sum(axis=1), coarse.d, atol=1e-12)
    np.testing.assert_allclose(coarse.d, P.T @ g.d, atol=1e-13)
    if np.all(g.w == 1):
        # unit weights: the row sums are exactly d_H, zero on interior aggregates
        assert np.array_equal(Ad.sum(axis=1), coarse.d)
        assert np.all(Ad.sum(axis=1)[coarse.d == 0] == 0)


@pytest.mark.parametrize("make,passes", CASES)
def test_pattern_is_quotient_graph(make, passes):
    """Edge (I,J) is in the coarse graph iff aggregates I and J are adjacent."""
    g = make()
    lvl = oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)
    agg, coarse = oracle.aggregate_level(lvl, passes)
    rows = lvl.rows()
    I, J = agg[rows], agg[lvl.col]
    want = sorted(set((a, b) for a, b in zip(I.tolist(), J.tolist()) if a != b))
    got = list(zip(coarse.rows().tolist(), coarse.col.tolist()))
    assert got == want
    assert np.all(coarse.W > 0)


def test_multipass_equals_direct_galerkin():
    """Quotient of quotients = one Galerkin product with the composed map."""
    g = inputs.random_graph(120, 0.04, seed=21, weighted=False)
    lvl = oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)
    agg, chained = oracle.aggregate_level(lvl, 3)
    direct = oracle.quotient(lvl, agg, chained.n)
    assert np.array_equal(direct.row_ptr, chained.row_ptr)
    assert np.array_equal(direct.col, chained.col)
    assert np.array_equal(direct.W, chained.W)
    assert np.array_equal(direct.D, chained.D)


@pytest.mark.parametrize("aggregation", ["matching", "mis"])
def test_transfers_are_the_piecewise_constant_prolongator(aggregation):
    """Restriction and prolongation equal P^T v and P e for the 0/1 matrix with
    P[i, agg(i)] = 1 (built here from its definition), and A_H = P^T A P."""
    g = inputs.poisson2d(30) if aggregation == "mis" else inputs.grid2d(30, 17)
    h = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d,
                               oracle.Params(agg_size=4, aggregation=aggregation, coarse_max=8))
    rng = np.random.default_rng(4)
    for l in range(h.L):
        agg, n, nc = h.aggs[l], h.levels[l].n, h.levels[l + 1].n
        P = np.zeros((n, nc))
        P[np.arange(n), agg] = 1.0
        v, e = rng.standard_normal(n), rng.standard_normal(nc)
        np.testing.assert_allclose(oracle.restrict(agg, nc, v), P.T @ v, rtol=0, atol=1e-12)
        np.testing.assert_allclose(oracle.prolong(agg, e), P @ e, rtol=0, atol=0)
        np.testing.assert_allclose(h.levels[l + 1].dense(), P.T @ h.levels[l].dense() @ P, rtol=0, atol=1e-12)
