"""Pins for the oracle's reported figures and limits: grid and operator
complexity, the iteration limit, the coarsest-size limit, the aggregate size
that a number of pairwise matching passes allows (Section 2), the inner
flexible CG on a zero right-hand side (Section 4's recursive NPCG), and the
count of recursive residuals replaced by the true one."""
import numpy as np
import pytest

import inputs
import oracle
from oracle.cycle import CoarsenError, fcg_fixed


def _hier(g, **kw):
    return oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(**kw))


@pytest.mark.parametrize("make,kw", [
    (lambda: inputs.grid2d(40), dict(degree=3, agg_size=4)),
    (lambda: inputs.rgg(1500, seed=3), dict(degree=3, agg_size=16)),
])
def test_complexities_from_dense_levels(make, kw):
    """Grid complexity is sum_l n_l / n_0; operator complexity is the number of
    nonzero entries of all A_l over that of A_0 (diagonal included), counted
    here on the dense matrices."""
    h = _hier(make(), **kw)
    assert h.L >= 2
    dense = [lvl.dense() for lvl in h.levels]
    nz = [np.count_nonzero(D) for D in dense]
    assert h.grid_complexity() == pytest.approx(sum(D.shape[0] for D in dense) / dense[0].shape[0], rel=1e-15)
    assert h.operator_complexity() == pytest.approx(sum(nz) / nz[0], rel=1e-15)
    assert 1.0 < h.grid_complexity() < h.operator_complexity() + 1.0


@pytest.mark.parametrize("max_iter", [1, 3, 7])
def test_iteration_limit_is_exact(max_iter):
    """A solve that cannot meet its tolerance stops after exactly max_iter
    preconditioner applications, with one residual norm per iteration."""
    g = inputs.grid2d(24)
    h = _hier(g, degree=3, agg_size=4, tol=1e-30, max_iter=max_iter)
    calls = []
    res = oracle.fcg(h, inputs.rhs(g.n, 2), callback=lambda x: calls.append(1))
    assert res.iters == max_iter and len(calls) == max_iter
    assert not res.converged and not res.breakdown
    assert len(res.res_history) == max_iter + 1


def test_inner_fcg_on_zero_rhs_is_zero():
    """The recursive flexible CG on a zero coarse right-hand side returns zero:
    both of its directions vanish, and a coefficient over rho = 0 is zero
    rather than a division by zero."""
    g = inputs.grid2d(40)
    h = _hier(g, degree=3, agg_size=4)
    assert h.L >= 3
    for steps in (1, 2, 3):
        e = fcg_fixed(h, 1, np.zeros(h.levels[1].n), steps)
        assert np.all(e == 0.0)


@pytest.mark.parametrize("agg_size,limit", [(2, 2), (4, 4), (16, 16)])
def test_aggregate_size_bounded_by_passes(agg_size, limit):
    """p passes of pairwise matching merge at most 2^p vertices: with a target
    size of 2 (one pass) no aggregate holds more than two vertices; the bound
    is reached on a grid, where the matching is close to perfect."""
    g = inputs.grid2d(32)
    h = _hier(g, degree=3, agg_size=agg_size, coarse_max=8)
    for l, agg in enumerate(h.aggs):
        sizes = np.bincount(agg, minlength=h.levels[l + 1].n)
        assert sizes.min() >= 1 and sizes.max() <= limit
    assert np.bincount(h.aggs[0]).max() == limit


def test_coarsest_size_limit_is_inclusive():
    """The coarsest level may hold exactly max_coarsest rows, not one more."""
    g = inputs.grid2d(20)
    nL = _hier(g, degree=3, agg_size=4, coarse_max=100).levels[-1].n
    assert _hier(g, degree=3, agg_size=4, coarse_max=100, max_coarsest=nL).levels[-1].n == nL
    with pytest.raises(CoarsenError):
        _hier(g, degree=3, agg_size=4, coarse_max=100, max_coarsest=nL - 1)


@pytest.mark.parametrize("N,agg,tol", [(32, 4, 1e-15), (48, 16, 3e-15)])
def test_replacement_count(N, agg, tol):
    """Each pass of the recursive residual that the true residual does not
    confirm is one replacement: on a converged solve, the count is the number
    of recursive passes (the residual history holds the recursive norms) less
    the final, confirmed one."""
    g = inputs.grid2d(N)
    h = _hier(g, degree=3, agg_size=agg, tol=tol, max_iter=80)
    res = oracle.fcg(h, inputs.rhs(g.n, 9))
    assert res.converged
    hist = np.array(res.res_history)
    passes = int(np.count_nonzero(hist[1:] <= tol * hist[0]))
    assert res.replacements >= 1 and res.replacements == passes - 1


def test_zero_direction_is_a_breakdown():
    """A preconditioner that returns zero for a nonzero residual gives rho =
    (p, A p) = 0: the outer iteration reports a breakdown at its first step and
    leaves the iterate unchanged."""
    g = inputs.grid2d(16)
    h = _hier(g, degree=3, agg_size=4)
    res = oracle.fcg(h, inputs.rhs(g.n, 4), precond=lambda r: np.zeros_like(r))
    assert res.breakdown and not res.converged and res.iters == 1
    assert np.all(res.x == 0.0)


def test_smoother_error_limit_is_strict():
    """E_m < 1 is required: with lambda1 / lambda0 = 3 the best constant
    (m = 0) has 1 - x q_0(x) = -1 at x = lambda1, so E_0 = 1 exactly and the
    setup refuses it, while m = 1 on the same interval is accepted."""
    g = inputs.grid2d(12)
    assert oracle.error_Em(0, 3.0) == 1.0
    p0 = oracle.best_poly(1.0, 0, 3.0)
    assert float(oracle.residual_poly_eval(p0, np.array([1.0]))[0]) == pytest.approx(-1.0, abs=1e-15)
    with pytest.raises(ValueError):
        _hier(g, degree=0, lambda0_ratio=3.0)
    assert _hier(g, degree=1, lambda0_ratio=3.0, coarse_max=16).L >= 1


@pytest.mark.parametrize("kappa,m", [(10.0, 3), (10.0, 5), (30.0, 9)])
def test_degree_for_takes_the_bound_inclusively(kappa, m):
    """The bound on m of Section 3 is E_m <= rho: at rho = E_m exactly the
    degree is m itself (E_m decreases strictly in m), and just below it m + 1."""
    from oracle.poly import degree_for
    e = oracle.error_Em(m, kappa)
    assert degree_for(e, kappa) == m
    assert degree_for(e * (1 - 1e-12), kappa) == m + 1
    # E_0 = 1 at kappa = 3: m = 0 fails E_m < 1 even for rho = 1
    assert degree_for(1.0, 3.0) == 1


def test_degree_cap():
    """The search runs up to and including the cap; without a degree that meets
    the bound by then, the cap itself is taken (first passing degree 4)."""
    from oracle.poly import degree_for
    e4 = oracle.error_Em(4, 10.0)
    assert degree_for(e4, 10.0) == 4
    assert degree_for(e4, 10.0, max_degree=3) == 3
    assert degree_for(e4, 10.0, max_degree=4) == 4
    assert degree_for(e4, 10.0, max_degree=5) == 4


@pytest.mark.parametrize("w_pair,w_tri,expected", [
    (0.1, 1.0, 5.0),        # the pair dominates: 1 / (2 * 0.1)
    (1.0, 0.1, 1.0 / 0.3),  # the triangle dominates: 1 / (3 * 0.1)
])
def test_local_cp_closed_forms(w_pair, w_tri, expected):
    """c_p of eq. (wap) on aggregates whose Laplacian spectra are known: a pair
    joined by weight w has eigenvalues 0, 2w; a triangle of weight w has 0, 3w,
    3w; a singleton contributes nothing; edges between aggregates do not enter.
    Aggregates: {0, 1, 2} triangle, {3, 4} pair, {5} singleton, with unit
    edges 2-3 and 4-5 joining them."""
    from oracle import spectral
    ei = np.array([0, 1, 0, 3, 2, 4])
    ej = np.array([1, 2, 2, 4, 3, 5])
    we = np.array([w_tri, w_tri, w_tri, w_pair, 1.0, 1.0])
    row_ptr, col, w = inputs.csr_from_edges(6, ei, ej, we)
    lvl = oracle.assemble(6, row_ptr, col, w, np.zeros(6))
    agg = np.array([0, 0, 0, 1, 1, 2])
    assert spectral.local_cp(lvl, agg) == pytest.approx(expected, rel=1e-12)
