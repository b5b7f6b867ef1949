"""Pins of the oracle's A-norm error stopping test (Section 4: the iteration
stops at a 1e-8 reduction of the relative A-norm of the error)."""
import numpy as np
import pytest

import inputs
import oracle


def _hier(g, **kw):
    return oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(**kw))


def test_energy_decreases_monotonically():
    # every flexible-CG step minimizes the A-norm of the error along its
    # direction, so the history cannot increase, whatever the preconditioner
    g = inputs.grid2d(48)
    h = _hier(g, degree=3, agg_size=4, stop="energy")
    u0 = inputs.rhs(g.n, 3)
    res = oracle.fcg(h, np.zeros(g.n), u0)
    assert res.converged and res.iters > 3
    hist = np.array(res.res_history)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    assert hist[-1] <= 1e-8 * hist[0] < hist[-2]


def test_energy_equals_dual_norm_of_residual():
    # ||x* - x||_A^2 = r^T A^-1 r with r = f - A x: the measured A-norms against a dense solve
    g = inputs.grid2d(20)
    lvl = oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)
    A = lvl.dense()
    f = inputs.rhs(g.n, 4)
    xs = np.linalg.solve(A, f)
    h = _hier(g, degree=3, agg_size=4, stop="energy", tol=1e-6)
    res = oracle.fcg(h, f, x_exact=xs)
    r = f - A @ res.x
    assert res.res_history[-1] == pytest.approx(np.sqrt(r @ np.linalg.solve(A, r)), rel=1e-6)
    assert res.res_history[0] == pytest.approx(np.sqrt(f @ xs), rel=1e-12)


def test_homogeneous_problem_is_the_error_equation():
    # solving A x = A x* from x* + e0 runs the same iteration as A e = 0 from e0
    g = inputs.grid2d(40, 23)
    h = _hier(g, degree=4, agg_size=4, stop="energy")
    lvl = h.levels[0]
    xs = inputs.rhs(g.n, 5)
    e0 = inputs.rhs(g.n, 6)
    a = oracle.fcg(h, oracle.apply_A(lvl, xs), xs + e0, x_exact=xs)
    b = oracle.fcg(h, np.zeros(g.n), e0)
    assert a.iters == b.iters
    assert np.linalg.norm((a.x - xs) - b.x) <= 1e-7 * np.linalg.norm(e0)


def test_energy_test_needs_the_solution_or_zero_rhs():
    g = inputs.grid2d(10)
    h = _hier(g, degree=3, agg_size=4, stop="energy")
    with pytest.raises(ValueError):
        oracle.fcg(h, inputs.rhs(g.n, 1))


def test_neumann_constants_do_not_count():
    # pure Neumann: the error is measured modulo the kernel (the constants)
    g = inputs.poisson2d(40)
    h = _hier(g, degree=4, aggregation="mis", stop="energy")
    u0 = inputs.project_range(inputs.rhs(g.n, 8))
    a = oracle.fcg(h, np.zeros(g.n), u0)
    b = oracle.fcg(h, np.zeros(g.n), u0 + 5.0)
    assert a.converged and a.iters == b.iters
    assert a.res_history[0] == pytest.approx(b.res_history[0], rel=1e-9)


def test_energy_and_residual_tests_agree_on_exact_solves():
    # a one-level hierarchy solves exactly in one step under either test
    g = inputs.grid2d(6)
    for stop in ("residual", "energy"):
        h = _hier(g, degree=3, agg_size=4, coarse_max=64, stop=stop)
        assert h.L == 0
        res = oracle.fcg(h, np.zeros(g.n), inputs.rhs(g.n, 2))
        assert res.converged and res.iters == 1, stop
