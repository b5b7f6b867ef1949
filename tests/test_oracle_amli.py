"""Pins for the stationary AMLI cycle of the oracle (Section 4's AMLI column;
readings in oracle/amli.py)."""
import numpy as np
import pytest

import inputs
import oracle


def test_splitmix64_reference_outputs():
    """The first outputs of splitmix64 seeded with 0, as published with the generator."""
    x, out = 0, []
    for _ in range(3):
        out.append(oracle.splitmix64(x))
        x = (x + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    v = oracle.start_vector(3, 1000)
    assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.1


@pytest.mark.parametrize("a", [0.2, 0.45, 0.8])
def test_degree_one_best_approximation(a):
    """p(t) = g0 + g1 t equioscillates at a, t* and 1 (Chebyshev alternation for
    degree 1), t* the interior extremum of 1/t - p(t); and p > 0 on [a, 1]."""
    g0, g1 = oracle.poly_coefficients(a)
    err = lambda t: 1.0 / t - g0 - g1 * t
    ts = 1.0 / np.sqrt(-g1)
    assert a < ts < 1.0
    e = [err(a), err(ts), err(1.0)]
    assert e[0] == pytest.approx(e[2], rel=1e-12)
    assert e[1] == pytest.approx(-e[0], rel=1e-12)
    t = np.linspace(a, 1.0, 20001)
    assert np.max(np.abs(err(t))) <= abs(e[0]) * (1 + 1e-9)
    assert g0 + g1 > 0.0


def _dense_BA(h, l, coef):
    lvl = h.levels[l]
    A = lvl.dense()
    B = np.column_stack([oracle.amli_cycle(h, l, np.eye(lvl.n)[:, j], coef) for j in range(lvl.n)])
    return A, B


@pytest.mark.parametrize("make,kw", [
    (lambda: inputs.grid2d(40), dict(degree=4, agg_size=4)),
    (lambda: inputs.tet3d(12), dict(degree=3, agg_size=4)),
    (lambda: inputs.rgg(1500, seed=3), dict(degree=4, agg_size=4)),
])
def test_power_estimate_and_spd(make, kw):
    """The power estimate of lambda_min(B A) matches a dense eigensolve on the
    small levels, and each level's B is symmetric positive definite."""
    g = make()
    h = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(**kw))
    assert h.L >= 3
    a, coef = oracle.amli_setup(h)
    checked = 0
    for l in range(h.L - 1, 0, -1):
        if h.levels[l].n > 400:
            continue
        A, B = _dense_BA(h, l, coef)
        assert np.allclose(B, B.T, rtol=1e-10, atol=1e-12)
        assert np.linalg.eigvalsh((B + B.T) / 2).min() > 0
        lam = np.linalg.eigvals(B @ A).real.min()
        assert a[l] == pytest.approx(lam, rel=2e-2)
        checked += 1
    assert checked >= 1


def test_exact_coarse_level_equals_kcycle():
    """Directly above the coarsest level both cycles use the exact solve."""
    g = inputs.grid2d(30)
    h = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=4, agg_size=4))
    r = inputs.rhs(h.levels[h.L - 1].n, 3)
    np.testing.assert_array_equal(oracle.amli_cycle(h, h.L - 1, r, {}), oracle.kcycle(h, h.L - 1, r))


@pytest.mark.parametrize("N,agg", [(64, 4), (96, 16)])
def test_amli_cg_converges(N, agg):
    g = inputs.grid2d(N)
    h = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=4, agg_size=agg))
    _, coef = oracle.amli_setup(h)
    f = inputs.rhs(g.n, 5)
    res = oracle.fcg(h, f, precond=lambda r: oracle.amli_cycle(h, 0, r, coef))
    ref = oracle.fcg(h, f)
    assert res.converged and not res.breakdown
    assert res.iters <= 1.5 * ref.iters + 2
    u = np.linalg.solve(h.levels[0].dense(), f) if g.n <= 5000 else None
    if u is not None:
        e = res.x - u
        lvl = h.levels[0]
        assert np.sqrt(e @ oracle.apply_A(lvl, e)) <= 1e-7 * np.sqrt(u @ oracle.apply_A(lvl, u))


def test_positivity_threshold():
    """The degree-1 best approximation to 1/t on [a, 1] is positive at t = 1
    exactly when a > 3 - 2 sqrt(2); the interval is clamped above it."""
    thr = 3 - 2 * np.sqrt(2)
    for a in (thr - 1e-3, thr + 1e-3):
        g0, g1 = oracle.poly_coefficients(a)
        assert (g0 + g1 > 0) == (a > thr)
    from oracle.amli import A_MIN
    assert A_MIN > thr
