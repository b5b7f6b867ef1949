"""Pins for the smoother polynomial (eq. (1x-1-min) and E_m, Section 3)."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _extrema(poly, npts=400001):
    x = np.linspace(poly.lam0, poly.lam1, npts)
    e = 1.0 / x - oracle.q_eval(poly, x)
    # local extrema of the error, endpoints included
    inner = np.nonzero((np.abs(e[1:-1]) >= np.abs(e[:-2])) & (np.abs(e[1:-1]) >= np.abs(e[2:])))[0] + 1
    idx = np.unique(np.concatenate([[0], inner, [npts - 1]]))
    return x, e, idx


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 7, 9])
@pytest.mark.parametrize("ratio", [10.0, 4.0, 30.0])
def test_equioscillation(m, ratio):
    """1/x - q_m(x) attains its maximum modulus with alternating sign at m+2
    points of [lambda0, lambda1]: by Chebyshev's alternation theorem that makes
    q_m the unique best uniform approximation."""
    lam1 = 12.0
    poly = oracle.best_poly(lam1, m, ratio)
    x, e, idx = _extrema(poly)
    emax = np.max(np.abs(e))
    big = idx[np.abs(e[idx]) > emax * (1 - 1e-6)]
    signs = np.sign(e[big])
    # merge neighbouring samples of the same extremum
    alternations = 1 + int(np.sum(signs[1:] != signs[:-1]))
    assert alternations == m + 2
    # magnitude: E_m / lambda1 with E_m = delta^m (kappa - 1) / 2
    kappa = ratio
    delta = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    assert emax == pytest.approx(delta ** m * (kappa - 1) / 2 / lam1, rel=1e-9)


def _remez(lam0, lam1, m, iters=60):
    """Independent Remez exchange for the best degree-m approximation to 1/x,
    in a monomial basis of the scaled variable t in [-1, 1]."""
    theta, eta = (lam1 + lam0) / 2, (lam1 - lam0) / 2
    k = np.arange(m + 2)
    ref = np.cos(np.pi * (m + 1 - k) / (m + 1))  # Chebyshev extrema as start
    grid = np.cos(np.linspace(np.pi, 0, 200001))
    for _ in range(iters):
        xr = theta + eta * ref
        M = np.zeros((m + 2, m + 2))
        M[:, : m + 1] = ref[:, None] ** np.arange(m + 1)[None, :]
        M[:, m + 1] = (-1.0) ** k
        sol = np.linalg.solve(M, 1.0 / xr)
        coef = sol[: m + 1]
        err = 1.0 / (theta + eta * grid) - np.polyval(coef[::-1], grid)
        # new reference: one extremum per sign run
        runs = np.split(np.arange(grid.size), np.nonzero(np.diff(np.sign(err)))[0] + 1)
        pts = [r[np.argmax(np.abs(err[r]))] for r in runs if r.size]
        if len(pts) != m + 2:
            break
        new = []
        for p in pts:  # refine each extremum on a local fine grid
            lo, hi = grid[max(p - 2, 0)], grid[min(p + 2, grid.size - 1)]
            loc = np.linspace(lo, hi, 4001)
            el = 1.0 / (theta + eta * loc) - np.polyval(coef[::-1], loc)
            new.append(loc[np.argmax(np.abs(el))])
        ref = np.array(new)
    return lambda x: np.polyval(coef[::-1], (x - theta) / eta)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 7])
def test_matches_independent_remez(m):
    lam1 = 9.5
    poly = oracle.best_poly(lam1, m, 10.0)
    rem = _remez(lam1 / 10, lam1, m)
    x = np.linspace(lam1 / 10, lam1, 1001)
    np.testing.assert_allclose(oracle.q_eval(poly, x), rem(x), rtol=1e-10)


def test_degree_zero_is_midpoint():
    lam1 = 10.0
    poly = oracle.best_poly(lam1, 0, 10.0)
    assert oracle.q_eval(poly, np.array([3.0]))[0] == pytest.approx((1 / 1.0 + 1 / 10.0) / 2, rel=1e-14)


def test_Em_values_at_kappa_10():
    """E_m at lambda0 = lambda1/10 (Section 4's interval) for the degrees used;
    the stored values are the paper's closed form delta^m (kappa-1)/2."""
    with open(os.path.join(GOLDEN, "em_kappa10.json")) as fh:
        gold = json.load(fh)
    for m_str, val in gold["E_m"].items():
        m = int(m_str)
        assert oracle.error_Em(m, 10.0) == pytest.approx(val, abs=5e-5)
        poly = oracle.best_poly(7.0, m, 10.0)
        x = np.linspace(0.7, 7.0, 200001)
        # E_m is attained at x = lambda1 (a point of Chebyshev alternance)
        r = oracle.residual_poly_eval(poly, x)
        assert np.max(np.abs(r)) == pytest.approx(val, abs=5e-5)
        assert abs(r[-1]) == pytest.approx(np.max(np.abs(r)), rel=1e-12)
    # degree 4 (the paper's choice) is the smallest with damping below 1/2
    assert oracle.error_Em(4, 10.0) < 0.5 < oracle.error_Em(3, 10.0)


@pytest.mark.parametrize("m", [3, 4, 5, 7])
def test_smoother_contracts_on_whole_spectrum(m):
    """With E_m < 1, |1 - x q_m(x)| <= 1 on [0, lambda1] and q_m > 0 there."""
    poly = oracle.best_poly(12.0, m, 10.0)
    x = np.linspace(0.0, 12.0, 100001)
    assert np.all(np.abs(oracle.residual_poly_eval(poly, x)) <= 1.0 + 1e-12)
    assert np.all(oracle.q_eval(poly, x) > 0)


def test_degree_two_diverges():
    """E_2 > 1 at kappa = 10: the A-norm contraction fails (reject m = 2)."""
    assert oracle.error_Em(2, 10.0) > 1.0
    g = __import__("inputs").grid2d(8)
    with pytest.raises(ValueError):
        oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=2))


def test_degree_for_matches_the_bound_on_m():
    """Automatic degree: the smallest m with E_m <= rho and E_m < 1.  Pinned
    against the closed form of Section 3's bound on m, with the positivity
    term read in consistent units (lambda1 -> 1):
    m = ceil(max(|ln(2 rho/(kappa-1))|, |ln(2/(kappa-1))|) / |ln delta|)."""
    for kappa in (10.0, 30.0, 100.0):
        delta = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
        for rho in (0.9, 0.6, 0.33, 0.2, 0.1, 0.05, 0.01, 1e-3):
            bound = max(abs(math.log(2 * rho / (kappa - 1))), abs(math.log(2 / (kappa - 1)))) / abs(math.log(delta))
            assert oracle.degree_for(rho, kappa) == math.ceil(bound), (kappa, rho)
    # Section 4: kappa = 10 and m = 4; the damping factors of the neighbouring degrees
    assert oracle.degree_for(0.33, 10.0) == 4
    assert oracle.degree_for(0.64, 10.0) == 3
    assert oracle.degree_for(0.2, 10.0) == 5
    assert oracle.degree_for(0.05, 10.0) == 7
    # rho = 1: only E_m < 1 binds, and m = 2 diverges at kappa = 10
    assert oracle.degree_for(1.0, 10.0) == 3
