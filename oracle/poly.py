"""Polynomial smoother of Section 3 -- oracle (test infrastructure only).

q_m is the polynomial of degree m of best uniform approximation to 1/x on
[lambda0, lambda1] (eq. (1x-1-min)), with lambda1 = ||A||_inf (an upper bound on
rho(A)) and, in the experiments of Section 4, lambda0 = lambda1 / 10.

The paper leaves how the coefficients are built (by a recurrence) to its
reference on polynomial smoothers.  Reading taken here:
Chebyshev's classical solution.  With theta = (lambda1+lambda0)/2,
eta = (lambda1-lambda0)/2, t = (x - theta)/eta and a = theta/eta = (k+1)/(k-1)
(k = lambda1/lambda0), 1/x = (1/eta) / (t + a), and with
delta = a - sqrt(a^2-1) = (sqrt(k)-1)/(sqrt(k)+1):

    1/(t+a) = 2 delta/(1-delta^2) T_0(t) + sum_{k>=1} 4 delta (-delta)^k/(1-delta^2) T_k(t).

The best approximation of degree m keeps the first m terms of this expansion
and replaces the coefficient of T_m by 4 delta (-delta)^m / (1-delta^2)^2; the
error 1/(t+a) - p(t) then equioscillates at m+2 points of [-1,1] with magnitude
4 delta^(m+2)/(1-delta^2)^2 = delta^m/(a^2-1), so by Chebyshev's alternation
theorem p is the unique best approximation (the tests check the alternation
and compare with an independent Remez exchange).  For m = 0 the best constant
is the midpoint (1/lambda0 + 1/lambda1)/2.

The error of Section 3: E_m = max |1 - x q_m(x)| = delta^m (k-1)/2, attained at
x = lambda1.  The paper's positivity condition "1/lambda1 - E_m > 0" mixes units
unless lambda1 = 1; the consistent condition is that the approximation error
E_m/lambda1 be smaller than 1/lambda1, i.e. E_m < 1, which is also what makes
|1 - x q_m(x)| <= 1 on the spectrum (A-norm convergent smoother).  That is the
condition validated here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .level import Level, row_abs_sums


@dataclass
class SmootherPoly:
    lam0: float
    lam1: float
    theta: float
    eta: float
    c: np.ndarray  # Chebyshev coefficients c_0..c_m of eta*q_m in the variable t

    @property
    def m(self) -> int:
        return int(self.c.shape[0]) - 1


def lambda_max_bound(lvl: Level) -> float:
    """lambda1 = ||A||_inf = max_i (D_i + sum_j W_ij)."""
    return float(np.max(row_abs_sums(lvl)))


def _delta(kappa: float) -> float:
    sk = math.sqrt(kappa)
    return (sk - 1.0) / (sk + 1.0)


def best_poly(lam1: float, m: int, ratio: float = 10.0) -> SmootherPoly:
    """Coefficients of q_m on [lam1/ratio, lam1] (module doc)."""
    lam0 = lam1 / ratio
    theta = 0.5 * (lam1 + lam0)
    eta = 0.5 * (lam1 - lam0)
    kappa = lam1 / lam0
    dl = _delta(kappa)
    one_m = 1.0 - dl * dl
    c = np.zeros(m + 1)
    if m == 0:
        c[0] = 2.0 * dl * (1.0 + dl * dl) / (one_m * one_m)
    else:
        c[0] = 2.0 * dl / one_m
        for k in range(1, m):
            c[k] = 4.0 * dl * (-dl) ** k / one_m
        c[m] = 4.0 * dl * (-dl) ** m / (one_m * one_m)
    return SmootherPoly(lam0, lam1, theta, eta, c)


def error_Em(m: int, kappa: float) -> float:
    """E_m = delta^m (kappa - 1) / 2 (Section 3)."""
    return _delta(kappa) ** m * (kappa - 1.0) / 2.0


def degree_for(rho: float, kappa: float, max_degree: int = 64) -> int:
    """Smallest degree m meeting the bound on m of Section 3: a damping factor
    E_m <= rho on [lambda0, lambda1] and E_m < 1 (the positivity condition read
    with consistent units, see the module docstring).  E_m decreases in m, so
    this is the first m that passes both tests."""
    for m in range(max_degree + 1):
        e = error_Em(m, kappa)
        if e <= rho and e < 1.0:
            return m
    return max_degree


def q_eval(poly: SmootherPoly, x: np.ndarray) -> np.ndarray:
    """q_m(x) evaluated through the Chebyshev series (numpy's chebval)."""
    t = (np.asarray(x, dtype=np.float64) - poly.theta) / poly.eta
    return np.polynomial.chebyshev.chebval(t, poly.c) / poly.eta


def residual_poly_eval(poly: SmootherPoly, x: np.ndarray) -> np.ndarray:
    """1 - x q_m(x)."""
    x = np.asarray(x, dtype=np.float64)
    return 1.0 - x * q_eval(poly, x)
