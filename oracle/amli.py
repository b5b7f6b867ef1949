"""Stationary AMLI cycle (the "AMLI" column of Section 4) -- oracle (test
infrastructure only).

Section 4 compares the nonlinear cycle with the stationary AMLI cycle, in which
the correction between two successive levels is a fixed polynomial in the
preconditioned coarse operator, built from the best uniform approximation to
1/x (the construction of Section 3, through the reference it defers to), and the
outer iteration is CG.  The paper gives neither the polynomial's degree nor the
interval it approximates on; readings taken here:

* W-cycle (nu = 2): on level l < L-1 the coarse correction is
  e = p(B_{l+1} A_{l+1}) B_{l+1} b, p the degree-1 best uniform approximation to
  1/t on [a_{l+1}, 1] (Section 3's closed form with lambda1 = 1,
  lambda0 = a_{l+1}), written p(t) = g0 + g1 t, so
  e = g0 y0 + g1 B_{l+1}(A_{l+1} y0) with y0 = B_{l+1} b: two recursive cycles,
  as in the nonlinear cycle.  Directly above the coarsest level the exact
  solve is used.  Smoothing, restriction and prolongation are those of the
  k-cycle.
* a_l estimates the smallest eigenvalue of B_l A_l: power iteration on
  I - B_l A_l in the A_l inner product, `AMLI_POWER_ITERS` steps, a = 1 - the
  last Rayleigh quotient, clamped to [0.18, 0.99]: the degree-1 best
  approximation is positive on (0, 1] only for a > 3 - 2 sqrt(2) = 0.1716, and
  CG needs the cycle to stay positive definite (for t < a the polynomial is
  larger still, so a clamped interval keeps it positive on the whole spectrum).  Levels are treated from the
  coarsest up (B_l needs a_{l+1}).  If the iterate w = (I - B_l A_l) v has no
  positive A-norm (it vanishes when the cycle solves v's equation exactly) the
  iteration stops with the quotient it has: there is nothing left to power.  The start vector is counter-based:
  v_i = 2 u(splitmix64(2^40 l + i)) - 1 with u(z) = (z >> 11) 2^-53, splitmix64
  as published by Steele, Lea and Flood (one output of the generator whose
  state is the argument).
* Outer iteration: the flexible CG of the nonlinear cycle; with this fixed
  symmetric positive definite preconditioner it produces the CG iterates (the
  extra orthogonalization terms vanish in exact arithmetic).
"""
from __future__ import annotations

import math

import numpy as np

from .cycle import Hierarchy, coarse_solve, prolong, residual, restrict, smooth
from .level import apply_A
from .poly import best_poly

from .rng import splitmix64

AMLI_POWER_ITERS = 20
A_MIN, A_MAX = 0.18, 0.99


def start_vector(level: int, n: int) -> np.ndarray:
    base = level << 40
    return np.array([2.0 * ((splitmix64(base + i) >> 11) * 2.0 ** -53) - 1.0 for i in range(n)])


def poly_coefficients(a: float) -> tuple[float, float]:
    """(g0, g1) of the degree-1 best uniform approximation to 1/t on [a, 1]."""
    p = best_poly(1.0, 1, 1.0 / a)
    c0, c1 = float(p.c[0]), float(p.c[1])
    return (c0 - c1 * p.theta / p.eta) / p.eta, c1 / p.eta ** 2


def amli_cycle(h: Hierarchy, l: int, r: np.ndarray, coef: dict) -> np.ndarray:
    """B_l r for the AMLI cycle; coef[l'] = (g0, g1) for the levels below l."""
    if l == h.L:
        return coarse_solve(h.chol, r)
    lvl, poly, agg = h.levels[l], h.polys[l], h.aggs[l]
    nc = h.levels[l + 1].n
    x = smooth(lvl, poly, r)
    s = residual(lvl, r, x)
    b = restrict(agg, nc, s)
    if l + 1 == h.L:
        e = coarse_solve(h.chol, b)
    else:
        g0, g1 = coef[l + 1]
        y0 = amli_cycle(h, l + 1, b, coef)
        y1 = amli_cycle(h, l + 1, apply_A(h.levels[l + 1], y0), coef)
        e = g0 * y0 + g1 * y1
    x = x + prolong(agg, e)
    s = residual(lvl, r, x)
    return x + smooth(lvl, poly, s)


def estimate_lambda_min(h: Hierarchy, l: int, coef: dict, iters: int = AMLI_POWER_ITERS) -> float:
    """Smallest eigenvalue of B_l A_l by power iteration on I - B_l A_l."""
    lvl = h.levels[l]
    v = start_vector(l, lvl.n)
    mu = 0.0
    for _ in range(iters):
        Av = apply_A(lvl, v)
        w = v - amli_cycle(h, l, Av, coef)
        Aw = apply_A(lvl, w)
        mu = float(np.dot(w, Av)) / float(np.dot(v, Av))
        ww = float(np.dot(w, Aw))
        if not (ww > 0.0 and math.isfinite(ww)):
            break
        v = w / math.sqrt(ww)
    return 1.0 - mu


def amli_setup(h: Hierarchy, iters: int = AMLI_POWER_ITERS):
    """(a, coef): a[l] and coef[l] = (g0, g1) for 1 <= l <= L-1, coarsest first."""
    a, coef = {}, {}
    for l in range(h.L - 1, 0, -1):
        est = estimate_lambda_min(h, l, coef, iters)
        a[l] = min(max(est, A_MIN), A_MAX)
        coef[l] = poly_coefficients(a[l])
    return a, coef
