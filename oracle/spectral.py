"""Dense two-level objects of Section 3 for tiny graphs -- oracle (test
infrastructure only).

* P: n x n_H with indicator columns 1_l of the aggregates (coarse space V_H of
  eq. (coarse)); Q = P (P^T P)^{-1} P^T, the l2 projection of eq. (Q).
* R = q_m(A) (dense, through an eigendecomposition of A).
* Two-level error operator E_TL = (I - RA)(I - pi_A), pi_A = P A_H^+ P^T A.
* Symmetrized preconditioner B = R_bar + (I-RA) P A_H^+ P^T (I-AR),
  R_bar = 2R - RAR.
* Weak approximation constant c_p = max_l 1/lambda_l over the aggregates, with
  lambda_l the second eigenvalue (the first nonzero one, G_l being connected)
  of the Laplacian of the aggregate's induced subgraph G_l (eq. (wap));
  singleton aggregates contribute nothing (v - Qv vanishes on them).
"""
from __future__ import annotations

import numpy as np

from .level import Level
from .poly import SmootherPoly, q_eval


def prolongator(agg: np.ndarray, nc: int) -> np.ndarray:
    P = np.zeros((agg.shape[0], nc))
    P[np.arange(agg.shape[0]), agg] = 1.0
    return P


def l2_projection(agg: np.ndarray, nc: int) -> np.ndarray:
    P = prolongator(agg, nc)
    return P @ np.linalg.inv(P.T @ P) @ P.T


def smoother_matrix(A: np.ndarray, poly: SmootherPoly) -> np.ndarray:
    lam, V = np.linalg.eigh(A)
    return (V * q_eval(poly, lam)) @ V.T


def two_level(A: np.ndarray, P: np.ndarray, R: np.ndarray):
    """(E_TL, B) of Section 3."""
    n = A.shape[0]
    I = np.eye(n)
    AH = P.T @ A @ P
    AHp = np.linalg.pinv(AH)
    piA = P @ AHp @ P.T @ A
    E = (I - R @ A) @ (I - piA)
    Rbar = 2 * R - R @ A @ R
    B = Rbar + (I - R @ A) @ P @ AHp @ P.T @ (I - A @ R)
    return E, B


def local_cp(lvl: Level, agg: np.ndarray) -> float:
    """c_p = max over aggregates with >= 2 vertices of 1/lambda_l (eq. (wap))."""
    nc = int(agg.max()) + 1
    W = lvl.W_csr().toarray()
    worst = 0.0
    for l in range(nc):
        mem = np.nonzero(agg == l)[0]
        if mem.size < 2:
            continue
        Wl = W[np.ix_(mem, mem)]
        Ll = np.diag(Wl.sum(axis=1)) - Wl
        ev = np.linalg.eigvalsh(Ll)
        lam = ev[1]  # smallest positive eigenvalue of a connected subgraph Laplacian
        worst = max(worst, 1.0 / lam)
    return worst
