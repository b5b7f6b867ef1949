"""The operator of eq. (prob), Section 1 -- oracle (test infrastructure only).

(Au, v) = sum_{e=(i,j)} w_e (u_i - u_j)(v_i - v_j) + sum_{i in S_b} d_i u_i v_i.

Expanding the edge sum gives A = L_w + diag(d) with L_w the weighted graph
Laplacian: off-diagonal entries -w_ij and diagonal D_i = d_i + sum_j w_ij.  A
level is stored as the off-diagonal weights W (symmetric CSR, both directions,
columns increasing, no self loops) plus d and D.

Summation order (the paper gives none): D_i is accumulated sequentially,
starting from d_i and adding W_ij in increasing column order.  The GPU path uses
the same order so that values, and the matching keys built from them, agree bit
for bit.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Level:
    n: int
    row_ptr: np.ndarray  # int64, n+1
    col: np.ndarray  # int64, nnz
    W: np.ndarray  # float64, nnz (off-diagonal weights, positive)
    d: np.ndarray  # float64, n (lower-order terms, zero off S_b)
    D: np.ndarray  # float64, n (diagonal of A)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (CSR order)."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def W_csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.W, self.col, self.row_ptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        A = -self.W_csr().toarray()
        A[np.diag_indices(self.n)] = self.D
        return A


def _sequential_row_sum(start: np.ndarray, row_ptr: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """start_i + vals[row_ptr[i]] + vals[row_ptr[i]+1] + ..., added left to right."""
    acc = np.array(start, dtype=np.float64, copy=True)
    deg = np.diff(row_ptr)
    for k in range(int(deg.max()) if deg.size else 0):
        r = np.nonzero(deg > k)[0]
        acc[r] += vals[row_ptr[r] + k]
    return acc


def assemble(n, row_ptr, col, w, d) -> Level:
    """A = L_w + diag(d) from eq. (prob): D_i = d_i + sum_j w_ij (sequential)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    W = np.asarray(w, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    D = _sequential_row_sum(d, row_ptr, W)
    return Level(int(n), row_ptr, col, W, d.copy(), D)


def apply_A(lvl: Level, u: np.ndarray) -> np.ndarray:
    """(Au)_i = D_i u_i - sum_j W_ij u_j."""
    return lvl.D * u - lvl.W_csr() @ u


def row_abs_sums(lvl: Level) -> np.ndarray:
    """Row sums of |A|: D_i + sum_j W_ij (sequential, starting from D_i)."""
    return _sequential_row_sum(lvl.D, lvl.row_ptr, lvl.W)


def bilinear_form(n, row_ptr, col, w, d, u, v) -> float:
    """(Au, v) summed straight from eq. (prob): one term per undirected edge
    (i < j) plus the lower-order terms.  Plain loops; tiny graphs only."""
    total = 0.0
    for i in range(n):
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            j = int(col[k])
            if j > i:
                total += w[k] * (u[i] - u[j]) * (v[i] - v[j])
    for i in range(n):
        if d[i] != 0.0:
            total += d[i] * u[i] * v[i]
    return total
