"""CPU FP64 oracle of the paper's solve phase -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library behind
``include/amg.h`` and its Python binding) never imports, links or calls it, and
this package never imports the product path: the two share no code, no
constants and no helpers.  Only the seeded problem generators in ``inputs``
serve both, and those hold none of the method's arithmetic.

What is computed, and where in the paper it comes from
(Brannick, "Aggregation-based aggressive coarsening with polynomial smoothing"):

* ``level``      -- the operator A of eq. (prob), Section 1: (Au,v) = sum_e w_e
                    d_e u d_e v + sum_{S_b} d_i u_i v_i, stored as off-diagonal
                    weights W and diagonal D_i = d_i + sum_j W_ij.
* ``aggregation``-- the matching-based graph partitioning of Section 2 (a
                    matching is the simplest partition into connected
                    subgraphs), the quotient graph of Section 2 and the Galerkin
                    operator A_H = P^T A P of Section 3, computed as the summation
                    of fine entries that the conclusion describes.
* ``poly``       -- the smoother interval [lambda0, lambda1] with lambda1 = the
                    l-infinity norm of A (Section 3 and Section 4), the best
                    uniform polynomial approximation q_m to 1/x of eq. (1x-1-min),
                    and its error E_m (Section 3).
* ``cycle``      -- the smoother application q_m(A)v, the coarsest-level
                    Cholesky solve, the nonlinear AMLI (k-cycle) preconditioner
                    and the flexible CG used as outer and inner iteration
                    (Section 4, the W(1,1) cycle of Table 1).
* ``spectral``   -- dense two-level objects of Section 3 (E_TL, the symmetrized
                    two-level preconditioner B, the weak approximation constant
                    c_p of eq. (wap)) for tiny graphs.

Every floating-point value is IEEE binary64 (numpy float64).  Where the paper is
silent, ambiguous or garbled, the reading taken is stated in the docstring of
the function that takes it.

Parity status: every function above is pinned by a test in ``tests/`` against
something other than itself (closed forms, dense eigensolves, library solves,
brute force on tiny graphs, an independent handshake matching); the exact outer
iteration counts of Table 1 are "parity unpinned" (different aggregation,
boundary terms and weights than the configurations built here).
"""
from .level import Level, assemble, apply_A, bilinear_form, row_abs_sums
from .aggregation import (
    edge_strengths,
    greedy_matching,
    coarse_ids,
    quotient,
    aggregate_level,
    mis_keys,
    distance_k_mis,
    nearest_owner,
    mis_aggregate,
)
from .poly import SmootherPoly, lambda_max_bound, best_poly, error_Em, degree_for, q_eval, residual_poly_eval
from .cycle import (
    Params,
    Hierarchy,
    build_hierarchy,
    smooth,
    residual,
    restrict,
    prolong,
    coarse_solve,
    kcycle,
    fcg,
    FCGResult,
)
from .amli import amli_cycle, amli_setup, estimate_lambda_min, poly_coefficients, splitmix64, start_vector

__all__ = [
    "Level", "assemble", "apply_A", "bilinear_form", "row_abs_sums",
    "edge_strengths", "greedy_matching", "coarse_ids", "quotient", "aggregate_level",
    "mis_keys", "distance_k_mis", "nearest_owner", "mis_aggregate",
    "SmootherPoly", "lambda_max_bound", "best_poly", "error_Em", "degree_for", "q_eval", "residual_poly_eval",
    "Params", "Hierarchy", "build_hierarchy", "smooth", "residual", "restrict", "prolong",
    "coarse_solve", "kcycle", "fcg", "FCGResult",
    "amli_cycle", "amli_setup", "estimate_lambda_min", "poly_coefficients", "splitmix64", "start_vector",
]
