"""Pins for the aggregation of Section 2 as the paper's experiments use it
(maximal independent set on the graph of A^k, then neighbour collection) and
for pure Neumann problems (oracle; readings in oracle/aggregation.py and
oracle/cycle.py)."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, shortest_path

import inputs
import oracle
from oracle.aggregation import distance_k_mis, mis_aggregate, mis_keys, nearest_owner

GRAPHS = [
    lambda: inputs.poisson2d(17),
    lambda: inputs.grid2d(13, 11),
    lambda: inputs.poisson3d(7),
    lambda: inputs.rgg(700, seed=4),
    lambda: inputs.random_graph(120, 0.04, seed=8, weighted=True),
]


def _level(g):
    return oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)


def _hops(lvl):
    A = csr_matrix((np.ones(lvl.nnz), lvl.col, lvl.row_ptr), shape=(lvl.n, lvl.n))
    return shortest_path(A, unweighted=True, directed=False)


def _rounds_mis(lvl, k):
    """The parallel form: in each round an undecided vertex joins when its key is
    the largest among the undecided vertices within distance k and no member is
    that close (Blelloch, Fineman and Shun: the same set as the greedy one)."""
    keys = mis_keys(lvl.n)
    rows = lvl.rows()
    state = np.zeros(lvl.n, dtype=np.int8)
    while np.any(state == 0):
        mx = np.where(state == 0, keys, np.uint64(0))
        near = state == 1
        for _ in range(k):
            m2, n2 = mx.copy(), near.copy()
            np.maximum.at(m2, rows, mx[lvl.col])
            np.logical_or.at(n2, rows, near[lvl.col])
            mx, near = m2, n2
        und = state == 0
        state[und & near] = 2
        state[und & ~near & (mx == keys)] = 1
    return np.nonzero(state == 1)[0]


@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("k", [1, 2, 4])
def test_mis_independent_maximal_greedy(make, k):
    g = make()
    lvl = _level(g)
    S = distance_k_mis(lvl, k)
    D = _hops(lvl)
    sub = D[np.ix_(S, S)]
    assert np.all(sub[~np.eye(len(S), dtype=bool)] > k)          # independent in the graph of A^k
    assert np.all(D[:, S].min(axis=1) <= k)                       # maximal
    np.testing.assert_array_equal(S, _rounds_mis(lvl, k))         # schedule-free


def test_mis_on_a_path_in_key_order():
    """Closed form: on a path that visits the vertices in decreasing priority,
    the greedy set is every (k+1)-th vertex of the path."""
    n, k = 40, 4
    keys = mis_keys(n)
    pi = np.argsort(keys)[::-1]
    g = inputs.Graph(n, *inputs.csr_from_edges(n, pi[:-1], pi[1:]), np.zeros(n))
    S = distance_k_mis(_level(g), k)
    np.testing.assert_array_equal(S, np.sort(pi[::k + 1]))


@pytest.mark.parametrize("make", GRAPHS)
def test_nearest_owner_and_connected_aggregates(make):
    g = make()
    lvl = _level(g)
    S = distance_k_mis(lvl, 4)
    owner = nearest_owner(lvl, S)
    D = _hops(lvl)
    dmin = D[:, S].min(axis=1)
    assert np.all(D[np.arange(lvl.n), owner] == dmin)             # a nearest set vertex
    # ties between set vertices at the same distance go to the smallest index
    # (brute force over the all-pairs hop distances)
    Sa = np.asarray(S)
    ties = 0
    for v in range(lvl.n):
        cand = Sa[D[v, Sa] == dmin[v]]
        ties += len(cand) > 1
        assert owner[v] == cand.min()
    if not g.name.startswith("random"):  # meshes and geometric graphs have equidistant set vertices
        assert ties > 0
    ids, nc = mis_aggregate(lvl, 4)
    assert nc == len(S) and set(np.unique(ids)) == set(range(nc))
    A = csr_matrix((np.ones(lvl.nnz), lvl.col, lvl.row_ptr), shape=(lvl.n, lvl.n))
    for I in range(nc):
        m = np.nonzero(ids == I)[0]
        assert connected_components(A[m][:, m], directed=False)[0] == 1


def test_aggressive_coarsening_rate():
    """Section 4 reports about 30x per level with k = 4: on the 5-point grid the
    level sizes shrink by about 20x first, then by about 28x."""
    g = inputs.poisson2d(96)
    h = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(aggregation="mis", coarse_max=100))
    ratios = [a.n / b.n for a, b in zip(h.levels[:-1], h.levels[1:])]
    assert 15 < ratios[0] < 30 and all(15 < r < 40 for r in ratios)
    assert h.grid_complexity() < 1.07


@pytest.mark.parametrize("make,kw", [
    (lambda: inputs.poisson2d(48), dict(aggregation="mis", coarse_max=100)),
    (lambda: inputs.poisson3d(12), dict(aggregation="mis", coarse_max=100)),
    (lambda: inputs.poisson2d(40), dict(agg_size=4)),
])
def test_neumann_solve(make, kw):
    """Pure Neumann: with f orthogonal to 1 the solve converges to a solution of
    A u = f (A singular), the minimum-norm one up to a constant."""
    g = make()
    h = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(**kw))
    f = inputs.project_range(inputs.rhs(g.n, 9))
    res = oracle.fcg(h, f)
    assert res.converged
    lvl = h.levels[0]
    assert np.linalg.norm(f - oracle.apply_A(lvl, res.x)) <= 1e-8 * np.linalg.norm(f)
    u = np.linalg.lstsq(lvl.dense(), f, rcond=None)[0]
    e = (res.x - res.x.mean()) - (u - u.mean())
    assert np.sqrt(e @ oracle.apply_A(lvl, e)) <= 1e-7 * np.sqrt(u @ oracle.apply_A(lvl, u))
    # the coarsest "inverse" is the pseudo-inverse on range(A_L)
    AL = h.levels[-1].dense()
    b = inputs.project_range(inputs.rhs(AL.shape[0], 10))
    x = oracle.coarse_solve(h.chol, b)
    np.testing.assert_allclose(AL @ x, b, atol=1e-10 * np.linalg.norm(b))
    assert abs(x.sum()) <= 1e-10 * np.linalg.norm(x) * AL.shape[0]
