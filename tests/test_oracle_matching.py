"""Pins for the oracle's matching aggregation (Section 2) and coarse numbering.

The greedy matching in a strict total edge order is the unique matching that
every locally-dominant (handshake) scheme produces under the same order; the
GPU path relies on that.  An independent handshake written here, in plain
Python, must agree with the oracle's greedy scan on random graphs.
"""
import numpy as np
import pytest

import inputs
import oracle
from oracle.aggregation import edge_strengths


def murmur_fmix32(a, b):
    """Written here from MurmurHash3's published 32-bit finalizer, on
    x = a * 2654435761 + b (mod 2^32), independently of the oracle's numpy
    version."""
    x = (a * 2654435761 + b) % (1 << 32)
    x ^= x >> 16
    x = (x * 0x85EBCA6B) % (1 << 32)
    x ^= x >> 13
    x = (x * 0xC2B2AE35) % (1 << 32)
    x ^= x >> 16
    return x


def handshake_matching(lvl, key, tie="index"):
    """Rounds of: every free vertex points at its best free neighbour; mutual
    pointers become matched.  Stops when no free vertex has a free neighbour."""
    n = lvl.n
    i, j, s = edge_strengths(lvl, key)
    nbrs = [[] for _ in range(n)]
    for a, b, sv in zip(i.tolist(), j.tolist(), s.tolist()):
        k = (-sv, a, b) if tie == "index" else (-sv, murmur_fmix32(a, b), a, b)
        nbrs[a].append((k, b))
        nbrs[b].append((k, a))
    mate = [-1] * n
    alive = [True] * n
    while True:
        cand = [-1] * n
        for v in range(n):
            if mate[v] >= 0 or not alive[v]:
                continue
            best = None
            for k, u in nbrs[v]:
                if mate[u] < 0 and alive[u] and (best is None or k < best[0]):
                    best = (k, u)
            if best is None:
                alive[v] = False
            else:
                cand[v] = best[1]
        changed = False
        for v in range(n):
            u = cand[v]
            if u >= 0 and cand[u] == v and v < u:
                mate[v], mate[u] = u, v
                changed = True
        if not changed:
            break
    return np.asarray(mate)


def _level(g):
    return oracle.assemble(g.n, g.row_ptr, g.col, g.w, g.d)


@pytest.mark.parametrize("seed", range(40))
@pytest.mark.parametrize("key", ["normalized", "raw"])
def test_greedy_equals_handshake(seed, key):
    g = inputs.random_graph(20 + seed % 17, 0.08 + 0.01 * (seed % 7), seed=seed, weighted=seed % 2 == 0)
    lvl = _level(g)
    assert np.array_equal(oracle.greedy_matching(lvl, key), handshake_matching(lvl, key))


def test_greedy_equals_handshake_on_grid_ties():
    for g in (inputs.grid2d(11, 8), inputs.tet3d(4), inputs.delaunay3d(6, 4)):
        lvl = _level(g)
        for key in ("normalized", "raw"):
            for tie in ("index", "hash"):
                assert np.array_equal(oracle.greedy_matching(lvl, key, tie), handshake_matching(lvl, key, tie))


@pytest.mark.parametrize("seed", range(12))
def test_greedy_equals_handshake_hash_ties(seed):
    g = inputs.random_graph(25 + seed, 0.1, seed=100 + seed, weighted=False)  # unit weights: many ties
    lvl = _level(g)
    for key in ("normalized", "raw"):
        assert np.array_equal(oracle.greedy_matching(lvl, key, "hash"), handshake_matching(lvl, key, "hash"))


def test_tie_hash_known_values_and_spread():
    # fmix32 maps 0 to 0 and is a bijection on 32-bit words; on the edges of a grid
    # the hashes are (almost) all distinct, which is what breaks the index chains
    from oracle.aggregation import tie_hash
    assert int(tie_hash(np.array([0]), np.array([0]))[0]) == 0
    i = np.arange(0, 5000)
    j = i + 1
    h = tie_hash(i, j)
    assert [int(x) for x in h[:64]] == [murmur_fmix32(int(a), int(b)) for a, b in zip(i[:64], j[:64])]
    assert len(np.unique(h)) == len(h)


def test_hash_ties_need_fewer_rounds_on_grids():
    # index ties chain along the grid (rounds grow with the side); hashed ties do not
    def rounds(lvl, tie):
        n = lvl.n
        i, j, s = edge_strengths(lvl, "normalized")
        keys = {}
        nbrs = [[] for _ in range(n)]
        for a, b, sv in zip(i.tolist(), j.tolist(), s.tolist()):
            k = (-sv, a, b) if tie == "index" else (-sv, murmur_fmix32(a, b), a, b)
            nbrs[a].append((k, b))
            nbrs[b].append((k, a))
        free = [True] * n
        r = 0
        while True:
            r += 1
            cand = {}
            for v in range(n):
                if free[v]:
                    opts = [(k, u) for k, u in nbrs[v] if free[u]]
                    if opts:
                        cand[v] = min(opts)[1]
            pairs = [(v, u) for v, u in cand.items() if cand.get(u) == v and v < u]
            if not pairs:
                return r
            for v, u in pairs:
                free[v] = free[u] = False
    lvl = _level(inputs.grid2d(40))
    assert rounds(lvl, "hash") * 3 < rounds(lvl, "index")


@pytest.mark.parametrize("seed", range(10))
def test_matching_valid_and_maximal(seed):
    g = inputs.random_graph(60, 0.05, seed=100 + seed, weighted=True)
    lvl = _level(g)
    mate = oracle.greedy_matching(lvl)
    rows = lvl.rows()
    adj = set(zip(rows.tolist(), lvl.col.tolist()))
    for v, u in enumerate(mate.tolist()):
        if u >= 0:
            assert mate[u] == v and (v, u) in adj
    free = mate < 0
    assert not np.any(free[rows] & free[lvl.col])  # maximal


def test_coarse_ids_smallest_member_order():
    g = inputs.random_graph(50, 0.1, seed=7)
    lvl = _level(g)
    mate = oracle.greedy_matching(lvl)
    ids, nc = oracle.coarse_ids(mate)
    first = [min(np.nonzero(ids == I)[0]) for I in range(nc)]
    assert first == sorted(first)
    assert set(ids.tolist()) == set(range(nc))
    sizes = np.bincount(ids)
    assert sizes.max() <= 2


def _block_ids(N):
    r, c = np.divmod(np.arange(N * N), N)
    return (r // 2) * (N // 2) + c // 2


def test_raw_key_structured_grid_closed_form():
    """Raw-weight key on a 2^k x 2^k triangulated grid: pass 1 pairs horizontal
    neighbours, pass 2 pairs vertical neighbours, i.e. 2x2 blocks; the coarse
    graph is again a triangulated grid with axis weight 2s+1 (s the fine axis
    weight) and diagonal weight 1."""
    g = inputs.grid2d(64)
    lvl = _level(g)
    s = 1.0
    N = 64
    while N > 8:
        mate = oracle.greedy_matching(lvl, "raw")
        idx = np.arange(N * N)
        assert np.array_equal(mate, np.where(idx % 2 == 0, idx + 1, idx - 1))
        agg, coarse = oracle.aggregate_level(lvl, 2, "raw")
        assert np.array_equal(agg, _block_ids(N))
        N //= 2
        assert coarse.n == N * N
        ref = inputs.grid2d(N)
        assert np.array_equal(coarse.row_ptr, ref.row_ptr)
        assert np.array_equal(coarse.col, ref.col)
        rows = coarse.rows()
        dr = np.abs(coarse.col // N - rows // N)
        dc = np.abs(coarse.col % N - rows % N)
        diag = (dr == 1) & (dc == 1)
        assert np.all(coarse.W[diag] == 1.0)
        assert np.all(coarse.W[~diag] == 2 * s + 1)
        s = 2 * s + 1
        lvl = coarse


def test_config1_level_sizes():
    """64x64 grid, aggregates of 4 (two passes), coarsen to <= 64 vertices."""
    g = inputs.grid2d(64)
    h = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=3, agg_size=4))
    assert [l.n for l in h.levels] == [4096, 1026, 264, 77, 23]
    hr = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d,
                                oracle.Params(degree=3, agg_size=4, match_key="raw"))
    assert [l.n for l in hr.levels] == [4096, 1024, 256, 64]


def test_aggregates_connected():
    g = inputs.rgg(3000, seed=5)
    lvl = _level(g)
    agg, coarse = oracle.aggregate_level(lvl, 3)
    rows = lvl.rows()
    same = agg[rows] == agg[lvl.col]
    # union-find over intra-aggregate edges: every aggregate is one component
    parent = np.arange(lvl.n)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in zip(rows[same].tolist(), lvl.col[same].tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    roots = {}
    for v in range(lvl.n):
        roots.setdefault(agg[v], set()).add(find(v))
    assert all(len(s) == 1 for s in roots.values())
