"""Matching-based aggregation and the Galerkin coarse operator -- oracle
(test infrastructure only).

Section 2 of the paper defines a graph partitioning as disjoint, non-empty,
connected subgraphs covering V, names a matching (a set of pairwise non-incident
edges) as its simplest non-trivial example, and defines the coarse graph as the
quotient of G under "same subgraph".  Section 3 uses the piecewise-constant
coarse space, so P has indicator columns and A_H = P^T A P; the conclusion notes
that this triple product reduces to summations of fine-level entries.

Readings taken where the paper is silent (the paper's own experiments aggregate
with a maximal independent set on the graph of A^4, Section 4; the workloads
built here use matching passes by default, and the MIS aggregation of Section 2
is the option at the end of this module):

* Edge strength.  ``normalized`` (default): s_ij = W_ij^2 / (D_i D_j), evaluated
  as the correctly rounded products W_ij*W_ij and D_i*D_j followed by one
  correctly rounded division -- no square root, no fused multiply-add.  ``raw``:
  s_ij = W_ij.
* Tie-breaking.  Edges (i < j) are totally ordered by the key (-s_ij, i, j),
  ascending ("index" ties, the default); the matching is the greedy one that
  scans edges in that order and takes an edge when both endpoints are still
  free.  This is the matching that every locally-dominant (handshake) algorithm
  produces under the same strict order, so it does not depend on how the work
  is scheduled.  "hash" ties order equal strengths by a fixed hash of the
  endpoints first, key (-s_ij, h(i, j), i, j) with h = the 32-bit finalizer of
  MurmurHash3 applied to (i * 2654435761 + j) mod 2^32 (see ``tie_hash``).
* Unmatched vertices stay singleton aggregates.
* Coarse numbering: rep(i) = min(i, mate(i)) (i itself if unmatched); coarse ids
  are assigned in increasing order of rep, i.e. by smallest member.
* Aggregate size 2^P means P matching passes per level, each pass matching the
  quotient graph of the previous pass.
* Galerkin summation order: W_H(I,J) = sum of W_ij over fine entries (i, j) with
  agg(i) = I != J = agg(j), added left to right in increasing i and then in the
  order of the entries within row i; d_H(I) = sum of d_i over i in I in
  increasing i; D_H from the level assembly rule.  With these orders the coarse
  values are reproducible bit for bit (and exact for integer weights).
"""
from __future__ import annotations

import numpy as np

from .level import Level, assemble
from .rng import splitmix64


def edge_strengths(lvl: Level, key: str = "normalized"):
    """Edges i < j of the level with their strengths s_ij (see module doc)."""
    rows = lvl.rows()
    up = lvl.col > rows
    i, j, w = rows[up], lvl.col[up], lvl.W[up]
    if key == "normalized":
        s = (w * w) / (lvl.D[i] * lvl.D[j])
    elif key == "raw":
        s = w.copy()
    else:
        raise ValueError(key)
    return i, j, s


def tie_hash(i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """h(i, j): x = (i * 2654435761 + j) mod 2^32, then MurmurHash3's 32-bit
    finalizer (x ^= x >> 16; x *= 0x85ebca6b; x ^= x >> 13; x *= 0xc2b2ae35;
    x ^= x >> 16, all mod 2^32)."""
    m = np.uint64(0xFFFFFFFF)
    x = (i.astype(np.uint64) * np.uint64(2654435761) + j.astype(np.uint64)) & m
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x85EBCA6B)) & m
    x ^= x >> np.uint64(13)
    x = (x * np.uint64(0xC2B2AE35)) & m
    x ^= x >> np.uint64(16)
    return x


def greedy_matching(lvl: Level, key: str = "normalized", tie: str = "index") -> np.ndarray:
    """Greedy matching in the strict edge order (-s, i, j) -- or (-s, h(i, j), i,
    j) with hash ties: mate[i] = j, or -1."""
    i, j, s = edge_strengths(lvl, key)
    if tie == "index":
        order = np.lexsort((j, i, -s))
    elif tie == "hash":
        order = np.lexsort((j, i, tie_hash(i, j), -s))
    else:
        raise ValueError(tie)
    mate = [-1] * lvl.n
    for a, b in zip(i[order].tolist(), j[order].tolist()):
        if mate[a] < 0 and mate[b] < 0:
            mate[a] = b
            mate[b] = a
    return np.asarray(mate, dtype=np.int64)


def coarse_ids(mate: np.ndarray):
    """Coarse id of every vertex, numbering aggregates by their smallest member."""
    n = mate.shape[0]
    idx = np.arange(n, dtype=np.int64)
    rep = np.where(mate >= 0, np.minimum(idx, mate), idx)
    flag = rep == idx
    first = np.cumsum(flag) - flag  # exclusive prefix sum
    return first[rep], int(flag.sum())


def _segmented_sequential_sum(seg: np.ndarray, vals: np.ndarray, nseg: int) -> np.ndarray:
    """Sum of vals per segment, added left to right; seg must be non-decreasing."""
    out = np.zeros(nseg, dtype=np.float64)
    if seg.size == 0:
        return out
    start = np.ones(seg.shape[0], dtype=bool)
    start[1:] = seg[1:] != seg[:-1]
    first_pos = np.nonzero(start)[0]
    seg_rank = np.cumsum(start) - 1
    pos = np.arange(seg.shape[0]) - first_pos[seg_rank]
    for k in range(int(pos.max()) + 1):
        sel = pos == k
        out[seg[sel]] += vals[sel]
    return out


def quotient(lvl: Level, ids: np.ndarray, nc: int) -> Level:
    """Galerkin operator P^T A P for the partition ``ids`` (module doc)."""
    rows = lvl.rows()
    I = ids[rows]
    J = ids[lvl.col]
    keep = I != J
    I, J, w = I[keep], J[keep], lvl.W[keep]
    order = np.lexsort((J, I))  # stable: CSR order kept inside each (I, J) group
    I, J, w = I[order], J[order], w[order]
    pair = I * nc + J
    newpair = np.ones(pair.shape[0], dtype=bool)
    newpair[1:] = pair[1:] != pair[:-1]
    gid = np.cumsum(newpair) - 1
    ng = int(newpair.sum())
    WH = _segmented_sequential_sum(gid, w, ng)
    IH = I[newpair]
    JH = J[newpair]
    row_ptr = np.zeros(nc + 1, dtype=np.int64)
    np.cumsum(np.bincount(IH, minlength=nc), out=row_ptr[1:])
    vorder = np.argsort(ids, kind="stable")  # members of each aggregate in increasing i
    dH = _segmented_sequential_sum(ids[vorder], lvl.d[vorder], nc)
    return assemble(nc, row_ptr, JH, WH, dH)


def aggregate_level(lvl: Level, passes: int, key: str = "normalized", tie: str = "index"):
    """``passes`` matching passes; returns (composite aggregate map, coarse level)."""
    agg = np.arange(lvl.n, dtype=np.int64)
    g = lvl
    for _ in range(passes):
        mate = greedy_matching(g, key, tie)
        ids, nc = coarse_ids(mate)
        g = quotient(g, ids, nc)
        agg = ids[agg]
    return agg, g


# ---- the paper's own aggregation: a maximal independent set of the graph of A^k


def mis_keys(n: int) -> np.ndarray:
    """Priority of vertex v: splitmix64(v) (distinct: the generator's output
    function is a bijection of 64-bit words)."""
    return np.array([splitmix64(v) for v in range(n)], dtype=np.uint64)


def _within(lvl: Level, v: int, k: int) -> np.ndarray:
    """Vertices at graph distance <= k from v (breadth-first, k hops)."""
    seen = {v}
    frontier = [v]
    for _ in range(k):
        nxt = []
        for u in frontier:
            for w in lvl.col[lvl.row_ptr[u]:lvl.row_ptr[u + 1]]:
                w = int(w)
                if w not in seen:
                    seen.add(w)
                    nxt.append(w)
        frontier = nxt
    return np.fromiter(seen, dtype=np.int64)


def distance_k_mis(lvl: Level, k: int) -> np.ndarray:
    """Step (A) of Section 2's partitioning: a maximal independent set of the
    graph of A^k (two vertices adjacent when at graph distance <= k).  Reading:
    the greedy set that takes vertices in decreasing priority (mis_keys) and
    skips those within distance k of a taken one.  Returned sorted."""
    keys = mis_keys(lvl.n)
    blocked = np.zeros(lvl.n, dtype=bool)
    S = []
    for v in np.argsort(keys)[::-1]:
        v = int(v)
        if blocked[v]:
            continue
        S.append(v)
        blocked[_within(lvl, v, k)] = True
    return np.array(sorted(S), dtype=np.int64)


def nearest_owner(lvl: Level, S: np.ndarray) -> np.ndarray:
    """Step (B): every vertex joins the set vertex nearest to it in graph
    distance (breadth-first from all of S at once); a vertex first reached at
    hop h takes the smallest owner among its neighbours reached at hop h-1."""
    n = lvl.n
    owner = -np.ones(n, dtype=np.int64)
    owner[S] = S
    frontier = list(S)
    while frontier:
        cand = {}
        for u in frontier:
            for w in lvl.col[lvl.row_ptr[u]:lvl.row_ptr[u + 1]]:
                w = int(w)
                if owner[w] < 0:
                    cand[w] = min(cand.get(w, n), int(owner[u]))
        for w, o in cand.items():
            owner[w] = o
        frontier = list(cand)
    return owner


def mis_aggregate(lvl: Level, k: int = 4):
    """(ids, nc): aggregates of steps (A) and (B), coarse ids in increasing
    order of the set vertex that owns them."""
    S = distance_k_mis(lvl, k)
    owner = nearest_owner(lvl, S)
    if np.any(owner < 0):
        raise ValueError("graph is not connected")
    return np.searchsorted(S, owner).astype(np.int64), int(S.shape[0])
