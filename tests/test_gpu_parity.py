"""GPU path (through the C ABI) against the CPU FP64 oracle.

Bars: aggregates, coarse sparsity patterns and coarse values bit-exact; single
kernels within 1e-12 relative; one k-cycle application within 1e-10 relative;
outer FCG iteration counts within one and the true FP64 relative residual at
most the tolerance."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1307_6305_amd as amg

    amg.load_library()
    return amg


def _oracle_params(amg, p):
    return oracle.Params(degree=p.degree, agg_size=p.agg_size, coarse_max=p.coarse_max,
                         lambda0_ratio=p.lambda0_ratio, inner_steps=p.inner_steps, restart=p.restart,
                         tol=p.tol, max_iter=p.max_iter,
                         match_key="raw" if p.match_key == 1 else "normalized",
                         tie_break="hash" if p.tie_break == 1 else "index",
                         max_coarsest=p.max_coarsest, stagnation=p.stagnation,
                         aggregation="mis" if p.aggregation == amg.AMG_AGG_MIS else "matching",
                         mis_distance=p.mis_distance)


CASES = {
    "grid64_agg4_m3": (lambda: inputs.grid2d(64), dict(degree=3, agg_size=4)),
    "grid100x37_agg16_m5": (lambda: inputs.grid2d(100, 37), dict(degree=5, agg_size=16)),
    "grid64_raw_agg4": (lambda: inputs.grid2d(64), dict(degree=3, agg_size=4, match_key=1)),
    "tet3d_12_agg8_m4": (lambda: inputs.tet3d(12), dict(degree=4, agg_size=8)),
    "delaunay11_agg16_m4": (lambda: inputs.delaunay3d(11, seed=inputs.seed_for(6, 11)), dict(degree=4, agg_size=16)),
    "rgg_6000_agg8_m4": (lambda: inputs.rgg(6000, seed=inputs.seed_for(4, 1)), dict(degree=4, agg_size=8)),
    "random_weighted_agg4": (lambda: inputs.random_graph(700, 0.006, seed=5, weighted=True),
                             dict(degree=4, agg_size=4, coarse_max=40)),
    "grid130_agg4_m7_inner3": (lambda: inputs.grid2d(130), dict(degree=7, agg_size=4, inner_steps=3, restart=3)),
    "grid120_hash_agg16": (lambda: inputs.grid2d(120), dict(degree=3, agg_size=16, tie_break=1)),
    "rgg_6000_hash_raw_agg8": (lambda: inputs.rgg(6000, seed=inputs.seed_for(4, 2)),
                               dict(degree=4, agg_size=8, tie_break=1, match_key=1)),
    # Section 2's own partitioning (independent set of the graph of A^k, then
    # nearest owner), on the pure Neumann model problems of Section 4
    "poisson2d_72_mis4_neumann": (lambda: inputs.poisson2d(72), dict(degree=3, aggregation="mis", neumann=1)),
    "poisson3d_20_mis4_neumann": (lambda: inputs.poisson3d(20), dict(degree=4, aggregation="mis", neumann=1)),
    "delaunay11_mis2": (lambda: inputs.delaunay3d(11, seed=inputs.seed_for(6, 11)),
                        dict(degree=4, aggregation="mis", mis_distance=2)),
    "grid100x37_mis1": (lambda: inputs.grid2d(100, 37), dict(degree=3, aggregation="mis", mis_distance=1)),
    # a path (one row of the grid): coarse levels of two neighbours per row, so
    # the tail program's padded width is 4 (the other cases give 8 to 44)
    "path3000_agg4_m3": (lambda: inputs.grid2d(3000, 1), dict(degree=3, agg_size=4)),
}


def _rhs(g, seed):
    """inputs.rhs, projected onto range(A) when d = 0 everywhere (pure Neumann)."""
    f = inputs.rhs(g.n, seed)
    return inputs.project_range(f) if not np.any(g.d) else f

_cache = {}


def _case(amg, name):
    if name not in _cache:
        make, kw = CASES[name]
        g = make()
        p = amg.amg_params_default(**kw)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(amg, p))
        _cache[name] = (g, p, h, ho)
    return _cache[name]


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else a
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_bit_exact(amg, name):
    g, p, h, ho = _case(amg, name)
    desc = amg.amg_describe(h)
    assert desc["n"] == [l.n for l in ho.levels]
    for l, lo in enumerate(ho.levels):
        ex = amg.amg_level_export(h, l)
        assert np.array_equal(ex["row_ptr"], lo.row_ptr), l
        assert np.array_equal(ex["col"], lo.col), l
        assert np.array_equal(ex["W"], lo.W), l
        assert np.array_equal(ex["d"], lo.d), l
        assert np.array_equal(ex["D"], lo.D), l
        if l < ho.L:
            assert np.array_equal(ex["agg"], ho.aggs[l]), l
        assert desc["lambda1"][l] == oracle.lambda_max_bound(lo)
    assert desc["grid_complexity"] == pytest.approx(ho.grid_complexity(), rel=1e-14)


@pytest.mark.parametrize("name", list(CASES))
def test_single_steps(amg, name):
    g, p, h, ho = _case(amg, name)
    rng = np.random.default_rng(7)
    for l in range(ho.L):
        lo = ho.levels[l]
        v = rng.standard_normal(lo.n)
        x = rng.standard_normal(lo.n)
        y = torch.zeros(lo.n, dtype=torch.float64, device="cuda")
        amg.amg_apply_smoother(h, l, _t(v), y)
        assert _rel(y, oracle.smooth(lo, ho.polys[l], v)) <= 1e-12, ("smoother", l)
        s = torch.zeros_like(y)
        amg.amg_apply_residual(h, l, _t(v), _t(x), s)
        assert _rel(s, oracle.residual(lo, v, x)) <= 1e-13, ("residual", l)
        nc = ho.levels[l + 1].n
        b = torch.zeros(nc, dtype=torch.float64, device="cuda")
        amg.amg_apply_restrict(h, l, _t(v), b)
        assert _rel(b, oracle.restrict(ho.aggs[l], nc, v)) <= 1e-14, ("restrict", l)
        e = rng.standard_normal(nc)
        xx = _t(x)
        amg.amg_apply_prolong(h, l, _t(e), xx)
        assert _rel(xx, x + oracle.prolong(ho.aggs[l], e)) <= 1e-15, ("prolong", l)
    nL = ho.levels[-1].n
    bL = rng.standard_normal(nL)
    xL = torch.zeros(nL, dtype=torch.float64, device="cuda")
    amg.amg_apply_coarse(h, _t(bL), xL)
    assert _rel(xL, oracle.coarse_solve(ho.chol, bL)) <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_cycle_application(amg, name):
    g, p, h, ho = _case(amg, name)
    for seed in (1, 2):
        r = inputs.rhs(g.n, seed)
        z = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        amg.amg_apply_cycle(h, _t(r), z)
        assert _rel(z, oracle.kcycle(ho, 0, r)) <= 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_solve_matches_oracle(amg, name):
    g, p, h, ho = _case(amg, name)
    f = _rhs(g, inputs.seed_for(1))
    u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, _t(f), u)
    res = oracle.fcg(ho, f)
    assert info["status"] == 0 and res.converged
    assert abs(info["iters"] - res.iters) <= 1, (info, res.iters)
    assert info["rel_res_true"] <= p.tol
    uo = res.x
    lo = ho.levels[0]
    e = u.cpu().numpy() - uo
    errA = np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(uo @ oracle.apply_A(lo, uo))
    assert errA <= 1e-6


def test_graph_replay_equals_eager(amg):
    g = inputs.grid2d(96, 71)
    f = _t(inputs.rhs(g.n, 3))
    out = []
    for use_graph in (0, 1, 1):
        p = amg.amg_params_default(degree=4, agg_size=8, use_graph=use_graph)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        info = amg.amg_solve(h, f, u)
        # a second solve on the same handle replays the recorded graphs
        u2 = torch.zeros_like(u)
        info2 = amg.amg_solve(h, f, u2)
        assert info["iters"] == info2["iters"]
        assert torch.equal(u, u2)
        out.append((info["iters"], u.cpu().numpy()))
        h.close()
    assert out[0][0] == out[1][0] == out[2][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[1][1], out[2][1])


def test_nonzero_initial_guess_and_zero_rhs(amg):
    g = inputs.grid2d(50)
    p = amg.amg_params_default(degree=3, agg_size=4)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(amg, p))
    f = inputs.rhs(g.n, 11)
    u0 = inputs.rhs(g.n, 12)
    u = _t(u0)
    info = amg.amg_solve(h, _t(f), u)
    res = oracle.fcg(ho, f, u0)
    assert abs(info["iters"] - res.iters) <= 1 and info["rel_res_true"] <= 1e-8
    z = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, torch.zeros_like(z), z)
    assert info["iters"] == 0 and info["status"] == 0 and float(z.abs().max()) == 0.0


def test_single_level_hierarchy(amg):
    g = inputs.grid2d(7, 9)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(degree=3))
    assert amg.amg_describe(h)["levels"] == 1
    f = inputs.rhs(g.n, 1)
    u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, _t(f), u)
    assert info["iters"] == 1 and info["rel_res_true"] <= 1e-12


def test_one_vertex(amg):
    """The smallest problem, n = 1 with no edges: A = [d] is its own coarsest
    level, the preconditioner is the exact solve, and one iteration gives
    u = f / d, in FP64 and in mixed precision (same as the oracle)."""
    rp = np.array([0, 0], dtype=np.int32)
    col = np.zeros(0, dtype=np.int32)
    w = np.zeros(0)
    d = np.array([2.5])
    res = oracle.fcg(oracle.build_hierarchy(1, rp, col, w, d, oracle.Params(degree=3)), np.array([5.0]))
    assert res.iters == 1 and res.x[0] == pytest.approx(2.0, rel=1e-15)
    for precision in ("fp64", "mixed"):
        h = amg.amg_setup(1, rp, col, w, d, amg.amg_params_default(degree=3, precision=precision))
        assert amg.amg_describe(h)["levels"] == 1
        u = torch.zeros(1, dtype=torch.float64, device="cuda")
        info = amg.amg_solve(h, torch.tensor([5.0], dtype=torch.float64, device="cuda"), u)
        assert info["status"] == 0 and info["iters"] == res.iters
        assert float(u[0]) == pytest.approx(2.0, rel=1e-15)


def test_stagnating_coarsening_uses_block_cholesky(amg):
    """A star graph coarsens by one pair per pass: stagnation stops the
    hierarchy and the coarsest level (> 64 rows) is solved by the workgroup
    Cholesky path."""
    n = 300
    hub = np.zeros(n - 1, dtype=np.int64)
    leaves = np.arange(1, n)
    rp, col, w = inputs.csr_from_edges(n, hub, leaves)
    d = np.zeros(n)
    d[5] = 1.0
    p = amg.amg_params_default(degree=3, agg_size=4, coarse_max=16)
    h = amg.amg_setup(n, rp, col, w, d, p)
    desc = amg.amg_describe(h)
    ho = oracle.build_hierarchy(n, rp, col, w, d, _oracle_params(amg, p))
    assert desc["n"] == [l.n for l in ho.levels] and desc["n"][-1] > 64
    b = np.random.default_rng(0).standard_normal(desc["n"][-1])
    x = torch.zeros(desc["n"][-1], dtype=torch.float64, device="cuda")
    amg.amg_apply_coarse(h, _t(b), x)
    assert _rel(x, oracle.coarse_solve(ho.chol, b)) <= 1e-11
    f = inputs.rhs(n, 2)
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, _t(f), u)
    assert info["status"] == 0 and abs(info["iters"] - oracle.fcg(ho, f).iters) <= 1


def test_determinism(amg):
    g = inputs.tet3d(10)
    p = amg.amg_params_default(degree=4, agg_size=8)
    f = _t(inputs.rhs(g.n, 4, "normal"))
    sols = []
    for _ in range(2):
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        amg.amg_solve(h, f, u)
        sols.append(u.cpu().numpy())
        h.close()
    assert np.array_equal(sols[0], sols[1])


@pytest.mark.parametrize("tail_rows", [0, 300, 1100, 70000])
def test_tail_program_matches_oracle(amg, tail_rows):
    """The one-workgroup tail interpreter (inner solves of levels with at most
    tail_rows rows) gives the same cycle as the device-wide kernels."""
    g = inputs.grid2d(90, 77)
    p = amg.amg_params_default(degree=4, agg_size=4, tail_rows=tail_rows)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(amg, p))
    r = inputs.rhs(g.n, 21)
    z = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    amg.amg_apply_cycle(h, _t(r), z)
    assert _rel(z, oracle.kcycle(ho, 0, r)) <= 1e-10
    f = inputs.rhs(g.n, 22)
    u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, _t(f), u)
    assert info["status"] == 0 and abs(info["iters"] - oracle.fcg(ho, f).iters) <= 1


@pytest.mark.parametrize("make,kw", [
    (lambda: inputs.tet3d(16), dict(degree=5, agg_size=16)),
    (lambda: inputs.grid2d(120, 97), dict(degree=3, agg_size=4)),
    (lambda: inputs.rgg(8000, seed=inputs.seed_for(4, 3)), dict(degree=4, agg_size=8)),
])
def test_mixed_precision_solve(amg, make, kw):
    """FP32 cycle under FP64 flexible CG: true FP64 residual <= 1e-8 and the
    A-norm error against the FP64 oracle solution <= 1e-6."""
    g = make()
    f = inputs.rhs(g.n, 31, "normal")
    p = amg.amg_params_default(precision=amg.AMG_MIXED, **kw)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(amg, p))
    # the hierarchy is the same (FP64 setup), only the cycle runs in FP32
    assert amg.amg_describe(h)["n"] == [l.n for l in ho.levels]
    r = _t(f)
    z = torch.zeros_like(r)
    amg.amg_apply_cycle(h, r, z)
    assert _rel(z, oracle.kcycle(ho, 0, f)) <= 1e-5
    u = torch.zeros_like(r)
    info = amg.amg_solve(h, r, u)
    res = oracle.fcg(ho, f)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-8
    assert info["iters"] <= res.iters + 3
    lo = ho.levels[0]
    e = u.cpu().numpy() - res.x
    errA = np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(res.x @ oracle.apply_A(lo, res.x))
    assert errA <= 1e-6


def test_hash_ties_fewer_rounds(amg):
    # index ties chain along a structured grid; hashed ties break the chains
    g = inputs.grid2d(256)
    rounds = {}
    for tie in ("index", "hash"):
        p = amg.amg_params_default(degree=3, agg_size=16, tie_break=tie)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        rounds[tie] = amg.amg_describe(h)["match_rounds"]
        f = _t(inputs.rhs(g.n, 3))
        u = torch.zeros_like(f)
        info = amg.amg_solve(h, f, u)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8
        h.close()
    assert rounds["hash"] * 4 < rounds["index"], rounds


@pytest.mark.parametrize("restart,use_graph", [(1, 1), (2, 0), (5, 1)])
def test_iteration_limit_and_window(amg, restart, use_graph):
    """The outer loop queues the next iteration before reading the test of the
    current one: an iteration limit still stops at exactly max_iter iterations
    with the oracle's iterate, and windows of one and two positions (one shared
    pinned slot, or alternating ones) solve as the oracle does."""
    g = inputs.grid2d(80, 53)
    kw = dict(degree=3, agg_size=4, restart=restart, use_graph=use_graph)
    p3 = amg.amg_params_default(max_iter=3, **kw)
    h3 = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p3)
    ho3 = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(amg, p3))
    f = inputs.rhs(g.n, 31)
    u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h3, _t(f), u)
    res = oracle.fcg(ho3, f)
    assert info["status"] == amg.AMG_ERR_MAXIT and info["iters"] == 3 and not res.converged
    assert _rel(u, res.x) <= 1e-9
    p = amg.amg_params_default(**kw)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(amg, p))
    u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, _t(f), u)
    res = oracle.fcg(ho, f)
    assert info["status"] == 0 and abs(info["iters"] - res.iters) <= 1
    assert info["rel_res_true"] <= p.tol


@pytest.mark.parametrize("N,agg,tol,use_graph", [(32, 4, 1e-15, 1), (48, 16, 3e-15, 0), (48, 16, 3e-15, 1)])
def test_true_residual_replaces_recursive(amg, N, agg, tol, use_graph):
    """Near the rounding floor the recursive residual passes the test before
    the true one does: the solve confirms on the true FP64 residual, restarts
    from it, and returns OK only with ||f - A u|| <= tol ||f||, as the oracle
    does (same number of replacements, iterations within two); the batched
    form confirms the same way per item."""
    g = inputs.grid2d(N)
    p = amg.amg_params_default(degree=3, agg_size=agg, tol=tol, max_iter=80, use_graph=use_graph)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(amg, p))
    f = inputs.rhs(g.n, 9)
    res = oracle.fcg(ho, f)
    assert res.converged and res.replacements >= 1
    u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, _t(f), u)
    assert info["status"] == 0 and info["rel_res_true"] <= tol, info
    assert info["replacements"] >= 1 and abs(info["iters"] - res.iters) <= 2, (info, res.iters)
    A = oracle.apply_A(ho.levels[0], u.cpu().numpy())
    assert np.linalg.norm(f - A) <= tol * np.linalg.norm(f)
    ub = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    bi = amg.amg_solve_batch([h], [_t(f)], [ub])[0]
    assert bi["status"] == 0 and bi["rel_res_true"] <= tol and bi["replacements"] >= 1, bi
    assert abs(bi["iters"] - res.iters) <= 2, (bi, res.iters)
    h.close()
