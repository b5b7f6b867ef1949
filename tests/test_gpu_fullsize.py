"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 1024 x 1024 grid (1,048,576 unknowns), aggregates of 16, degree 3,
FP64; Section 4's 1024^2 Neumann square with its own partitioning; the
128^3 tetrahedral cube (hierarchy bit-exact, FP64 and mixed solves against the
oracle's FP64 solution); and the batch of 256 random geometric graphs
(properties, sampled items)."""
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


@pytest.fixture(scope="module")
def grid1024(amg):
    g = inputs.grid2d(1024)
    p = amg.amg_params_default(degree=3, agg_size=16)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=3, agg_size=16))
    return g, p, h, ho


def test_fullsize_hierarchy_bit_exact(amg, grid1024):
    g, p, h, ho = grid1024
    assert amg.amg_describe(h)["n"] == [l.n for l in ho.levels]
    for l, lo in enumerate(ho.levels):
        ex = amg.amg_level_export(h, l)
        assert np.array_equal(ex["col"], lo.col) and np.array_equal(ex["W"], lo.W), l
        if l < ho.L:
            assert np.array_equal(ex["agg"], ho.aggs[l]), l


def test_fullsize_cycle_and_solve(amg, grid1024):
    g, p, h, ho = grid1024
    f = inputs.rhs(g.n, inputs.seed_for(2))
    r = torch.tensor(f, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    amg.amg_apply_cycle(h, r, z)
    zo = oracle.kcycle(ho, 0, f)
    assert np.linalg.norm(z.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
    u = torch.zeros_like(r)
    info = amg.amg_solve(h, r, u)
    res = oracle.fcg(ho, f)
    assert info["status"] == 0 and abs(info["iters"] - res.iters) <= 1
    assert info["rel_res_true"] <= 1e-8
    e = u.cpu().numpy() - res.x
    lo = ho.levels[0]
    assert np.sqrt(e @ oracle.apply_A(lo, e)) <= 1e-6 * np.sqrt(res.x @ oracle.apply_A(lo, res.x))


@pytest.fixture(scope="module")
def tet128():
    """The 128^3 tetrahedral cube (2,097,152 unknowns), its oracle hierarchy
    (degree 5, aggregates of 16) and the Gaussian right-hand side."""
    g = inputs.tet3d(128)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=5, agg_size=16))
    f = inputs.rhs(g.n, inputs.seed_for(3), "normal")
    return g, ho, f


def _levels_equal(amg, h, ho):
    assert amg.amg_describe(h)["n"] == [l.n for l in ho.levels]
    for l, lo in enumerate(ho.levels):
        ex = amg.amg_level_export(h, l)
        assert np.array_equal(ex["row_ptr"], lo.row_ptr) and np.array_equal(ex["col"], lo.col), l
        assert np.array_equal(ex["W"], lo.W) and np.array_equal(ex["d"], lo.d), l
        if l < ho.L:
            assert np.array_equal(ex["agg"], ho.aggs[l]), l


@pytest.mark.timeout(300)
def test_fullsize_tet3d_hierarchy_bit_exact(amg, tet128):
    """128^3 cube at the bench's configuration: the FP64 and the mixed
    hierarchies (set up in FP64 alike) equal the oracle's level by level."""
    g, ho, _ = tet128
    for prec in ("fp64", "mixed"):
        p = amg.amg_params_default(degree=5, agg_size=16, precision=prec)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        _levels_equal(amg, h, ho)
        h.close()


@pytest.mark.timeout(300)
def test_fullsize_tet3d_mixed_vs_oracle(amg, tet128):
    """128^3 cube: the FP64 solve within one iteration of the oracle's, the
    mixed solve (FP32 cycle under FP64 FCG) at a true FP64 residual of at most
    1e-8 and within 1e-6 of the oracle's FP64 solution in the A-norm."""
    g, ho, f = tet128
    res = oracle.fcg(ho, f)
    assert res.converged
    lo = ho.levels[0]
    xo = res.x
    nx = np.sqrt(xo @ oracle.apply_A(lo, xo))
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    its = {}
    for prec in ("fp64", "mixed"):
        p = amg.amg_params_default(degree=5, agg_size=16, precision=prec)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        u = torch.zeros_like(ft)
        info = amg.amg_solve(h, ft, u)
        h.close()
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8, (prec, info)
        its[prec] = info["iters"]
        e = u.cpu().numpy() - xo
        assert np.sqrt(e @ oracle.apply_A(lo, e)) <= 1e-6 * nx, prec
    assert abs(its["fp64"] - res.iters) <= 1, (its, res.iters)
    assert abs(its["mixed"] - its["fp64"]) <= 2, its


def test_fullsize_section4_square(amg):
    """Section 4's 2D model problem at the bench size (1024^2 pure Neumann FE
    square, independent set of A^4, m = 4, coarsest below 100 rows, the A-norm
    test on A u = 0), in the bench's launch configuration: every level and
    aggregate map bit-exact, one cycle within 1e-10, iterations within one of
    the oracle's and the A-norm ratio of the result at most the tolerance."""
    g = inputs.poisson2d(1024)
    p = amg.amg_params_default(degree=4, aggregation="mis", mis_distance=4, neumann=1, coarse_max=99,
                               stop="energy")
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(
        degree=4, aggregation="mis", mis_distance=4, coarse_max=99, stop="energy"))
    assert amg.amg_describe(h)["n"] == [l.n for l in ho.levels]
    for l, lo in enumerate(ho.levels):
        ex = amg.amg_level_export(h, l)
        assert np.array_equal(ex["col"], lo.col) and np.array_equal(ex["W"], lo.W), l
        if l < ho.L:
            assert np.array_equal(ex["agg"], ho.aggs[l]), l
    u0 = inputs.project_range(inputs.rhs(g.n, inputs.seed_for(9, 2024), "uniform"))
    z = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    amg.amg_apply_cycle(h, torch.tensor(u0, device="cuda"), z)
    zo = oracle.kcycle(ho, 0, u0)
    assert np.linalg.norm(z.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, torch.zeros_like(u), u)
    res = oracle.fcg(ho, np.zeros(g.n), u0)
    assert info["status"] == 0 and res.converged and abs(info["iters"] - res.iters) <= 1, (info, res.iters)
    lo = ho.levels[0]
    uh = u.cpu().numpy()
    assert np.sqrt(uh @ oracle.apply_A(lo, uh)) <= p.tol * np.sqrt(u0 @ oracle.apply_A(lo, u0))


def test_fullsize_batch_rgg256(amg):
    """The batched form at the bench's full size and launch configuration (256
    random geometric graphs, 9.8 M unknowns, mixed precision, agg 8, m 4, one
    amg_solve_batch): every item converges with its true FP64 residual at most
    the tolerance (a property at any size), and sampled items (the smallest
    and two others) match the oracle to the mixed-precision bar."""
    sizes = inputs.rgg_batch_sizes(256, inputs.seed_for(4))
    graphs = [inputs.rgg(int(n), inputs.seed_for(4, i)) for i, n in enumerate(sizes)]
    p = amg.amg_params_default(degree=4, agg_size=8, precision="mixed")
    hs = [amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p) for g in graphs]
    fs = [torch.tensor(inputs.rhs(g.n, inputs.seed_for(4, 1000 + i)), dtype=torch.float64, device="cuda")
          for i, g in enumerate(graphs)]
    us = [torch.zeros_like(f) for f in fs]
    infos = amg.amg_solve_batch(hs, fs, us)
    assert all(i["status"] == 0 and i["rel_res_true"] <= 1e-8 for i in infos)
    order = np.argsort([g.n for g in graphs])
    for k in (int(order[0]), int(order[len(order) // 3]), 17):
        g = graphs[k]
        ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=4, agg_size=8))
        res = oracle.fcg(ho, fs[k].cpu().numpy())
        assert infos[k]["iters"] <= res.iters + 3, (k, infos[k]["iters"], res.iters)
        e = us[k].cpu().numpy() - res.x
        lo = ho.levels[0]
        assert np.sqrt(e @ oracle.apply_A(lo, e)) <= 1e-6 * np.sqrt(res.x @ oracle.apply_A(lo, res.x)), k
    for h in hs:
        h.close()
