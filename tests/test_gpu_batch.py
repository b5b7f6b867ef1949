"""Batched solves (amg_solve_batch) against the CPU oracle, and isolation:
an item's result is the same alone and in any mix."""
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


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _oracle_params(p):
    return oracle.Params(degree=p.degree, agg_size=p.agg_size, coarse_max=p.coarse_max,
                         lambda0_ratio=p.lambda0_ratio, inner_steps=p.inner_steps, restart=p.restart,
                         tol=p.tol, max_iter=p.max_iter, match_key="normalized")


def _graphs():
    gs = [inputs.rgg(int(n), seed=inputs.seed_for(4, i)) for i, n in enumerate([1200, 5000, 17000, 2600])]
    gs += [inputs.grid2d(70, 33), inputs.tet3d(9), inputs.grid2d(6, 7)]  # the last one has a single level
    return gs


@pytest.fixture(scope="module")
def batch_setup(amg):
    out = {}
    for prec in ("fp64", "mixed"):
        p = amg.amg_params_default(degree=4, agg_size=8, precision=prec)
        gs = _graphs()
        hs = [amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p) for g in gs]
        out[prec] = (p, gs, hs)
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_matches_oracle(amg, batch_setup, prec):
    p, gs, hs = batch_setup[prec]
    fs = [_t(inputs.rhs(g.n, 40 + i)) for i, g in enumerate(gs)]
    us = [torch.zeros_like(f) for f in fs]
    infos = amg.amg_solve_batch(hs, fs, us)
    for i, (g, info) in enumerate(zip(gs, infos)):
        ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, _oracle_params(p))
        res = oracle.fcg(ho, fs[i].cpu().numpy())
        assert info["status"] == 0, (i, info)
        assert info["rel_res_true"] <= 1e-8, (i, info)
        if prec == "fp64":
            assert abs(info["iters"] - res.iters) <= 1, (i, info["iters"], res.iters)
        else:
            assert info["iters"] <= res.iters + 3, (i, info["iters"], res.iters)
        lo = ho.levels[0]
        e = us[i].cpu().numpy() - res.x
        errA = np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(res.x @ oracle.apply_A(lo, res.x))
        assert errA <= 1e-6, (i, errA)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_item_same_alone_and_in_mix(amg, batch_setup, prec):
    p, gs, hs = batch_setup[prec]
    fs = [_t(inputs.rhs(g.n, 60 + i, "normal")) for i, g in enumerate(gs)]
    mix = [torch.zeros_like(f) for f in fs]
    infos = amg.amg_solve_batch(hs, fs, mix)
    for i in (0, 2, 4, 6):
        alone = torch.zeros_like(fs[i])
        inf1 = amg.amg_solve_batch([hs[i]], [fs[i]], [alone])
        assert inf1[0]["iters"] == infos[i]["iters"]
        assert torch.equal(alone, mix[i]), i
    # a different mix (reversed order, fewer items) gives the same bits again
    order = [5, 3, 1, 0]
    sub = [torch.zeros_like(fs[i]) for i in order]
    amg.amg_solve_batch([hs[i] for i in order], [fs[i] for i in order], sub)
    for k, i in enumerate(order):
        assert torch.equal(sub[k], mix[i]), i


def test_several_rhs_on_one_hierarchy(amg, batch_setup):
    p, gs, hs = batch_setup["mixed"]
    h = hs[2]
    n = gs[2].n
    fs = [_t(inputs.rhs(n, 80 + k)) for k in range(4)]
    us = [torch.zeros_like(f) for f in fs]
    infos = amg.amg_solve_batch([h] * 4, fs, us)
    for k in range(4):
        assert infos[k]["status"] == 0 and infos[k]["rel_res_true"] <= 1e-8
        alone = torch.zeros_like(fs[k])
        amg.amg_solve_batch([h], [fs[k]], [alone])
        assert torch.equal(alone, us[k])
        # the same system through the one-at-a-time path agrees to solver accuracy
        u1 = torch.zeros_like(fs[k])
        info1 = amg.amg_solve(h, fs[k], u1)
        assert info1["status"] == 0
        assert float((u1 - us[k]).norm() / u1.norm()) <= 1e-6


def test_zero_rhs_and_nonzero_guess_in_batch(amg, batch_setup):
    p, gs, hs = batch_setup["fp64"]
    f0 = torch.zeros(gs[0].n, dtype=torch.float64, device="cuda")
    u0 = torch.zeros_like(f0)
    f1 = _t(inputs.rhs(gs[1].n, 7))
    g1 = _t(inputs.rhs(gs[1].n, 8))
    u1 = g1.clone()
    infos = amg.amg_solve_batch([hs[0], hs[1]], [f0, f1], [u0, u1])
    assert infos[0]["iters"] == 0 and infos[0]["status"] == 0 and float(u0.abs().max()) == 0.0
    assert infos[1]["status"] == 0 and infos[1]["rel_res_true"] <= 1e-8
    ho = oracle.build_hierarchy(gs[1].n, gs[1].row_ptr, gs[1].col, gs[1].w, gs[1].d, _oracle_params(p))
    res = oracle.fcg(ho, f1.cpu().numpy(), g1.cpu().numpy())
    assert abs(infos[1]["iters"] - res.iters) <= 1


def test_batch_maxit_status(amg):
    g = inputs.grid2d(40)
    p = amg.amg_params_default(degree=3, agg_size=4, max_iter=2)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    f = _t(inputs.rhs(g.n, 3))
    u = torch.zeros_like(f)
    infos = amg.amg_solve_batch([h], [f], [u])
    assert infos[0]["status"] == amg.AMG_ERR_MAXIT and infos[0]["iters"] == 2


def test_batch_mis_neumann_items(amg):
    """Hierarchies from Section 2's partitioning, pure Neumann ones included,
    batched with a matching hierarchy: each item against the oracle."""
    specs = [(inputs.poisson2d(60), dict(aggregation="mis", neumann=1)),
             (inputs.poisson3d(14), dict(aggregation="mis", neumann=1)),
             (inputs.delaunay3d(9, seed=inputs.seed_for(6, 9)), dict(aggregation="mis", mis_distance=2)),
             (inputs.grid2d(50, 41), dict(agg_size=8))]
    hs, fs, hos = [], [], []
    for i, (g, kw) in enumerate(specs):
        p = amg.amg_params_default(degree=4, **kw)
        hs.append(amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p))
        f = inputs.rhs(g.n, 80 + i)
        fs.append(inputs.project_range(f) if not np.any(g.d) else f)
        hos.append(oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(
            degree=4, agg_size=p.agg_size, aggregation="mis" if p.aggregation == amg.AMG_AGG_MIS else "matching",
            mis_distance=p.mis_distance)))
    us = [torch.zeros(g.n, dtype=torch.float64, device="cuda") for g, _ in specs]
    infos = amg.amg_solve_batch(hs, [_t(f) for f in fs], us)
    for i, ((g, _), info, ho) in enumerate(zip(specs, infos, hos)):
        res = oracle.fcg(ho, fs[i])
        assert info["status"] == 0 and res.converged, (i, info)
        assert abs(info["iters"] - res.iters) <= 1, (i, info["iters"], res.iters)
        lo = ho.levels[0]
        e = us[i].cpu().numpy() - res.x
        errA = np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(res.x @ oracle.apply_A(lo, res.x))
        assert errA <= 1e-6, (i, errA)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_grouped_rhs_on_a_large_level(amg, prec):
    # several right-hand sides on one hierarchy whose finest level spans more
    # than 1024 tiles of 64 rows: the batched executor loads each row's
    # entries once for the group and applies them to every right-hand side;
    # every item must give the bits it gives alone (where it is not grouped),
    # in any mix, and converge like the one-at-a-time solve
    g = inputs.grid2d(300)
    g2 = inputs.rgg(4000, seed=inputs.seed_for(4, 5))
    p = amg.amg_params_default(degree=4, agg_size=8, precision=prec)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    h2 = amg.amg_setup(g2.n, g2.row_ptr, g2.col, g2.w, g2.d, p)
    assert g.n >= 1024 * 64
    fs = [_t(inputs.rhs(g.n, 90 + k)) for k in range(5)]
    f2 = _t(inputs.rhs(g2.n, 99))
    us = [torch.zeros_like(f) for f in fs]
    u2 = torch.zeros_like(f2)
    infos = amg.amg_solve_batch([h, h2, h, h, h, h], [fs[0], f2] + fs[1:], [us[0], u2] + us[1:])
    for k in range(5):
        info = infos[0] if k == 0 else infos[k + 1]
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8, info
        alone = torch.zeros_like(fs[k])
        inf1 = amg.amg_solve_batch([h], [fs[k]], [alone])
        assert inf1[0]["iters"] == info["iters"]
        assert torch.equal(alone, us[k]), k
    alone2 = torch.zeros_like(f2)
    amg.amg_solve_batch([h2], [f2], [alone2])
    assert torch.equal(alone2, u2)
    # three of them in another mix (a group of three, reversed)
    sub = [torch.zeros_like(fs[k]) for k in (4, 2, 0)]
    amg.amg_solve_batch([h] * 3, [fs[4], fs[2], fs[0]], sub)
    for j, k in enumerate((4, 2, 0)):
        assert torch.equal(sub[j], us[k]), k
    # against the one-at-a-time solve of the same system
    u1 = torch.zeros_like(fs[1])
    ref = amg.amg_solve(h, fs[1], u1)
    assert abs(ref["iters"] - infos[2]["iters"]) <= 1
    assert (torch.linalg.norm(u1 - us[1]) / torch.linalg.norm(u1)).item() <= 1e-6
    h.close()
    h2.close()
