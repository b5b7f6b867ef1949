"""Stationary AMLI cycle (cycle = AMG_CYCLE_AMLI) against the oracle's
(oracle/amli.py): the estimated intervals, one cycle application, the solve."""
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


CASES = {
    "grid64_agg4": (lambda: inputs.grid2d(64), dict(degree=4, agg_size=4)),
    "rgg5000_agg4": (lambda: inputs.rgg(5000, seed=inputs.seed_for(7, 1)), dict(degree=4, agg_size=4)),
    "tet12_agg8_m3": (lambda: inputs.tet3d(12), dict(degree=3, agg_size=8)),
}
_cache = {}


def _case(name):
    if name not in _cache:
        make, kw = CASES[name]
        g = make()
        ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(**kw))
        a, coef = oracle.amli_setup(ho)
        _cache[name] = (g, kw, ho, a, coef)
    return _cache[name]


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("tail_rows", [0, 4096])
@pytest.mark.parametrize("name", list(CASES))
def test_amli_matches_oracle(amg, name, tail_rows):
    g, kw, ho, a, coef = _case(name)
    p = amg.amg_params_default(cycle="amli", tail_rows=tail_rows, **kw)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    d = amg.amg_describe(h)
    assert d["n"] == [lv.n for lv in ho.levels]
    # the intervals: the same power iteration, rounding apart
    for l in range(1, ho.L):
        assert d["amli_lambda_min"][l] == pytest.approx(a[l], rel=1e-6), l
    # one cycle application with the device's intervals in the oracle
    coef_dev = {l: oracle.poly_coefficients(d["amli_lambda_min"][l]) for l in range(1, ho.L)}
    r = inputs.rhs(g.n, 61, "normal")
    z = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    amg.amg_apply_cycle(h, _t(r), z)
    zo = oracle.amli_cycle(ho, 0, r, coef_dev)
    assert np.linalg.norm(z.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
    # the solve
    f = inputs.rhs(g.n, 62)
    u = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, _t(f), u)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-8, info
    res = oracle.fcg(ho, f, precond=lambda rr: oracle.amli_cycle(ho, 0, rr, coef_dev))
    assert abs(info["iters"] - res.iters) <= 1
    e = u.cpu().numpy() - res.x
    lo = ho.levels[0]
    assert np.sqrt(e @ oracle.apply_A(lo, e)) <= 1e-6 * np.sqrt(res.x @ oracle.apply_A(lo, res.x))
    h.close()


def test_amli_mixed_precision(amg):
    g, kw, ho, a, coef = _case("grid64_agg4")
    p = amg.amg_params_default(cycle="amli", precision="mixed", **kw)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    d = amg.amg_describe(h)
    for l in range(1, ho.L):
        assert d["amli_lambda_min"][l] == pytest.approx(a[l], rel=1e-3)
    f = _t(inputs.rhs(g.n, 63))
    u = torch.zeros_like(f)
    info = amg.amg_solve(h, f, u)
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-8
    h.close()


def _device_coef(amg, h, ho):
    d = amg.amg_describe(h)
    return {l: oracle.poly_coefficients(d["amli_lambda_min"][l]) for l in range(1, ho.L)}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_amli_matches_oracle(amg, prec):
    """The batched form with the stationary cycle: grids, a geometric graph and
    a pure Neumann problem with Section 2's partitioning in one batch; each
    item against the oracle's AMLI-preconditioned CG (the device's intervals),
    and the same bits alone as in the mix."""
    specs = [(inputs.grid2d(64), dict(agg_size=4)), (inputs.rgg(5000, seed=inputs.seed_for(7, 1)), dict(agg_size=4)),
             (inputs.poisson2d(48), dict(aggregation="mis", neumann=1)), (inputs.grid2d(90, 31), dict(agg_size=8))]
    hs, fs, refs = [], [], []
    for i, (g, kw) in enumerate(specs):
        p = amg.amg_params_default(degree=4, cycle="amli", precision=prec, **kw)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(
            degree=4, agg_size=p.agg_size, aggregation="mis" if p.aggregation == amg.AMG_AGG_MIS else "matching"))
        f = inputs.rhs(g.n, 70 + i)
        if not np.any(g.d):
            f = inputs.project_range(f)
        coef = _device_coef(amg, h, ho)
        refs.append((ho, oracle.fcg(ho, f, precond=lambda r, ho=ho, coef=coef: oracle.amli_cycle(ho, 0, r, coef))))
        hs.append(h)
        fs.append(_t(f))
    us = [torch.zeros_like(f) for f in fs]
    infos = amg.amg_solve_batch(hs, fs, us)
    for i, (info, (ho, res)) in enumerate(zip(infos, refs)):
        assert info["status"] == 0 and res.converged, (i, info)
        assert info["rel_res_true"] <= 1e-8, (i, info)
        if prec == "fp64":
            assert abs(info["iters"] - res.iters) <= 1, (i, info["iters"], res.iters)
        else:
            assert info["iters"] <= res.iters + 3, (i, info["iters"], res.iters)
        lo = ho.levels[0]
        e = us[i].cpu().numpy() - res.x
        assert np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(res.x @ oracle.apply_A(lo, res.x)) <= 1e-6, i
    for i in (0, 2):
        alone = torch.zeros_like(fs[i])
        amg.amg_solve_batch([hs[i]], [fs[i]], [alone])
        assert torch.equal(alone, us[i]), i
    for h in hs:
        h.close()


def test_batch_items_share_the_cycle(amg):
    g = inputs.grid2d(40)
    hk = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(degree=4, agg_size=4))
    ha = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(degree=4, agg_size=4, cycle="amli"))
    f = _t(inputs.rhs(g.n, 3))
    with pytest.raises(amg.AmgError) as e:
        amg.amg_solve_batch([hk, ha], [f, f], [torch.zeros_like(f), torch.zeros_like(f)])
    assert e.value.code == amg.AMG_ERR_ARG
    hk.close()
    ha.close()


def test_served_amli(amg):
    """The served form with the stationary cycle: every completion against the
    oracle (the device's intervals, which a served hierarchy estimates at its
    own setup)."""
    graphs = [inputs.grid2d(50, 40), inputs.rgg(4000, seed=inputs.seed_for(7, 2))]
    reqs = []
    for i, (gid, k) in enumerate([(0, 1), (1, 2), (0, 2), (1, 1)]):
        g = graphs[gid]
        reqs.append({"arrival_s": 0.0, "graph_id": gid, "graph": g,
                     "f": np.stack([inputs.rhs(g.n, 500 + 10 * i + j) for j in range(k)])})
    p = amg.amg_params_default(degree=4, agg_size=4, cycle="amli")
    cfg = amg.amg_serve_cfg_default(p, realtime=0, iters_per_step=2)
    comps, stats, sols = amg.amg_serve(cfg, reqs)
    assert len(comps) == 6 and all(c["status"] == 0 for c in comps)
    for gid, g in enumerate(graphs):
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=4, agg_size=4))
        coef = _device_coef(amg, h, ho)
        lo = ho.levels[0]
        for i, r in enumerate(reqs):
            if r["graph_id"] != gid:
                continue
            for j, f in enumerate(np.atleast_2d(r["f"])):
                uo = oracle.fcg(ho, f, precond=lambda v: oracle.amli_cycle(ho, 0, v, coef)).x
                e = sols[i][j] - uo
                assert np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(uo @ oracle.apply_A(lo, uo)) <= 1e-6, (i, j)
        h.close()
