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
    assert info["status"] == 0 and info["rel_res_true"] <= 1.05e-8, info
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
    assert info["status"] == 0 and info["rel_res_true"] <= 1.05e-8
    h.close()


def test_batched_form_rejects_amli(amg):
    g, kw, ho, a, coef = _case("grid64_agg4")
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(cycle="amli", **kw))
    f = _t(inputs.rhs(g.n, 64))
    u = torch.zeros_like(f)
    with pytest.raises(amg.AmgError):
        amg.amg_solve_batch([h], [f], [u])
    h.close()
