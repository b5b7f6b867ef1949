"""Section 4's stopping test on the device (relative A-norm of the error, the
homogeneous problem A u = 0 from a random initial guess) against the oracle,
which measures the A-norm from its definition.  Bars: outer iterations within
one; the A-norm ratio of the returned u, recomputed on the host, at most the
tolerance and equal to the one the device reports to 1e-6."""
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
    "poisson2d_72_mis_neumann": (lambda: inputs.poisson2d(72), dict(degree=4, aggregation="mis", neumann=1)),
    "poisson3d_20_mis_neumann_amli": (lambda: inputs.poisson3d(20),
                                      dict(degree=4, aggregation="mis", neumann=1, cycle="amli")),
    "grid100x37_agg4": (lambda: inputs.grid2d(100, 37), dict(degree=3, agg_size=4)),
    "delaunay11_mis2": (lambda: inputs.delaunay3d(11, seed=inputs.seed_for(6, 11)),
                        dict(degree=4, aggregation="mis", mis_distance=2)),
}


def _oracle(amg, g, p, u0):
    op = oracle.Params(degree=p.degree, agg_size=p.agg_size, coarse_max=p.coarse_max, tol=p.tol,
                       aggregation="mis" if p.aggregation == amg.AMG_AGG_MIS else "matching",
                       mis_distance=p.mis_distance, stop="energy")
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, op)
    precond = None
    if p.cycle == amg.AMG_CYCLE_AMLI:
        _, coef = oracle.amli_setup(ho)
        precond = lambda r: oracle.amli_cycle(ho, 0, r, coef)  # noqa: E731
    return ho, oracle.fcg(ho, np.zeros(g.n), u0, precond=precond)


@pytest.mark.parametrize("name", list(CASES))
def test_energy_stop_matches_oracle(amg, name):
    make, kw = CASES[name]
    g = make()
    p = amg.amg_params_default(stop="energy", **kw)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    u0 = inputs.rhs(g.n, inputs.seed_for(9))
    if not np.any(g.d):
        u0 = inputs.project_range(u0)
    ho, res = _oracle(amg, g, p, u0)
    f = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    info = amg.amg_solve(h, f, u)
    assert info["status"] == 0 and res.converged, info
    assert abs(info["iters"] - res.iters) <= 1, (info, res.iters)
    lvl = ho.levels[0]
    uh = u.cpu().numpy()
    ratio = np.sqrt(uh @ oracle.apply_A(lvl, uh)) / np.sqrt(u0 @ oracle.apply_A(lvl, u0))
    assert ratio <= p.tol, ratio
    assert info["rel_res"] == pytest.approx(ratio, rel=1e-6)


def test_energy_stop_rejects_nonzero_rhs(amg):
    g = inputs.grid2d(40)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(stop="energy"))
    f = torch.tensor(inputs.rhs(g.n, 1), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    with pytest.raises(amg.AmgError) as e:
        amg.amg_solve(h, f, u)
    assert e.value.code == amg.AMG_ERR_ARG


def test_energy_stop_zero_initial_guess(amg):
    # u0 = 0 solves A u = 0 already: no iteration
    g = inputs.grid2d(40)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(stop="energy"))
    f = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    info = amg.amg_solve(h, f, u)
    assert info["status"] == 0 and info["iters"] == 0
