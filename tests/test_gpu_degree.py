"""Automatic smoother degree (degree = -1): the hierarchy uses the smallest m
of the bound on m (Section 3) and then behaves exactly as with that m given."""
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


@pytest.mark.parametrize("rho,ratio", [(0.33, 10.0), (0.1, 10.0), (0.05, 30.0)])
def test_auto_degree(amg, rho, ratio):
    g = inputs.grid2d(96, 80)
    m = oracle.degree_for(rho, ratio)
    f = torch.tensor(inputs.rhs(g.n, 51), dtype=torch.float64, device="cuda")
    out = []
    for deg in (-1, m):
        p = amg.amg_params_default(degree=deg, smoother_rho=rho, lambda0_ratio=ratio, agg_size=8)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        assert amg.amg_describe(h)["degree"] == m
        u = torch.zeros_like(f)
        info = amg.amg_solve(h, f, u)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8
        out.append(u)
        h.close()
    assert torch.equal(out[0], out[1])
