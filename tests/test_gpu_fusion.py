"""Kernel fusion on launch-bound levels (folded inner flexible-CG updates,
residual and restriction in one pass) must not change a single bit: every
fused kernel computes exactly the values the separate steps would store."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def amg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1307_6305_amd as amg

    amg.load_library()
    return amg


GRAPHS = {
    "grid160": lambda: inputs.grid2d(160, 160),
    "rgg30k": lambda: inputs.rgg(30000, seed=inputs.seed_for(6, 1)),
    "tet14": lambda: inputs.tet3d(14),
}


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("tail_rows", [0, 4096])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_fused_equals_unfused(amg, name, prec, tail_rows):
    g = GRAPHS[name]()
    f = _t(inputs.rhs(g.n, 41))
    r = _t(inputs.rhs(g.n, 42, "normal"))
    out = []
    for fuse in (1, 0):
        p = amg.amg_params_default(degree=3, agg_size=4, precision=prec, fuse=fuse, tail_rows=tail_rows)
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        u = torch.zeros_like(f)
        info = amg.amg_solve(h, f, u)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8, info
        z = torch.zeros_like(r)
        amg.amg_apply_cycle(h, r, z)
        torch.cuda.synchronize()
        out.append((u, info["iters"], z))
        h.close()
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][2], out[1][2]), "cycle"
    assert torch.equal(out[0][0], out[1][0]), "solve"
