"""Sliced-ELL layouts (slice height, lanes per row, rows sorted inside 64-row groups)
and their autotuner: every layout must give the same bits -- the row sums are
added in a fixed order of entry classes and inner products in row order -- so
the choice the autotuner makes can only change speed."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LAYOUTS = [(h, k, s) for (h, k) in [(64, 1), (32, 1), (16, 1), (8, 1), (32, 2), (16, 4)] for s in (0, 1)]


@pytest.fixture(scope="module")
def amg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1307_6305_amd as amg

    amg.load_library()
    return amg


GRAPHS = {
    # uneven degrees (1..18): sorting matters
    "rgg40k": lambda: inputs.rgg(40000, seed=inputs.seed_for(4, 7)),
    "grid70x33": lambda: inputs.grid2d(70, 33),
    "tet12": lambda: inputs.tet3d(12),
}

_graphs = {}


def _graph(name):
    if name not in _graphs:
        _graphs[name] = GRAPHS[name]()
    return _graphs[name]


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _setup(amg, g, prec, layout=None, **kw):
    if layout is None:
        p = amg.amg_params_default(degree=4, agg_size=8, precision=prec, autotune=1, **kw)
    else:
        sh, k, srt = layout
        p = amg.amg_params_default(degree=4, agg_size=8, precision=prec, autotune=0, slice_height=sh,
                                   lanes_per_row=k, sort_rows=srt, **kw)
    return amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_layouts_same_bits(amg, name, prec):
    g = _graph(name)
    r = _t(inputs.rhs(g.n, 11, "normal"))
    f = _t(inputs.rhs(g.n, 12))
    ref = None
    for layout in LAYOUTS + [None]:
        h = _setup(amg, g, prec, layout)
        desc = amg.amg_describe(h)
        if layout is not None:
            for lay in desc["layouts"]:
                assert (lay["slice_height"], lay["lanes_per_row"], lay["sorted_rows"]) == layout
        z = torch.zeros_like(r)
        amg.amg_apply_cycle(h, r, z)
        u = torch.zeros_like(f)
        info = amg.amg_solve(h, f, u)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8, (layout, info)
        y = None
        if prec == "fp64":
            y = torch.zeros_like(r)
            amg.amg_apply_smoother(h, 0, r, y)
        torch.cuda.synchronize()
        if ref is None:
            ref = (z, u, info["iters"], y)
        else:
            assert torch.equal(z, ref[0]), (layout, "cycle")
            assert torch.equal(u, ref[1]), (layout, "solve")
            assert info["iters"] == ref[2], layout
            if y is not None:
                assert torch.equal(y, ref[3]), (layout, "smoother")
        h.close()


def test_layout_cycle_matches_oracle(amg):
    g = _graph("rgg40k")
    p = amg.amg_params_default(degree=4, agg_size=8, autotune=0, slice_height=16, lanes_per_row=1, sort_rows=1)
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=4, agg_size=8))
    r = inputs.rhs(g.n, 13, "normal")
    z = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    amg.amg_apply_cycle(h, _t(r), z)
    zo = oracle.kcycle(ho, 0, r)
    assert np.linalg.norm(z.cpu().numpy() - zo) / np.linalg.norm(zo) <= 1e-10


def test_tail_with_sorted_layouts(amg):
    # every level in a sorted 16-row layout, the tail taking the largest level that fits
    g = _graph("rgg40k")
    f = _t(inputs.rhs(g.n, 14))
    outs = []
    for tail_rows in (0, 70000):
        h = _setup(amg, g, "fp64", (16, 1, 1), tail_rows=tail_rows)
        u = torch.zeros_like(f)
        info = amg.amg_solve(h, f, u)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8
        outs.append((u, info["iters"]))
        h.close()
    # tail and kernels add their inner products in different trees: same solution to solver accuracy
    assert abs(outs[0][1] - outs[1][1]) <= 1
    assert float((outs[0][0] - outs[1][0]).norm() / outs[0][0].norm()) <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_mixed_layouts(amg, prec):
    # items with different layouts (1, 2 and 4 lanes per row) share launches
    gs = [_graph("rgg40k"), _graph("grid70x33"), _graph("tet12"), _graph("rgg40k")]
    lays = [(16, 1, 1), (32, 2, 0), (16, 4, 1), (64, 1, 0)]
    hs = [_setup(amg, g, prec, lay) for g, lay in zip(gs, lays)]
    fs = [_t(inputs.rhs(g.n, 20 + i)) for i, g in enumerate(gs)]
    us = [torch.zeros_like(f) for f in fs]
    infos = amg.amg_solve_batch(hs, fs, us)
    assert all(i["status"] == 0 and i["rel_res_true"] <= 1e-8 for i in infos), infos
    # the same systems with the default layout, one at a time in the batched path
    for k, g in enumerate(gs):
        h1 = _setup(amg, g, prec, (64, 1, 0))
        u1 = torch.zeros_like(fs[k])
        inf1 = amg.amg_solve_batch([h1], [fs[k]], [u1])
        assert inf1[0]["iters"] == infos[k]["iters"]
        assert torch.equal(u1, us[k]), k
        h1.close()
    for h in hs:
        h.close()


def test_autotuner_reports(amg):
    # 150k rows: the finest level is large enough to be timed
    g = inputs.rgg(150000, seed=inputs.seed_for(4, 8))
    h = _setup(amg, g, "mixed")
    d = amg.amg_describe(h)
    assert d["layout_ms"] > 0.0
    for lay, nnz in zip(d["layouts"], d["nnz"]):
        assert lay["slice_height"] in (8, 16, 32, 64) and lay["lanes_per_row"] in (1, 2, 4)
        assert lay["entries"] >= nnz
    # the same graph with a fixed layout gives the same solution bits
    f = _t(inputs.rhs(g.n, 15))
    u = torch.zeros_like(f)
    amg.amg_solve(h, f, u)
    h2 = _setup(amg, g, "mixed", (64, 1, 0))
    u2 = torch.zeros_like(f)
    amg.amg_solve(h2, f, u2)
    assert torch.equal(u, u2)
