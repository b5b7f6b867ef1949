"""Serving (amg_serve): continuous batching over a request stream, admission
against a memory budget, and results that are the same alone and in the mix."""
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


GRAPHS = {
    0: lambda: inputs.rgg(3000, seed=inputs.seed_for(5, 0)),
    1: lambda: inputs.grid2d(60, 45),
    2: lambda: inputs.rgg(9000, seed=inputs.seed_for(5, 2)),
    3: lambda: inputs.tet3d(10),
}


@pytest.fixture(scope="module")
def graphs():
    return {k: v() for k, v in GRAPHS.items()}


def _stream(graphs, spacing=0.0):
    """Requests: a first solve on each graph, then repeats with 1..4 RHS."""
    rng = np.random.default_rng(5)
    reqs = []
    t = 0.0
    plan = [(0, 1), (1, 1), (0, 3), (2, 1), (1, 2), (3, 1), (2, 4), (0, 1), (3, 2), (1, 1)]
    for i, (gid, k) in enumerate(plan):
        g = graphs[gid]
        f = np.stack([inputs.rhs(g.n, 1000 + 10 * i + j) for j in range(k)])
        reqs.append({"arrival_s": t, "graph_id": gid, "graph": g, "f": f})
        t += spacing * rng.exponential()
    return reqs


def _params(amg, prec="mixed"):
    return amg.amg_params_default(degree=4, agg_size=8, precision=prec)


def test_serve_batched_results(amg, graphs):
    cfg = amg.amg_serve_cfg_default(_params(amg), realtime=0, iters_per_step=2)
    reqs = _stream(graphs)
    comps, stats, sols = amg.amg_serve(cfg, reqs)
    assert len(comps) == sum(np.atleast_2d(r["f"]).shape[0] for r in reqs)
    assert stats["setups"] == len(graphs)
    k = 0
    for i, r in enumerate(reqs):
        g = r["graph"]
        ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=4, agg_size=8))
        lo = ho.levels[0]
        for j, f in enumerate(np.atleast_2d(r["f"])):
            c = comps[k]
            k += 1
            assert (c["request"], c["rhs"]) == (i, j)
            assert c["status"] == 0 and c["rel_res_true"] <= 1e-8, c
            assert c["finish_s"] >= c["admit_s"] >= 0.0
            uo = oracle.fcg(ho, f).x
            e = sols[i][j] - uo
            assert np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(uo @ oracle.apply_A(lo, uo)) <= 1e-6


def test_serve_same_alone_and_in_mix(amg, graphs):
    cfg = amg.amg_serve_cfg_default(_params(amg), realtime=0, iters_per_step=3)
    reqs = _stream(graphs)
    _, _, mix = amg.amg_serve(cfg, reqs)
    for i in (2, 6, 8):
        alone_cfg = amg.amg_serve_cfg_default(_params(amg), realtime=0, iters_per_step=1)
        _, _, alone = amg.amg_serve(alone_cfg, [dict(reqs[i], arrival_s=0.0)])
        assert np.array_equal(alone[0], mix[i]), i


def test_serve_realtime_arrivals(amg, graphs):
    cfg = amg.amg_serve_cfg_default(_params(amg), realtime=1, iters_per_step=2)
    reqs = _stream(graphs, spacing=0.02)
    comps, stats, _ = amg.amg_serve(cfg, reqs)
    for c in comps:
        assert c["status"] == 0
        assert c["admit_s"] + 1e-9 >= c["arrival_s"]
        assert c["finish_s"] >= c["admit_s"]
    assert stats["wall_s"] >= reqs[-1]["arrival_s"]


def _tiny_budget(amg, graphs):
    # room for about two hierarchies at a time
    p = _params(amg, "fp64")
    sizes = []
    for g in graphs.values():
        h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
        sizes.append(amg.amg_describe(h)["device_bytes"])
        h.close()
    return int(2.5 * max(sizes))


def test_serve_tiny_budget_queues_and_evicts(amg, graphs):
    # requests must queue and graphs must be evicted, with every result still
    # correct (all requests visible at once: requests on resident graphs go
    # first, so each graph may need only one setup)
    budget = _tiny_budget(amg, graphs)
    cfg = amg.amg_serve_cfg_default(_params(amg, "fp64"), realtime=0, hbm_budget_bytes=float(budget),
                                    iters_per_step=2)
    reqs = _stream(graphs)
    comps, stats, sols = amg.amg_serve(cfg, reqs)
    assert all(c["status"] == 0 and c["rel_res_true"] <= 1e-8 for c in comps), comps
    assert stats["evictions"] >= 1 and stats["setups"] >= len(graphs)
    assert stats["peak_bytes"] <= budget
    # the same stream with room to spare gives the same bits
    cfg2 = amg.amg_serve_cfg_default(_params(amg, "fp64"), realtime=0, iters_per_step=2)
    _, _, sols2 = amg.amg_serve(cfg2, reqs)
    for a, b in zip(sols, sols2):
        assert np.array_equal(a, b)


def test_server_evicted_graph_is_set_up_again(amg, graphs):
    # one request at a time on graphs 0, 1, 2, 3 and then 0 again: graph 0 has
    # been evicted by then and is set up a second time, with the same result
    budget = _tiny_budget(amg, graphs)
    cfg = amg.amg_serve_cfg_default(_params(amg, "fp64"), hbm_budget_bytes=float(budget), iters_per_step=2)
    srv = amg.Server(cfg)
    out = []
    for gid in (0, 1, 2, 3, 0):
        g = graphs[gid]
        srv.submit(gid, inputs.rhs(g.n, 77), graph=g)
        out += _drain(srv, 1)
    stats = srv.close()
    assert len(out) == 5 and all(c["status"] == 0 and c["rel_res_true"] <= 1e-8 for c in out), out
    assert stats["evictions"] >= 1 and stats["setups"] == 5
    assert stats["peak_bytes"] <= budget
    assert np.array_equal(out[0]["u"], out[4]["u"])


def test_serve_sequential_mode(amg, graphs):
    cfg = amg.amg_serve_cfg_default(_params(amg, "fp64"), realtime=0, mode="sequential")
    reqs = _stream(graphs)
    comps, stats, sols = amg.amg_serve(cfg, reqs)
    assert all(c["status"] == 0 and c["rel_res_true"] <= 1e-8 for c in comps)
    cfgb = amg.amg_serve_cfg_default(_params(amg, "fp64"), realtime=0)
    _, _, solb = amg.amg_serve(cfgb, reqs)
    for a, b in zip(sols, solb):
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)


def test_serve_unknown_graph_without_data_fails_cleanly(amg, graphs):
    g = graphs[1]
    cfg = amg.amg_serve_cfg_default(_params(amg), realtime=0)
    reqs = [{"graph_id": 7, "graph": None, "n": g.n, "f": inputs.rhs(g.n, 1)},
            {"graph_id": 1, "graph": g, "f": inputs.rhs(g.n, 2)}]
    comps, _, _ = amg.amg_serve(cfg, reqs)
    assert comps[0]["status"] == amg.AMG_ERR_ARG
    assert comps[1]["status"] == 0


def _drain(srv, expect, wait_s=0.5, limit_s=60.0):
    """Poll until `expect` completions have come back (bounded)."""
    import time

    got = []
    t0 = time.monotonic()
    while len(got) < expect and time.monotonic() - t0 < limit_s:
        got += srv.poll(16, wait_s)
    return got


@pytest.mark.parametrize("mode", ["batched", "sequential"])
def test_server_incremental_submit_poll(amg, graphs, mode):
    # requests submitted one by one while earlier ones are in flight; every
    # solution equals the one the request gets on its own
    reqs = _stream(graphs)
    cfg = amg.amg_serve_cfg_default(_params(amg), mode=mode, iters_per_step=2)
    srv = amg.Server(cfg)
    tickets, comps = [], []
    for i, r in enumerate(reqs):
        tickets.append(srv.submit(r["graph_id"], r["f"], graph=r["graph"]))
        if i % 3 == 2:
            comps += srv.poll(16, 0.0)
    assert tickets == list(range(len(reqs)))
    total = sum(np.atleast_2d(r["f"]).shape[0] for r in reqs)
    comps += _drain(srv, total - len(comps))
    stats = srv.close()
    assert len(comps) == total
    assert sorted((c["request"], c["rhs"]) for c in comps) == [
        (i, j) for i, r in enumerate(reqs) for j in range(np.atleast_2d(r["f"]).shape[0])]
    assert stats["setups"] == len(graphs)
    for c in comps:
        assert c["status"] == 0 and c["rel_res_true"] <= 1e-8, c
        assert c["finish_s"] >= c["admit_s"] >= c["arrival_s"] - 1e-9
    alone_cfg = amg.amg_serve_cfg_default(_params(amg), mode=mode, realtime=0, iters_per_step=1)
    by = {(c["request"], c["rhs"]): c["u"] for c in comps}
    for i in (0, 6, 8):
        _, _, alone = amg.amg_serve(alone_cfg, [dict(reqs[i], arrival_s=0.0)])
        for j in range(alone[0].shape[0]):
            if mode == "batched":
                assert np.array_equal(alone[0][j], by[(i, j)]), (i, j)
            else:
                assert np.linalg.norm(alone[0][j] - by[(i, j)]) <= 1e-12 * np.linalg.norm(alone[0][j])


def test_server_resident_graph_and_errors(amg, graphs):
    g = graphs[0]
    cfg = amg.amg_serve_cfg_default(_params(amg, "fp64"))
    srv = amg.Server(cfg)
    f = inputs.rhs(g.n, 31)
    t0 = srv.submit(0, f, graph=g)
    c0 = _drain(srv, 1)
    # the graph stays resident: a later request needs no graph data
    t1 = srv.submit(0, np.stack([f, inputs.rhs(g.n, 32)]), n=g.n)
    c1 = _drain(srv, 2)
    # an unknown graph without data fails, the server goes on
    t2 = srv.submit(9, inputs.rhs(50, 33), n=50)
    c2 = _drain(srv, 1)
    with pytest.raises(amg.AmgError):
        srv.submit(0, np.zeros((1, 0)), n=0)
    assert srv.poll(4, 0.05) == []
    stats = srv.close()
    assert (t0, t1, t2) == (0, 1, 2)
    assert c0[0]["status"] == 0 and c0[0]["request"] == 0
    assert sorted(c["rhs"] for c in c1) == [0, 1] and all(c["status"] == 0 for c in c1)
    assert np.array_equal(c0[0]["u"], [c for c in c1 if c["rhs"] == 0][0]["u"])
    assert c2[0]["status"] == amg.AMG_ERR_ARG and c2[0]["request"] == 2
    assert stats["setups"] == 1
    ho = oracle.build_hierarchy(g.n, g.row_ptr, g.col, g.w, g.d, oracle.Params(degree=4, agg_size=8))
    uo = oracle.fcg(ho, f).x
    e = c0[0]["u"] - uo
    lo = ho.levels[0]
    assert np.sqrt(e @ oracle.apply_A(lo, e)) / np.sqrt(uo @ oracle.apply_A(lo, uo)) <= 1e-6
