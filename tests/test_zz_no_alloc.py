"""The no-allocation solve (amg_solve_noalloc) against amg_solve, through the C ABI.

Both run the same kernels in the same order; the no-allocation form keeps its
reduction scratch in the library's static device array and queues no
iteration ahead of the stopping test.  Bar (the solve's parity bar): the
iteration at which the stopping test passed is the same, executed iterations
differ by at most the one amg_solve may queue ahead, the solutions are
bitwise equal when both executed the same iterations and within 1e-6 in the
A-norm otherwise, and both true FP64 relative residuals are at most tol.
Two calls in a row, the second on a smaller system, then the first again:
the shared scratch keeps the previous call's contents, which must not leak
into the next result."""
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


def _a_norm(g, v):
    rp, c, w, d = g.row_ptr, g.col, g.w, g.d
    Av = d * v
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    np.add.at(Av, rows, w * (v[rows] - v[c]))
    return float(np.sqrt(max(v @ Av, 0.0)))


def _solve_both(amg, g, p, seed):
    dev = torch.device("cuda:0")
    h = amg.amg_setup(g.n, g.row_ptr, g.col, g.w, g.d, p)
    f = torch.tensor(inputs.rhs(g.n, seed), dtype=torch.float64, device=dev)
    u_ref = torch.zeros_like(f)
    i_ref = amg.amg_solve(h, f, u_ref, check=True)
    u_na = torch.zeros_like(f)
    i_na = amg.amg_solve_noalloc(h, f, u_na, check=True)
    torch.cuda.synchronize()
    return h, f, u_ref.cpu().numpy(), i_ref, u_na.cpu().numpy(), i_na


def _check(g, p, u_ref, i_ref, u_na, i_na, label):
    print(f"{label}: amg_solve iters {i_ref['iters']} (test {i_ref['test_iter']}), "
          f"noalloc iters {i_na['iters']} (test {i_na['test_iter']}), "
          f"true rel res {i_ref['rel_res_true']:.3e} / {i_na['rel_res_true']:.3e}", flush=True)
    assert i_na["status"] == 0 and i_ref["status"] == 0
    assert i_na["test_iter"] == i_ref["test_iter"]
    assert 0 <= i_ref["iters"] - i_na["iters"] <= 1
    assert i_na["rel_res_true"] <= p.tol and i_ref["rel_res_true"] <= p.tol
    if i_na["iters"] == i_ref["iters"]:
        assert np.array_equal(u_na, u_ref)
    else:
        assert _a_norm(g, u_na - u_ref) <= 1e-6 * _a_norm(g, u_ref)


def test_noalloc_matches_solve_twice_then_smaller(amg):
    big = inputs.grid2d(64)
    p_big = amg.amg_params_default(degree=3, agg_size=4)
    h1, f1, u_ref1, i_ref1, u_na1, i_na1 = _solve_both(amg, big, p_big, inputs.seed_for(1))
    _check(big, p_big, u_ref1, i_ref1, u_na1, i_na1, "grid64 fp64")

    small = inputs.rgg(2500, seed=inputs.seed_for(4, 7))
    assert small.n < big.n
    p_small = amg.amg_params_default(degree=4, agg_size=8, precision="mixed")
    h2, f2, u_ref2, i_ref2, u_na2, i_na2 = _solve_both(amg, small, p_small, inputs.seed_for(4, 7))
    _check(small, p_small, u_ref2, i_ref2, u_na2, i_na2, f"rgg n={small.n} mixed")

    # the first system again after the smaller one: bitwise the first result
    u_again = torch.zeros_like(f1)
    i_again = amg.amg_solve_noalloc(h1, f1, u_again, check=True)
    assert i_again["iters"] == i_na1["iters"]
    assert np.array_equal(u_again.cpu().numpy(), u_na1)
    h1.close()
    h2.close()
