"""The C ABI without a GPU: the library loads, exports every entry point that
include/amg.h declares, and reports invalid input on the host before any device
call."""
import ctypes
import os
import re

import numpy as np
import pytest

import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def amg():
    import paper_1307_6305_amd as amg

    if not os.path.exists(amg.LIB_PATH):
        from paper_1307_6305_amd import build

        build.build()
    amg.load_library()
    return amg


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(amg_[a-z_]+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(amg):
    names = _declared_functions()
    assert "amg_setup" in names and "amg_solve" in names
    lib = amg.load_library()
    for name in names:
        assert hasattr(lib, name), name
        assert name in amg.SIGNATURES, f"binding lacks {name}"


def test_params_default(amg):
    p = amg.amg_params_default()
    assert (p.degree, p.agg_size, p.coarse_max, p.inner_steps, p.restart) == (4, 4, 64, 2, 5)
    assert p.lambda0_ratio == 10.0 and p.tol == 1e-8 and p.precision == amg.AMG_FP64
    assert (p.autotune, p.slice_height, p.lanes_per_row, p.sort_rows) == (1, 64, 1, 0)
    assert p.tie_break == amg.AMG_TIE_INDEX and amg.amg_params_default(tie_break="hash").tie_break == amg.AMG_TIE_HASH
    assert p.fuse == 1 and p.smoother_rho == 0.33 and p.cycle == amg.AMG_CYCLE_K
    assert (p.aggregation, p.mis_distance, p.neumann) == (amg.AMG_AGG_MATCHING, 4, 0)
    assert p.stop == amg.AMG_STOP_RESIDUAL and amg.amg_params_default(stop="energy").stop == amg.AMG_STOP_ENERGY
    assert amg.amg_params_default(aggregation="mis").aggregation == amg.AMG_AGG_MIS
    with pytest.raises(TypeError):
        amg.amg_params_default(no_such_field=1)


def test_strerror(amg):
    assert amg.amg_strerror(0) == "ok"
    assert "degree" in amg.amg_strerror(amg.AMG_ERR_DEGREE)


def _setup_code(amg, n, rp, col, w, d, params=None):
    lib = amg.load_library()
    out = ctypes.c_void_p()
    p = params if params is not None else amg.amg_params_default()
    P = ctypes.c_void_p
    rp = np.ascontiguousarray(rp, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    w = np.ascontiguousarray(w, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    code = lib.amg_setup(n, rp.ctypes.data_as(P), col.ctypes.data_as(P), w.ctypes.data_as(P),
                         d.ctypes.data_as(P), ctypes.byref(p), None, ctypes.byref(out))
    return code, out


def test_validation_errors_before_device(amg):
    g = inputs.grid2d(5)
    # self loop
    col = g.col.copy()
    col[0] = 0
    assert _setup_code(amg, g.n, g.row_ptr, col, g.w, g.d)[0] == amg.AMG_ERR_GRAPH
    # asymmetric weight
    w = g.w.copy()
    w[0] = 2.0
    assert _setup_code(amg, g.n, g.row_ptr, g.col, w, g.d)[0] == amg.AMG_ERR_GRAPH
    # non-positive weight
    w = g.w.copy()
    w[:] = -1.0
    assert _setup_code(amg, g.n, g.row_ptr, g.col, w, g.d)[0] == amg.AMG_ERR_GRAPH
    # all d = 0: singular
    assert _setup_code(amg, g.n, g.row_ptr, g.col, g.w, np.zeros(g.n))[0] == amg.AMG_ERR_SINGULAR
    # negative d
    d = g.d.copy()
    d[3] = -1
    assert _setup_code(amg, g.n, g.row_ptr, g.col, g.w, d)[0] == amg.AMG_ERR_GRAPH
    # disconnected: two copies of the grid side by side
    rp2 = np.concatenate([g.row_ptr, g.row_ptr[1:] + g.row_ptr[-1]])
    col2 = np.concatenate([g.col, g.col + g.n])
    code, _ = _setup_code(amg, 2 * g.n, rp2, col2, np.concatenate([g.w, g.w]), np.concatenate([g.d, g.d]))
    assert code == amg.AMG_ERR_DISCONNECTED
    # smoother degree too low (E_2 > 1 at kappa = 10)
    assert _setup_code(amg, g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(degree=2))[0] == \
        amg.AMG_ERR_DEGREE
    # bad parameters
    assert _setup_code(amg, g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(restart=0))[0] == \
        amg.AMG_ERR_ARG
    assert _setup_code(amg, 0, g.row_ptr, g.col, g.w, g.d)[0] == amg.AMG_ERR_ARG
    for bad in (dict(slice_height=4), dict(slice_height=48), dict(lanes_per_row=3), dict(lanes_per_row=8),
                dict(sort_rows=2), dict(autotune=-1), dict(tie_break=2), dict(fuse=2),
                dict(degree=-2), dict(degree=-1, smoother_rho=0.0), dict(degree=-1, smoother_rho=1.5),
                dict(cycle=2), dict(cycle=1, inner_steps=3), dict(aggregation=2), dict(aggregation=-1),
                dict(aggregation=1, mis_distance=0), dict(aggregation=1, mis_distance=9), dict(neumann=2),
                dict(stop=2), dict(stop=-1)):
        code = _setup_code(amg, g.n, g.row_ptr, g.col, g.w, g.d, amg.amg_params_default(**bad))[0]
        assert code == amg.AMG_ERR_ARG, bad
    # unsorted columns
    col = g.col.copy()
    col[g.row_ptr[7]], col[g.row_ptr[7] + 1] = col[g.row_ptr[7] + 1], col[g.row_ptr[7]]
    assert _setup_code(amg, g.n, g.row_ptr, col, g.w, g.d)[0] == amg.AMG_ERR_GRAPH
    assert "increasing" in amg.amg_last_error()


def test_valid_input_without_gpu_reports_device(amg):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = inputs.grid2d(5)
    code, out = _setup_code(amg, g.n, g.row_ptr, g.col, g.w, g.d)
    assert code == amg.AMG_ERR_DEVICE and not out.value
    # a pure Neumann problem (d = 0) passes validation when neumann = 1
    p = amg.amg_params_default(aggregation="mis", neumann=1)
    code, out = _setup_code(amg, g.n, g.row_ptr, g.col, g.w, np.zeros(g.n), p)
    assert code == amg.AMG_ERR_DEVICE and not out.value


def test_server_argument_errors_before_device(amg):
    lib = amg.load_library()
    hnd = ctypes.c_void_p()
    assert lib.amg_server_create(None, None, ctypes.byref(hnd)) == amg.AMG_ERR_ARG and not hnd.value
    for bad in (dict(mode=7), dict(max_slots=0), dict(hbm_budget_bytes=0.0)):
        cfg = amg.amg_serve_cfg_default(**bad)
        assert lib.amg_server_create(ctypes.byref(cfg), None, ctypes.byref(hnd)) == amg.AMG_ERR_ARG, bad
        assert not hnd.value
    cfg = amg.amg_serve_cfg_default(amg.amg_params_default(restart=0))
    assert lib.amg_server_create(ctypes.byref(cfg), None, ctypes.byref(hnd)) == amg.AMG_ERR_ARG
    cfg = amg.amg_serve_cfg_default(amg.amg_params_default(stop="energy"))
    assert lib.amg_server_create(ctypes.byref(cfg), None, ctypes.byref(hnd)) == amg.AMG_ERR_ARG
    assert lib.amg_server_create(ctypes.byref(amg.amg_serve_cfg_default()), None, None) == amg.AMG_ERR_ARG
    cnt = ctypes.c_int32()
    out = (amg.amg_completion * 2)()
    assert lib.amg_server_submit(None, None, None) == amg.AMG_ERR_ARG
    assert lib.amg_server_poll(None, out, 2, 0.0, ctypes.byref(cnt)) == amg.AMG_ERR_ARG
    assert lib.amg_server_destroy(None, None) == amg.AMG_OK


def test_server_without_gpu_reports_device(amg):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    hnd = ctypes.c_void_p()
    cfg = amg.amg_serve_cfg_default()
    assert amg.load_library().amg_server_create(ctypes.byref(cfg), None, ctypes.byref(hnd)) == amg.AMG_ERR_DEVICE
    assert not hnd.value
