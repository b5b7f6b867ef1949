"""Python binding of the MI355X graph-Laplacian solver (C ABI in include/amg.h).

The binding only marshals arguments: every step of setup and solve runs in the
HIP library ``libamg.so`` built from ``csrc/``.  Device vectors are torch
tensors on the current HIP device (float64, contiguous); graphs are host numpy
arrays.  The functions keep the names of the C entry points.

There is no fallback: if the library is missing or cannot be loaded, importing
the binding's entry points raises.
"""
from __future__ import annotations

import ctypes
import threading
import os

import numpy as np

try:  # torch first: the library must bind to the HIP runtime torch already loaded
    import torch
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamg.so")

AMG_OK = 0
AMG_ERR_ARG = -1
AMG_ERR_GRAPH = -2
AMG_ERR_DISCONNECTED = -3
AMG_ERR_SINGULAR = -4
AMG_ERR_DEGREE = -5
AMG_ERR_COARSEN = -6
AMG_ERR_NOMEM = -7
AMG_ERR_DEVICE = -8
AMG_ERR_BREAKDOWN = -9
AMG_ERR_MAXIT = -10
AMG_ERR_BUDGET = -11
AMG_FP64 = 0
AMG_MIXED = 1
AMG_KEY_NORMALIZED = 0
AMG_KEY_RAW = 1
AMG_TIE_INDEX = 0
AMG_TIE_HASH = 1
AMG_CYCLE_K = 0
AMG_CYCLE_AMLI = 1
AMG_AGG_MATCHING = 0
AMG_AGG_MIS = 1
AMG_STOP_RESIDUAL = 0
AMG_STOP_ENERGY = 1
AMG_MAX_LEVELS = 32


class amg_params(ctypes.Structure):
    _fields_ = [
        ("degree", ctypes.c_int32),
        ("agg_size", ctypes.c_int32),
        ("coarse_max", ctypes.c_int32),
        ("lambda0_ratio", ctypes.c_double),
        ("inner_steps", ctypes.c_int32),
        ("restart", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("match_key", ctypes.c_int32),
        ("max_coarsest", ctypes.c_int32),
        ("stagnation", ctypes.c_double),
        ("use_graph", ctypes.c_int32),
        ("tail_rows", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("slice_height", ctypes.c_int32),
        ("lanes_per_row", ctypes.c_int32),
        ("sort_rows", ctypes.c_int32),
        ("tie_break", ctypes.c_int32),
        ("fuse", ctypes.c_int32),
        ("smoother_rho", ctypes.c_double),
        ("cycle", ctypes.c_int32),
        ("aggregation", ctypes.c_int32),
        ("mis_distance", ctypes.c_int32),
        ("neumann", ctypes.c_int32),
        ("stop", ctypes.c_int32),
    ]


class amg_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("rel_res", ctypes.c_double),
        ("rel_res_true", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("test_iter", ctypes.c_int32),
        ("replacements", ctypes.c_int32),
    ]


def _info_dict(i: amg_info) -> dict:
    return {"status": i.status, "iters": i.iters, "rel_res": i.rel_res, "rel_res_true": i.rel_res_true,
            "solve_ms": i.solve_ms, "test_iter": i.test_iter, "replacements": i.replacements}


class amg_hier_desc(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("n", ctypes.c_int32 * AMG_MAX_LEVELS),
        ("nnz", ctypes.c_int64 * AMG_MAX_LEVELS),
        ("lambda1", ctypes.c_double * AMG_MAX_LEVELS),
        ("grid_complexity", ctypes.c_double),
        ("operator_complexity", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("aggregation_ms", ctypes.c_double),
        ("galerkin_ms", ctypes.c_double),
        ("match_rounds", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("device_bytes", ctypes.c_double),
        ("layout_ms", ctypes.c_double),
        ("slice_height", ctypes.c_int32 * AMG_MAX_LEVELS),
        ("lanes_per_row", ctypes.c_int32 * AMG_MAX_LEVELS),
        ("sorted_rows", ctypes.c_int32 * AMG_MAX_LEVELS),
        ("sell_entries", ctypes.c_int64 * AMG_MAX_LEVELS),
        ("degree", ctypes.c_int32),
        ("amli_lambda_min", ctypes.c_double * AMG_MAX_LEVELS),
    ]


class amg_kernel_timing(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int32),
        ("avg_ms", ctypes.c_double),
        ("rows", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("entries", ctypes.c_int64),
        ("grid", ctypes.c_int32),
        ("value_bytes", ctypes.c_int32),
    ]


AMG_SERVE_BATCHED = 0
AMG_SERVE_SEQUENTIAL = 1


class amg_request(ctypes.Structure):
    _fields_ = [
        ("arrival_s", ctypes.c_double),
        ("graph_id", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("row_ptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("d", ctypes.c_void_p),
        ("nrhs", ctypes.c_int32),
        ("f", ctypes.c_void_p),
        ("u", ctypes.c_void_p),
    ]


class amg_completion(ctypes.Structure):
    _fields_ = [
        ("request", ctypes.c_int32),
        ("rhs", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("rel_res_true", ctypes.c_double),
        ("arrival_s", ctypes.c_double),
        ("admit_s", ctypes.c_double),
        ("finish_s", ctypes.c_double),
    ]


class amg_serve_cfg(ctypes.Structure):
    _fields_ = [
        ("params", amg_params),
        ("hbm_budget_bytes", ctypes.c_double),
        ("max_slots", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("iters_per_step", ctypes.c_int32),
        ("realtime", ctypes.c_int32),
    ]


class amg_serve_stats(ctypes.Structure):
    _fields_ = [
        ("wall_s", ctypes.c_double),
        ("peak_bytes", ctypes.c_double),
        ("evictions", ctypes.c_int32),
        ("setups", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("max_in_flight", ctypes.c_int32),
        ("schedule_s", ctypes.c_double),
        ("admit_s", ctypes.c_double),
        ("release_s", ctypes.c_double),
        ("iterate_s", ctypes.c_double),
    ]


class AmgError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        super().__init__(f"{where}: {amg_strerror(code)} ({code}): {detail}")


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32

# C signatures: name -> (restype, argtypes)
SIGNATURES = {
    "amg_params_default": (None, [ctypes.POINTER(amg_params)]),
    "amg_strerror": (ctypes.c_char_p, [_I32]),
    "amg_last_error": (ctypes.c_char_p, []),
    "amg_setup": (_I32, [_I32, _P, _P, _P, _P, ctypes.POINTER(amg_params), _P, ctypes.POINTER(_P)]),
    "amg_free": (None, [_P]),
    "amg_describe": (_I32, [_P, ctypes.POINTER(amg_hier_desc)]),
    "amg_solve": (_I32, [_P, _P, _P, _P, ctypes.POINTER(amg_info)]),
    "amg_solve_noalloc": (_I32, [_P, _P, _P, _P, ctypes.POINTER(amg_info)]),
    "amg_solve_batch": (_I32, [_I32, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), _P,
                               ctypes.POINTER(amg_info)]),
    "amg_serve_cfg_default": (None, [ctypes.POINTER(amg_serve_cfg)]),
    "amg_serve": (_I32, [ctypes.POINTER(amg_serve_cfg), ctypes.POINTER(amg_request), _I32,
                         ctypes.POINTER(amg_completion), ctypes.POINTER(amg_serve_stats), _P]),
    "amg_server_create": (_I32, [ctypes.POINTER(amg_serve_cfg), _P, ctypes.POINTER(_P)]),
    "amg_server_submit": (_I32, [_P, ctypes.POINTER(amg_request), ctypes.POINTER(_I32)]),
    "amg_server_poll": (_I32, [_P, ctypes.POINTER(amg_completion), _I32, ctypes.c_double, ctypes.POINTER(_I32)]),
    "amg_server_destroy": (_I32, [_P, ctypes.POINTER(amg_serve_stats)]),
    "amg_time_step": (_I32, [_P, _I32, _P, ctypes.POINTER(amg_kernel_timing)]),
    "amg_time_step_rotating": (_I32, [_P, _I32, _I32, _P, ctypes.POINTER(amg_kernel_timing)]),
    "amg_level_export": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P]),
    "amg_apply_smoother": (_I32, [_P, _I32, _P, _P, _P]),
    "amg_apply_residual": (_I32, [_P, _I32, _P, _P, _P, _P]),
    "amg_apply_restrict": (_I32, [_P, _I32, _P, _P, _P]),
    "amg_apply_prolong": (_I32, [_P, _I32, _P, _P, _P]),
    "amg_apply_coarse": (_I32, [_P, _P, _P, _P]),
    "amg_apply_cycle": (_I32, [_P, _P, _P, _P]),
}


def load_library(path: str = LIB_PATH):
    """Load libamg.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code: int, where: str):
    if code != AMG_OK:
        raise AmgError(code, where, load_library().amg_last_error().decode())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, n: int | None = None, name: str = "vector"):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def amg_strerror(code: int) -> str:
    return load_library().amg_strerror(int(code)).decode()


def amg_last_error() -> str:
    return load_library().amg_last_error().decode()


def amg_params_default(**overrides) -> amg_params:
    p = amg_params()
    load_library().amg_params_default(ctypes.byref(p))
    names = {f[0] for f in amg_params._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise TypeError(f"amg_params has no field {k!r}")
        if k == "precision" and isinstance(v, str):
            v = {"fp64": AMG_FP64, "mixed": AMG_MIXED}[v]
        if k == "match_key" and isinstance(v, str):
            v = {"normalized": AMG_KEY_NORMALIZED, "raw": AMG_KEY_RAW}[v]
        if k == "tie_break" and isinstance(v, str):
            v = {"index": AMG_TIE_INDEX, "hash": AMG_TIE_HASH}[v]
        if k == "cycle" and isinstance(v, str):
            v = {"k": AMG_CYCLE_K, "amli": AMG_CYCLE_AMLI}[v]
        if k == "aggregation" and isinstance(v, str):
            v = {"matching": AMG_AGG_MATCHING, "mis": AMG_AGG_MIS}[v]
        if k == "stop" and isinstance(v, str):
            v = {"residual": AMG_STOP_RESIDUAL, "energy": AMG_STOP_ENERGY}[v]
        setattr(p, k, v)
    return p


class Hierarchy:
    """Owns an amg_hier handle; amg_free runs when it is collected or closed."""

    def __init__(self, handle: int, n: int, params: amg_params):
        self.handle = ctypes.c_void_p(handle)
        self.n = n
        self.params = params

    def close(self):
        if self.handle and self.handle.value:
            load_library().amg_free(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def amg_setup(n, row_ptr, col, w, d, params: amg_params | None = None, stream=None) -> Hierarchy:
    """Build the hierarchy from host CSR arrays (copied by the library)."""
    lib = load_library()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    wv = np.ascontiguousarray(w, dtype=np.float64)
    dv = np.ascontiguousarray(d, dtype=np.float64)
    p = params if params is not None else amg_params_default()
    out = ctypes.c_void_p()
    st = _stream(stream) if torch is not None and torch.cuda.is_available() else ctypes.c_void_p(None)
    code = lib.amg_setup(int(n), rp.ctypes.data_as(_P), cl.ctypes.data_as(_P), wv.ctypes.data_as(_P),
                         dv.ctypes.data_as(_P), ctypes.byref(p), st, ctypes.byref(out))
    _check(code, "amg_setup")
    return Hierarchy(out.value, int(n), p)


def amg_free(h: Hierarchy):
    h.close()


def amg_describe(h: Hierarchy) -> dict:
    ds = amg_hier_desc()
    _check(load_library().amg_describe(h.handle, ctypes.byref(ds)), "amg_describe")
    L = ds.levels
    return {
        "levels": L,
        "n": list(ds.n[:L]),
        "nnz": list(ds.nnz[:L]),
        "lambda1": list(ds.lambda1[:L]),
        "grid_complexity": ds.grid_complexity,
        "operator_complexity": ds.operator_complexity,
        "setup_ms": ds.setup_ms,
        "aggregation_ms": ds.aggregation_ms,
        "galerkin_ms": ds.galerkin_ms,
        "match_rounds": ds.match_rounds,
        "precision": ds.precision,
        "device_bytes": ds.device_bytes,
        "layout_ms": ds.layout_ms,
        "degree": ds.degree,
        "amli_lambda_min": list(ds.amli_lambda_min[:L]),
        # sliced-ELL layout of every smoothed level (the finest at least)
        "layouts": [{"slice_height": ds.slice_height[l], "lanes_per_row": ds.lanes_per_row[l],
                     "sorted_rows": ds.sorted_rows[l], "entries": ds.sell_entries[l]}
                    for l in range(max(L - 1, 1))],
    }


def amg_solve(h: Hierarchy, f, u, stream=None, check: bool = False) -> dict:
    """Solve A u = f (u: initial guess in, solution out).  Returns the info
    record; raises only for argument/device errors unless ``check``."""
    info = amg_info()
    code = load_library().amg_solve(h.handle, _dev(f, h.n, "f"), _dev(u, h.n, "u"), _stream(stream),
                                    ctypes.byref(info))
    if code in (AMG_ERR_ARG, AMG_ERR_DEVICE, AMG_ERR_NOMEM) or (check and code != AMG_OK):
        _check(code, "amg_solve")
    return _info_dict(info)


def amg_solve_noalloc(h: Hierarchy, f, u, stream=None, check: bool = False) -> dict:
    """amg_solve with its reduction scratch in the library's static device
    array: no allocation, no graphs, no events (include/amg.h)."""
    info = amg_info()
    code = load_library().amg_solve_noalloc(h.handle, _dev(f, h.n, "f"), _dev(u, h.n, "u"), _stream(stream),
                                            ctypes.byref(info))
    if code in (AMG_ERR_ARG, AMG_ERR_DEVICE, AMG_ERR_NOMEM) or (check and code != AMG_OK):
        _check(code, "amg_solve_noalloc")
    return _info_dict(info)


def amg_solve_batch(hs, fs, us, stream=None, check: bool = False) -> list:
    """Solve len(hs) systems together; hs may repeat (several right-hand
    sides).  fs/us: float64 device tensors.  Returns one info dict per item."""
    nb = len(hs)
    if not (nb == len(fs) == len(us)) or nb < 1:
        raise ValueError("hs, fs and us must have the same positive length")
    H = (_P * nb)(*[h.handle.value for h in hs])
    F = (_P * nb)(*[_dev(f, h.n, "f").value for h, f in zip(hs, fs)])
    U = (_P * nb)(*[_dev(u, h.n, "u").value for h, u in zip(hs, us)])
    infos = (amg_info * nb)()
    code = load_library().amg_solve_batch(nb, H, F, U, _stream(stream), infos)
    if code in (AMG_ERR_ARG, AMG_ERR_DEVICE, AMG_ERR_NOMEM) or (check and code != AMG_OK):
        _check(code, "amg_solve_batch")
    return [_info_dict(i) for i in infos]


def amg_serve_cfg_default(params: amg_params | None = None, **overrides) -> amg_serve_cfg:
    c = amg_serve_cfg()
    load_library().amg_serve_cfg_default(ctypes.byref(c))
    if params is not None:
        c.params = params
    for k, v in overrides.items():
        if k == "mode" and isinstance(v, str):
            v = {"batched": AMG_SERVE_BATCHED, "sequential": AMG_SERVE_SEQUENTIAL}[v]
        setattr(c, k, v)
    return c


def _completion_dict(c) -> dict:
    return {"request": c.request, "rhs": c.rhs, "status": c.status, "iters": c.iters,
            "rel_res_true": c.rel_res_true, "arrival_s": c.arrival_s, "admit_s": c.admit_s,
            "finish_s": c.finish_s}


def _stats_dict(stats) -> dict:
    return {"wall_s": stats.wall_s, "peak_bytes": stats.peak_bytes, "evictions": stats.evictions,
            "setups": stats.setups, "steps": stats.steps, "max_in_flight": stats.max_in_flight,
            "schedule_s": stats.schedule_s, "admit_s": stats.admit_s, "release_s": stats.release_s,
            "iterate_s": stats.iterate_s}


class Server:
    """Incremental server (amg_server_create/submit/poll/destroy): requests
    are submitted one at a time while earlier ones are being solved.  The
    solution buffers of a request are kept here until all of its completions
    have been polled."""

    def __init__(self, cfg: amg_serve_cfg, stream=None):
        self._lib = load_library()
        self._cfg = cfg
        hnd = _P()
        _check(self._lib.amg_server_create(ctypes.byref(cfg), _stream(stream), ctypes.byref(hnd)),
               "amg_server_create")
        self.handle = hnd
        self._pending = {}  # ticket -> [solution array, completions still to come]
        self._polled = 0
        self._submitted = 0  # tickets are handed out in submission order
        self._lock = threading.Lock()  # submit and poll may run on different threads

    def submit(self, graph_id: int, f, graph=None, n: int | None = None) -> int:
        """Submit right-hand sides f ((nrhs, n) or (n,)) for graph ``graph_id``;
        ``graph`` (n, row_ptr, col, w, d) is needed unless that graph is
        resident.  Returns the ticket."""
        f = np.ascontiguousarray(np.atleast_2d(np.asarray(f, dtype=np.float64)))
        nn = graph.n if graph is not None else int(n if n is not None else f.shape[1])
        if f.shape[1] != nn:
            raise ValueError(f"f has {f.shape[1]} columns, graph has {nn} vertices")
        r = amg_request()
        r.graph_id = int(graph_id)
        r.n = nn
        keep = []
        if graph is not None:
            rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int32)
            cl = np.ascontiguousarray(graph.col, dtype=np.int32)
            wv = np.ascontiguousarray(graph.w, dtype=np.float64)
            dv = np.ascontiguousarray(graph.d, dtype=np.float64)
            keep += [rp, cl, wv, dv]
            r.row_ptr, r.col, r.w, r.d = (a.ctypes.data for a in (rp, cl, wv, dv))
        r.nrhs = f.shape[0]
        r.f = f.ctypes.data
        u = np.zeros_like(f)
        r.u = u.ctypes.data
        ticket = _I32(-1)
        with self._lock:
            # registered before the call: a poll on another thread may see
            # the completion as soon as the server has the request
            expect = self._submitted
            self._pending[expect] = [u, f.shape[0]]
            code = self._lib.amg_server_submit(self.handle, ctypes.byref(r), ctypes.byref(ticket))
            if code != AMG_OK:
                del self._pending[expect]
            else:
                self._submitted += 1
                if ticket.value != expect:
                    self._pending[ticket.value] = self._pending.pop(expect)
        _check(code, "amg_server_submit")
        return ticket.value

    def poll(self, max_count: int = 64, wait_s: float = 0.0):
        """Finished completions (oldest first), each a dict with the ticket
        in "request" and the solution row in "u"."""
        out = (amg_completion * max_count)()
        cnt = _I32(0)
        code = self._lib.amg_server_poll(self.handle, out, max_count, float(wait_s), ctypes.byref(cnt))
        res = []
        with self._lock:
            for c in out[:cnt.value]:
                d = _completion_dict(c)
                ent = self._pending[c.request]
                d["u"] = ent[0][c.rhs]
                ent[1] -= 1
                if ent[1] == 0:
                    del self._pending[c.request]
                res.append(d)
        _check(code, "amg_server_poll")
        return res

    def close(self) -> dict:
        """Finish every submitted request, stop the server, return its stats."""
        if self.handle is None:
            return {}
        stats = amg_serve_stats()
        code = self._lib.amg_server_destroy(self.handle, ctypes.byref(stats))
        self.handle = None
        self._pending.clear()
        _check(code, "amg_server_destroy")
        return _stats_dict(stats)

    def __del__(self):
        try:
            if self.handle is not None:
                self._lib.amg_server_destroy(self.handle, None)
        except Exception:
            pass


def amg_serve(cfg: amg_serve_cfg, requests: list, stream=None, want_u: bool = True):
    """Replay a request stream.  Each request is a dict with keys arrival_s,
    graph_id, graph (an object with n, row_ptr, col, w, d; may be None when the
    graph is resident) or n, and f (array of shape (nrhs, n) or (n,)).
    Returns (completions: list of dicts, stats: dict, solutions: list of
    (nrhs, n) arrays or None)."""
    keep = []
    reqs = (amg_request * len(requests))()
    sols = []
    for i, rq in enumerate(requests):
        g = rq.get("graph")
        f = np.ascontiguousarray(np.atleast_2d(np.asarray(rq["f"], dtype=np.float64)))
        n = g.n if g is not None else int(rq["n"])
        if f.shape[1] != n:
            raise ValueError(f"request {i}: f has {f.shape[1]} columns, graph has {n} vertices")
        r = reqs[i]
        r.arrival_s = float(rq.get("arrival_s", 0.0))
        r.graph_id = int(rq["graph_id"])
        r.n = n
        if g is not None:
            rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
            cl = np.ascontiguousarray(g.col, dtype=np.int32)
            wv = np.ascontiguousarray(g.w, dtype=np.float64)
            dv = np.ascontiguousarray(g.d, dtype=np.float64)
            keep += [rp, cl, wv, dv]
            r.row_ptr, r.col, r.w, r.d = (a.ctypes.data for a in (rp, cl, wv, dv))
        r.nrhs = f.shape[0]
        r.f = f.ctypes.data
        keep.append(f)
        if want_u:
            u = np.zeros_like(f)
            keep.append(u)
            r.u = u.ctypes.data
            sols.append(u)
        else:
            sols.append(None)
    total = sum(reqs[i].nrhs for i in range(len(requests)))
    out = (amg_completion * total)()
    stats = amg_serve_stats()
    code = load_library().amg_serve(ctypes.byref(cfg), reqs, len(requests), out, ctypes.byref(stats),
                                    _stream(stream))
    _check(code, "amg_serve")
    return [_completion_dict(c) for c in out], _stats_dict(stats), sols


def amg_time_step(h: Hierarchy, reps: int = 200, stream=None) -> dict:
    """Mean duration of the finest level's storing Chebyshev step over ``reps``
    back-to-back launches between HIP events on ``stream``."""
    t = amg_kernel_timing()
    _check(load_library().amg_time_step(h.handle, int(reps), _stream(stream), ctypes.byref(t)), "amg_time_step")
    return {"launches": t.launches, "avg_ms": t.avg_ms, "rows": t.rows, "nnz": t.nnz, "entries": t.entries,
            "grid": t.grid, "value_bytes": t.value_bytes}


def amg_time_step_rotating(h: Hierarchy, reps: int = 200, copies: int = 8, stream=None) -> dict:
    """The same step timed over ``copies`` rotating copies of the finest level
    (each launch streams from HBM, not the Infinity Cache)."""
    t = amg_kernel_timing()
    _check(load_library().amg_time_step_rotating(h.handle, int(reps), int(copies), _stream(stream), ctypes.byref(t)),
           "amg_time_step_rotating")
    return {"launches": t.launches, "avg_ms": t.avg_ms, "rows": t.rows, "nnz": t.nnz, "entries": t.entries,
            "grid": t.grid, "value_bytes": t.value_bytes, "copies": int(copies)}


def amg_level_export(h: Hierarchy, level: int) -> dict:
    """Level ``level`` as host numpy arrays (CSR, d, D and the aggregate map)."""
    desc = amg_describe(h)
    n, nnz = desc["n"][level], desc["nnz"][level]
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(max(nnz, 1), np.int32)
    W = np.zeros(max(nnz, 1), np.float64)
    d = np.zeros(n, np.float64)
    D = np.zeros(n, np.float64)
    coarsest = level == desc["levels"] - 1
    agg = None if coarsest else np.zeros(n, np.int32)
    code = load_library().amg_level_export(
        h.handle, int(level), rp.ctypes.data_as(_P), col.ctypes.data_as(_P), W.ctypes.data_as(_P),
        d.ctypes.data_as(_P), D.ctypes.data_as(_P), None if agg is None else agg.ctypes.data_as(_P))
    _check(code, "amg_level_export")
    return {"n": n, "row_ptr": rp, "col": col[:nnz], "W": W[:nnz], "d": d, "D": D, "agg": agg}


def _sizes(h: Hierarchy):
    return amg_describe(h)["n"]


def amg_apply_smoother(h: Hierarchy, level: int, r, y, stream=None):
    n = _sizes(h)[level]
    _check(load_library().amg_apply_smoother(h.handle, int(level), _dev(r, n, "r"), _dev(y, n, "y"),
                                             _stream(stream)), "amg_apply_smoother")


def amg_apply_residual(h: Hierarchy, level: int, f, x, s, stream=None):
    n = _sizes(h)[level]
    _check(load_library().amg_apply_residual(h.handle, int(level), _dev(f, n, "f"), _dev(x, n, "x"),
                                             _dev(s, n, "s"), _stream(stream)), "amg_apply_residual")


def amg_apply_restrict(h: Hierarchy, level: int, s, b, stream=None):
    ns = _sizes(h)
    _check(load_library().amg_apply_restrict(h.handle, int(level), _dev(s, ns[level], "s"),
                                             _dev(b, ns[level + 1], "b"), _stream(stream)), "amg_apply_restrict")


def amg_apply_prolong(h: Hierarchy, level: int, e, x, stream=None):
    ns = _sizes(h)
    _check(load_library().amg_apply_prolong(h.handle, int(level), _dev(e, ns[level + 1], "e"),
                                            _dev(x, ns[level], "x"), _stream(stream)), "amg_apply_prolong")


def amg_apply_coarse(h: Hierarchy, b, x, stream=None):
    n = _sizes(h)[-1]
    _check(load_library().amg_apply_coarse(h.handle, _dev(b, n, "b"), _dev(x, n, "x"), _stream(stream)),
           "amg_apply_coarse")


def amg_apply_cycle(h: Hierarchy, r, z, stream=None):
    _check(load_library().amg_apply_cycle(h.handle, _dev(r, h.n, "r"), _dev(z, h.n, "z"), _stream(stream)),
           "amg_apply_cycle")
