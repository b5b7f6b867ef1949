"""Host-side pieces of bench.py (no GPU): the one-GPU contract, the byte model
of the dominant step, the stored counter figures and the workload table."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
    assert r.stdout == ""


def test_cheb_step_bytes():
    # FP64: column index + weight per stored entry, D, w_k, w_k-1, y read, y and w_k+1 written
    assert bench.cheb_step_bytes(1_048_576, 6_283_266, False) == 12 * 6_283_266 + 48 * 1_048_576
    assert bench.cheb_step_bytes(10, 100, True) == 8 * 100 + 24 * 10


def test_stored_traffic_matches_the_source_hash():
    path = os.path.join(ROOT, "profiles", "traffic_cheb_step_grid2d-1024.md")
    txt = open(path).read()
    stored_hash = txt.split("kernel_source_hash:")[1].split()[0]
    t = bench.stored_traffic("grid2d-1024")
    if stored_hash == bench.kernel_source_hash():
        assert t is not None and 0.9 < t / bench.cheb_step_bytes(1_048_576, 6_283_266, False) < 1.2
    else:
        assert t is None  # counters taken on other code are not reported
    assert bench.stored_traffic("no-such-workload") is None


@pytest.mark.parametrize("name", sorted(bench.WORKLOADS))
def test_workload_parameters_are_valid(name):
    import paper_1307_6305_amd as amg

    _, kind, cfg, kw = bench.WORKLOADS[name]
    assert kind in ("uniform", "normal")
    p = amg.amg_params_default(**kw)
    assert p.degree == kw.get("degree", 4)


def test_table1_families():
    g = bench.table1_graph("2d", 8)
    assert g.n == 64 and not g.d.any()
    g = bench.table1_graph("3d", 4)
    assert g.n == 64 and not g.d.any()
    with pytest.raises(ValueError):
        bench.table1_graph("4d", 3)
    assert set(bench.PAPER_TABLE1) >= {("2d", 1024), ("3d", 128), ("unstruct", 64)}
