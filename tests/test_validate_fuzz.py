"""Host-side validation of the problem data (eq. (prob)) under the address and
undefined-behaviour sanitizers: random connected graphs, valid or with one
defect each, must get the status the C ABI documents for that defect, and no
read may leave the caller's arrays (tests/validate_fuzz.cpp).  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_validate_graph_fuzz_under_sanitizers(tmp_path):
    exe = str(tmp_path / "validate_fuzz")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "validate_fuzz.cpp"),
                    os.path.join(ROOT, "paper_1307_6305_amd", "csrc", "validate.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "14000"], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    counts = dict(line.split() for line in r.stdout.splitlines())
    assert len(counts) == 14 and all(int(v) == 1000 for v in counts.values()), counts
