"""Host-side contract of bench.py: one GPU only (a request for more exits with
status 2 and says so), a machine without a GPU is refused before any child
process starts, and the primer's trace time is read from the line a frame
run prints."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    p = _run("--gpus", "2")
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_no_gpu_is_refused_before_the_primer():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    p = _run()
    assert p.returncode == 2
    assert "needs a GPU" in p.stderr and "primer" not in p.stderr and p.stdout == ""


def test_primer_trace_time_is_parsed_from_the_frame_log():
    import re
    line = ("[bench] 2 steps: 3.694 ms/step (wall 3.697); trace 0.355, noreuse 0.010, reuse_biased 0.262, "
            "validate 2.759, reuse_unbiased 0.303")
    # the pattern run_primer applies to the child's log
    src = open(os.path.join(ROOT, "bench.py")).read()
    pat = re.search(r're\.findall\(r"(.+?)", p\.stderr\)', src).group(1)
    assert [float(x) for x in re.findall(pat, "noise\n" + line + "\n")] == [0.355]
