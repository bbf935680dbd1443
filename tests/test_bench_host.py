"""Host-side checks of bench.py (no GPU needed): the contract's refusal of
more than one GPU, and the validity of the committed traffic record."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and "--gpus must be 1" in line["error"]


def test_committed_traffic_matches_the_kernel_sources():
    # the HBM traffic in the bench line comes from rocprofv3 counters taken
    # on the current kernel sources; a source change without new counters
    # makes bench.py report null, which this test turns into a failure
    sys.path.insert(0, ROOT)
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for key in ("fp64:stream2", "fp32:stream2"):
        t = bench.measured_traffic(key)
        assert t is not None and t > 0, key
