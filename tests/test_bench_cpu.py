"""Host checks of bench.py's contract that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    # one GPU only: any other count exits with a message, before touching a device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_counter_figures_are_well_formed():
    # the HBM counter figures: one fetch and one write value per search launch
    sys.path.insert(0, ROOT)
    import bench
    c = bench.SEARCH_COUNTERS
    assert len(c["fetch_kib"]) == len(c["write_kib"]) > 0
    assert all(v > 0 for v in c["fetch_kib"]) and all(v >= 0 for v in c["write_kib"])
    assert len(c["sources_sha256"]) == 64
