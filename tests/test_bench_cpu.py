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


def test_roofline_labels_cache_served_rates():
    # the line's algorithmic rate above the HBM peak, per launch or per step,
    # is labelled cache-served; with counters the achieved rate is theirs
    sys.path.insert(0, ROOT)
    import bench
    peak = bench.PEAK_HBM_GBS
    r = bench.roofline_line(40e9, 4.0, 12, 52.0, None)  # 10 TB/s algorithmic
    assert r["basis"] == "algorithmic" and r["cache_served"]
    assert r["achieved"] == r["algorithmic_gbs"] == 10000.0
    r = bench.roofline_line(40e9, 4.0, 12, 52.0, 21e9)  # counters: 5.25 TB/s
    assert r["basis"] == "hbm_counters" and r["cache_served"]
    assert r["achieved"] == 5250.0 and r["frac"] == round(5250.0 / peak, 4) and r["frac"] <= 1
    # algorithmic below peak per launch but above it over the whole step
    r = bench.roofline_line(20e9, 4.0, 12, 20.0, None)
    assert r["algorithmic_gbs"] == 5000.0 and r["algorithmic_step_gbs"] == 12000.0
    assert r["cache_served"]
    r = bench.roofline_line(20e9, 4.0, 12, 60.0, None)
    assert not r["cache_served"] and r["frac"] == round(5000.0 / peak, 4)
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r


def test_counter_figures_are_well_formed():
    # per form: one fetch and one write value per search launch, and the
    # sources they were taken on
    sys.path.insert(0, ROOT)
    import bench
    for form, c in bench.SEARCH_COUNTERS.items():
        assert form in ("fp32", "bf16")
        assert len(c["fetch_kib"]) == len(c["write_kib"]) > 0
        assert all(v > 0 for v in c["fetch_kib"]) and all(v >= 0 for v in c["write_kib"])
        assert len(c["sources_sha256"]) == 64

