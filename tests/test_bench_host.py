"""Host logic of bench.py that runs without a GPU: the record's peak fractions are checked, and
the command line refuses more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_fractions_above_one_are_refused():
    import bench
    bench.check_fractions({"roofline": {"frac": 0.11}, "extras": {"x": [{"frac_peak": 1.0, "ms": 5.0}]}})
    with pytest.raises(ValueError, match="frac_peak_executed"):
        bench.check_fractions({"extras": {"elasticity": {"results": [{"frac_peak_executed": 1.2}]}}})
    with pytest.raises(ValueError):
        bench.check_fractions({"frac_hbm": -0.1})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
