"""Host logic of bench.py: each workload's defaults (size, harmonics, tolerance,
smoother ratio, wave size) and the message for more than one GPU (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("workload,tets,harm,rtol,ratio,post0,batch", [
    ("tree", 12_000_000, 64, 2e-12, 10.0, 1, 2),
    ("pipe", 200_000, 16, 4e-12, 10.0, 0, 0),
    ("ybatch", 200_000, 16, 2e-12, 4.0, 0, 0),
    ("ylearn", 1_200_000, 32, 2e-12, 4.0, 0, 16),
])
def test_workload_defaults(workload, tets, harm, rtol, ratio, post0, batch):
    a = bench.parse(["--workload", workload])
    assert (a.tets, a.harmonics, a.rtol, a.mg_ratio, a.mg_post0, a.batch) == (tets, harm, rtol, ratio, post0, batch)
    assert a.gpus == 1 and a.restart == 40 and a.precision == "mixed"


def test_explicit_options_win():
    a = bench.parse(["--workload", "tree", "--rtol", "1e-11", "--mg-ratio", "6", "--mg-post0", "0", "--batch", "3"])
    assert (a.rtol, a.mg_ratio, a.mg_post0, a.batch) == (1e-11, 6.0, 0, 3)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
