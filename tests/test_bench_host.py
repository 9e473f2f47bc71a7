"""Host-side parts of bench.py: the one-GPU guard and the CPU-baseline legs
(the oracle timed on a bounded sample, with all its threads and with one)."""
import os
import subprocess
import sys

import bench
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_fields():
    cb = bench.cpu_baseline("d2q9_e8_256", target_s=0.2)
    assert set(cb) == {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["unit"] == "MLUPS" and cb["value"] > 0
    assert cb["cores"] == O.num_threads()
    assert "d2q9_e8_256" in cb["sample"]


def test_cpu_one_core_leg():
    cb = bench.cpu_one_core("d2q9_e8_256", target_s=0.2)
    assert cb["cores"] == 1 and cb["value"] > 0


def test_workloads_name_their_sizes():
    for name, w in bench.WORKLOADS.items():
        assert "x".join(str(s) for s in w["shape"][:2]) in w["desc"] or str(w["shape"][0]) in w["desc"], name
        assert w["lattice"] in name.upper() or w["lattice"].lower() in name, name
