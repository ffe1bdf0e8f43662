"""bench.py's command line and bookkeeping, without a GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_workloads_listed():
    r = run("--help")
    assert r.returncode == 0
    for w in ("lowrank16384", "lowrank4096", "uniform256", "geom4096", "geom16384", "batched512", "serving"):
        assert w in r.stdout
    for flag in ("--no-parallel", "--no-lazy", "--no-rect", "--no-batched", "--no-serving",
                 "--serve-summary-seconds", "--sustained-rate", "--copy-calibration"):
        assert flag in r.stdout


@pytest.mark.parametrize("n", [1, 256, 16384])
def test_algorithmic_bytes_per_unit(n):
    nn = n * n
    assert bench.algorithmic_bytes("range", n, 0, 0) == 4 * nn
    assert bench.algorithmic_bytes("scan", n, 0, 0) == 4 * nn
    assert bench.algorithmic_bytes("layout", n, 0, 0) == 16 * nn  # transpose and W: each read + write
    # per switch 16n B; the loop's own re-evaluations (8n B each) are reported apart
    assert bench.algorithmic_bytes("switch", n, 3, 5) == 16 * n * 3
    assert bench.reevaluation_bytes(n, 5) == 8 * n * 5
    with pytest.raises(KeyError):
        bench.algorithmic_bytes("nope", n, 0, 0)


def test_sizes_of_the_named_workloads():
    assert bench.spec_n("lowrank16384") == 16384 and bench.spec_n("geom16384") == 16384
    assert bench.spec_n("uniform256") == 256
