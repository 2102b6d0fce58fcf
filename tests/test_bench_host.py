"""Host-side behaviour of bench.py that needs no GPU: the one-GPU refusal of
--gpus N > 1 and the lookup of measured HBM traffic, which must come back
empty for a configuration the committed counters were not taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr


def test_traffic_lookup_only_for_the_measured_configuration():
    for kernel in ("p2p", "m2l"):
        assert bench.measured_traffic(kernel, "gauss131k", "fp64", "fp64",
                                      "mean") is None
        assert bench.measured_traffic(kernel, "gauss131k", "fp32", "fp32",
                                      "source") is None
        assert bench.measured_traffic(kernel, "no-such-workload", "fp32",
                                      "fp32", "mean") is None
