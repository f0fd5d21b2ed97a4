"""Host-side checks of the benchmark script (no GPU): the one-GPU guard, the
roofline helpers and the two-group sweep's grid."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2503_00264_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_padded_cell_sizes():
    assert [bench.padded(n) for n in (1, 8, 9, 24, 64, 120, 192, 256, 512)] == \
        [8, 8, 16, 32, 64, 128, 256, 256, 512]


def test_setup_model_counts_two_np_cubed_per_cell():
    p = W.multigroup(seed=3, J=16, N=16, G=4, n_regions=4, length=1.0, dt=1e-3)
    m = bench.setup_model([p], [0.5], True)
    assert m["flop"] == 2.0 * 256 ** 3 * 16
    assert m["bound"] == "mfma" and m["kernels"] == ["k_gj_invert<float,32,256>"]
    assert abs(m["achieved"] - m["flop"] / 0.5 / 1e12) < 1e-3
    small = bench.setup_model([W.homogeneous(J=8, N=8)], [1.0], False)
    assert small["bound"] == "alu" and small["kernels"] == ["k_assemble_factor<double>"]


def test_recorded_traffic_needs_the_matching_kernel_and_summary():
    assert bench.recorded_traffic("k_not_a_kernel<float,64,1024>") is None
    assert bench.recorded_traffic("k_oci_res<float,64,1024>", "no_such_summary.md") is None


@pytest.mark.parametrize("delta", bench.ROSA_DELTAS)
def test_rosa_sweep_grid_hits_each_delta(delta):
    J = max(1, int(round(W.ROSA_SIGMA_MIN * W.ROSA_LENGTH / delta)))
    got = W.ROSA_SIGMA_MIN * W.ROSA_LENGTH / J
    assert abs(got - delta) <= 0.1 * delta
    p = W.rosa(J=J, N=8)
    assert abs(p["sigma_t"][0, 1] * p["dx"][0] - got) < 1e-12
