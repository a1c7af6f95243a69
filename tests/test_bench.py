"""Host-side checks of bench.py (no GPU): the one-GPU rule, the traffic record, the CPU
baseline on a small sample."""
import subprocess
import sys

import numpy as np

import bench


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=bench.ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_only_for_the_profiled_configuration():
    """The counters were taken on C3 with the library's team policy; any other configuration
    reports no traffic, and the record's hash covers the kernel sources."""
    assert bench.measured_traffic("c2", 0) is None
    assert bench.measured_traffic("c3", 16) is None
    t = bench.measured_traffic("c3", 0)
    h = bench.kernel_source_hash()
    assert len(h) == 64
    if t is not None:                      # valid only while the sources hash as recorded
        assert t > 0


def test_cpu_baseline_on_one_small_instance():
    wl = bench.make_workload("c1")
    rec, ref = bench.cpu_baseline(wl, n_sample=1)
    assert rec["kind"] == "oracle" and rec["unit"] == "images/s" and rec["cores"] == 1
    assert rec["value"] > 0 and rec["single_core_images_per_s"] > 0
    dirty, beam, R, model, abc = ref
    N = int(wl.n_img[0])
    assert dirty.shape == (N, N) and beam.shape == (2 * N, 2 * N) and R.shape == (N, N)
    assert np.count_nonzero(model) > 0 and len(abc) >= 3
