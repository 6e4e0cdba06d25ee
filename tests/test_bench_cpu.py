"""bench.py on the host: the one-GPU contract, the profiling-leg option and
the algorithmic work model behind the roofline figures (no GPU needed)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_unknown_profile_leg_is_rejected():
    r = _bench("--profile-leg", "nonsense")
    assert r.returncode == 2
    assert "invalid choice" in r.stderr


def test_level0_lk_algorithmic_bytes():
    """640x480 level 0 (18,921 patches, FP64 records) densifying level 1
    (4,661 patches over a 160x120 fallback field): the uint8 images, the
    records, the level-1 records and the level-2 field read; the level-1
    field is not written."""
    expect = 2 * 640 * 480 + 18921 * (3 * 8 + 1) + 4661 * 2 * 8 + 160 * 120 * 8
    assert bench.lk_bytes(640, 480, 18921, 8, True, 320 * 240, (4661, 160 * 120)) == expect == 1315601


def test_lk_bytes_unfolded_reads_the_coarse_field():
    # level 1 of a pair, not folded: FP64 images, records, the level-2 field read
    assert bench.lk_bytes(320, 240, 4661, 8, False, 160 * 120) == \
        2 * 320 * 240 * 8 + 4661 * 25 + 160 * 120 * 8


def test_net_flops_per_layer():
    """Four 3x3 layers 16 -> 32 -> 32 -> 32 -> 2 over 64 x 40 x 30 pixels: the
    hidden layers' sums equal the MFMA op counts rocprofv3 reports for them."""
    px = 64 * 40 * 30
    layers = [2 * 9 * ci * co * px for ci, co in ((16, 32), (32, 32), (32, 32), (32, 2))]
    assert layers[:3] == [707788800, 1415577600, 1415577600]
    assert bench.net_flops(32, px) == sum(layers) == 3627417600


def test_lds_peak_from_unit_counts():
    assert bench.PEAK_LDS == 128 * 256 * 2.4e9


def test_cpu_leg_threads_follow_affinity_and_budget(monkeypatch):
    """The CPU leg uses every core the process may run on, capped by the
    job's thread budget when OMP_NUM_THREADS is set."""
    usable = len(os.sched_getaffinity(0))
    monkeypatch.delenv("OMP_NUM_THREADS", raising=False)
    assert bench.host_threads() == usable
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    assert bench.host_threads() == 1
    monkeypatch.setenv("OMP_NUM_THREADS", str(usable + 100))
    assert bench.host_threads() == usable
    assert bench._cpu_model()
