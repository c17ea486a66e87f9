"""Host-side behaviour of the benchmark script (no GPU): the one-GPU
contract and the name of the exchange kernel a workload runs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


@pytest.mark.parametrize("n,name", [
    (1000, "k_2opt_pair<16>"),                # 16-bit rows, two wavefronts (n > 128 among <= 1024 particles)
    (1024, "k_2opt_pair<16>"),
    (1021, "k_2opt_pair<16>"),                # padded 16-bit rows
    (516, "k_2opt_pair<16>"),
    (512, "k_2opt_pair<8>"),
    (260, "k_2opt_pair<8>"),
    (256, "k_2opt_wave<4, true, false>"),     # int32 rows straight into LDS (n <= 256, n % 4 == 0)
    (255, "k_2opt_pair<4>"),                  # rows of D off 16 bytes: 16-bit copy
    (100, "k_2opt_wave<2, true, false>"),
    (101, "k_2opt_wave<2, true, true>"),      # n <= 128: one wavefront
    (64, "k_2opt_wave<1, true, false>"),
    (9, "k_2opt_wave<1, true, true>"),
    (5, "k_2opt_wave<1, false, false>"),      # below 8: int32 rows through registers
    (1025, "k_2opt_rows"),
])
def test_exchange_kernel_name_follows_the_default_rows(n, name):
    """The kernel bench.py names for the library's default row form of n
    (the tuning table is read on the host; no GPU)."""
    from paper_1706_04399_amd import dpso
    dpso.tuning_reset()
    rows = dpso.tuning_get(n, 1024)["exchange_rows"]
    assert bench.exchange_kernel_name(n, rows) == name


@pytest.mark.parametrize("n,name", [
    (1000, "k_2opt_wave<16, true, true>"),    # the headline: 16-bit rows, one wavefront
    (516, "k_2opt_wave<16, true, true>"),
    (260, "k_2opt_wave<8, true, true>"),
    (256, "k_2opt_wave<4, true, true>"),      # above 1024 particles every n >= 8 takes 16-bit rows
])
def test_exchange_kernel_name_among_many_particles(n, name):
    from paper_1706_04399_amd import dpso
    dpso.tuning_reset()
    rows = dpso.tuning_get(n, 4096)["exchange_rows"]
    assert bench.exchange_kernel_name(n, rows) == name
