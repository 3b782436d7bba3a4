"""Host-side logic of bench.py (no GPU): the algorithmic flop count, the band
width rule, the traffic figure read from the committed counter summary, and the
refusal of multi-GPU runs."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("M", [1, 255, 256, 2047, 2048, 32768])
def test_alg_flops_closed_form(M):
    # (23/3) M^3 + 6 b M^2 + F_D&C: R1 M^3/3, R2-4 M^3, S1 4M^3/3, S4 2M^3, S5 2M^3,
    # R5 M^3, S2 6bM^2, and the divide and conquer's measured merge flops
    for b in (16, 32, 64):
        assert bench.alg_flops(M, b) == pytest.approx(23.0 / 3.0 * M ** 3 + 6.0 * b * M ** 2,
                                                      rel=1e-12)
        assert bench.alg_flops(M, b, 1.5e9) == pytest.approx(bench.alg_flops(M, b) + 1.5e9)


def test_band_width_is_the_library_value():
    from paper_1504_06443_amd import _binding
    L = _binding.lib()
    for M in (100, 300, 1000, 3000, 32768):
        assert bench.band_width(M) == L.gep_tune_get(b"band_width", M)


def test_alg_flops_at_the_benchmark_size():
    # 2.70e14 at M = 32768 (b = 64), before the divide and conquer's merge flops
    assert bench.alg_flops(32768, 64) == pytest.approx(2.7016e14, rel=1e-4)


def test_kernel_traffic_matches_the_committed_summary():
    path = os.path.join(ROOT, "profiles", "dgemm_fast_kernel_m32768_traffic.txt")
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, fields["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    t = bench.kernel_traffic("dgemm_fast_kernel", "m32768")
    if sha != fields["source_sha256"]:
        # the kernel's source changed after the counters were taken: no figure
        assert t is None
    else:
        assert t == pytest.approx(float(fields["fetch_bytes_per_launch"])
                                  + float(fields["write_bytes_per_launch"]), rel=1e-6)
        assert t == float(fields["bytes_per_launch"])
    assert bench.kernel_traffic("no_such_kernel", "m32768") is None


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
