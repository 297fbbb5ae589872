"""The benchmark's contract on the host (no GPU needed): it measures one GPU and says so,
and the committed rocprofv3 summary it reads for the roofline matches the kernel sources
(a kernel change without new counters would turn the roofline back to its HBM fallback)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_summary_matches_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    prof = bench.kernel_profile()
    assert prof is not None, "profiles/k_render_1080p_summary.txt was taken on other sources"
    for k in ("fp32_flops_per_pixel", "valu_insts_per_wave", "fetch_bytes", "write_bytes",
              "avg_duration_us"):
        assert prof[k] > 0
