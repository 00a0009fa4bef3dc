"""Host-side checks of bench.py: the one-GPU contract and the provenance of
the roofline's measured traffic (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    """--gpus above 1 exits with status 2 and says why, before touching a GPU."""
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=60)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_traffic_summary_was_taken_on_the_current_filter_kernel():
    """The roofline's HBM traffic comes from the committed counter summary
    only when that summary names the current zfilter.hip by hash: it must, so
    that the figure bench.py reports belongs to the kernel it times."""
    sys.path.insert(0, ROOT)
    import bench
    traffic = bench.traffic_for_current_kernel()
    assert traffic is not None, "profiles/zfilter_step_traffic.txt is stale: retake FETCH_SIZE / WRITE_SIZE"
    # between the algorithmic bytes of a launch (H once, about 7 GB at N =
    # 20000) and a re-read of X per 128-row panel of H (tens of GB)
    assert 5e9 < traffic < 1e11
