"""Host-side parts of the benchmark: it refuses more than one GPU before
touching any device, and its per-window read-stream model gives the byte
counts of 3 bits per base spread over a 150 bp read's windows."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("argv", [["--gpus", "2"], ["--gpus", "8", "--steps", "1"]])
def test_more_than_one_gpu_is_refused(argv):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv,
                       capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, WORLD_SIZE="1"))
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")],
                       capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, WORLD_SIZE="2"))
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_stream_bytes_per_window():
    import bench
    # 3/8 B per base times 150 / (151 - k), to three decimals
    want = {21: 0.433, 33: 0.477, 55: 0.586, 77: 0.760, 99: 1.082}
    for k, v in want.items():
        assert round(bench.stream_bytes_per_window(150, k), 3) == v
    # one window per read (k = L): the whole read's 3 bits per base
    assert bench.stream_bytes_per_window(150, 150) == pytest.approx(150 * 3 / 8)
