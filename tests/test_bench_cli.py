"""Host-side checks of bench.py's contract that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_fused_step():
    """32 B per grid point for the fused extension + FFT when every point is IN
    or STRIP (the figure the roofline divides by)."""
    sys.path.insert(0, ROOT)
    import bench

    class Info:
        n_in = 0
        n_strip = 0
        n_far = 0
        B = 0
        d = 5

    n, nf = 64, 3
    info = Info()
    info.n_in = n * n
    half = n * (n // 2 + 1)
    rows = bench.algorithmic_bytes("k_rows_r2c_ext", n, nf, info)
    cols = bench.algorithmic_bytes("k_cols", n, nf, info)
    assert rows == nf * (8 * n * n + 16 * half)
    assert cols == nf * 32 * half
    assert abs((rows + cols) / (nf * n * n) - 32.0) < 32.0 * 3 / n   # the Nyquist column adds 1/(n/2)
