"""Host-side checks of bench.py (no GPU): it refuses more than one GPU
before touching the device, and its full-field byte model gives the figure
derived by hand for the 256x256x128 workload."""
import importlib.util
import os
import subprocess
import sys

from paper_1707_09898_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_full_field_byte_model_at_256x256x128():
    """Two scalar convolutions over the 512x512x256 box in FP32: per field
    n + 4 hx ny nz + 4 hx Ly nz words read and written across the five
    passes, the 257 x 257 x 129 tensor octant once per convolution, rho once:
    1.853 GB, the figure the design notes quote."""
    b = load_bench()
    w = wl.config3()
    nx, ny, nz = w.n
    hx = 257
    per_field = nx * ny * nz + 4 * hx * ny * nz + 4 * hx * 512 * nz
    K = hx * 257 * 129
    expect = 4 * (4 * per_field + 2 * K + nx * ny * nz)
    got = b.model_bytes_per_eval(w, 4, (512, 512, 256))
    assert got == expect
    assert abs(got / 1e9 - 1.853) < 0.001
