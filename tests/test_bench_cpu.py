"""bench.py's contract on the host: it refuses more than one GPU with a
message and status 2 before touching a device, its algorithmic byte counts
follow the definitions stated in their docstrings (targets written once,
triangles read once per pass; per-pixel gather traffic), and a traced BF16
stage maps to the profiled kernel of the launch variant it ran in."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    b = _bench()
    fl, by = b.raster_costs(19632, 1080, 1920, 2048)["raster light+camera"]
    assert fl == 0.0 and by == 2048 * 2048 * 4 + 1080 * 1920 * 8 + 2 * 19632 * 36
    fl, by = b.gather_costs(19632, 1080, 1920, 6, "gather hard6")["gather hard6"]
    assert by == 1080 * 1920 * (8 + 4 + 24 + 1) + 19632 * 48


def test_stage_symbols_follow_the_launch_variant():
    b = _bench()
    d1 = "conv3x3 32+64->32 Store phase bf16"
    e0 = "conv3x3 6+0->16 Pool bf16"
    assert b.kernel_symbol(d1, [0, 0, 0, 0, 0]) == "k_conv3x3_up<bf16, 32, 64, 32, Store, 8, 4>"
    assert b.kernel_symbol(d1, [0, 0, 0, 1, 0]) == "k_conv3x3_up_persist<bf16, 32, 64, 32, Store, 8, 4>"
    assert b.kernel_symbol(e0, [2, 0, 0, 0, 0]) == "k_conv3x3<bf16, true, 6, 0, 16, Pool, 16>"
    assert b.kernel_symbol(e0, [3, 0, 0, 0, 0]) == "k_conv3x3_persist<bf16, true, 6, 0, 16, Pool, 16>"
    d0 = "conv3x3 16+32->16 Head phase bf16"
    assert b.kernel_symbol(d0, [0, 0, 0, 0, 2]) == "k_conv3x3_up<bf16, 16, 32, 16, Head, 16, 8>"
    assert b.kernel_symbol("raster light+camera", None) == "k_raster"
