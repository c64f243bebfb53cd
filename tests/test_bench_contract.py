"""The benchmark's command-line contract, on the CPU: more than one GPU is
refused with a message, and the source digest that keys the stored counter
traffic covers the kernel sources and nothing else."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_traffic_digest_is_stable_and_hex():
    m = load_bench()
    d1, d2 = m.src_digest(), m.src_digest()
    assert d1 == d2 and len(d1) == 16 and int(d1, 16) >= 0
