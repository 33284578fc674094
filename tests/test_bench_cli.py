"""The benchmark's command line, CPU only: one GPU per run (a request for
several exits with a message and status 2 before touching a device), and
the algorithmic counts it prices the force kernel with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_counts():
    """Positions (d doubles) and the type (one byte) in, forces out (d
    doubles): 16 d + 1 bytes per atom; 33 flops per in-cutoff pair."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.FORCE_BYTES_PER_ATOM == {d: 2 * 8 * d + 1 for d in (2, 3)}
    assert bench.FLOPS_PER_PAIR == 33


def test_unknown_form_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--forms", "nonsense"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""
