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


def test_algorithmic_bytes_per_atom():
    """Positions (d doubles) and the type (one byte) in, velocities in for
    F.v and forces out (d doubles each): 24 d + 1 bytes."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.FORCE_BYTES_PER_ATOM == {d: 3 * 8 * d + 1 for d in (2, 3)}
