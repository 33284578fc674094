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


def test_committed_traffic_counters_match_the_kernel_sources():
    """The force kernel's copy-calibrated counter summary under profiles/ was
    taken with the kernel sources as they are (same hash), so the benchmark
    line carries its traffic; and that traffic is (read + written bytes per
    atom) x atoms per launch."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "k_force_3d_hbm_traffic.txt")) as fh:
        t = [json.loads(line.split(":", 1)[1]) for line in fh if line.startswith("traffic_json:")]
    assert len(t) == 1 and t[0]["sources_sha256"] == bench.kernel_sources_sha256()
    per_atom = t[0]["fetch_bytes_per_atom"] + t[0]["write_bytes_per_atom"]
    assert per_atom > bench.FORCE_BYTES_PER_ATOM[3]
    assert bench.force_traffic(3, 1000.0) == per_atom * 1000.0
    assert bench.force_traffic(2, 1000.0) is None or bench.force_traffic(2, 1000.0) > 0
