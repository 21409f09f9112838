"""Host-side logic of bench.py, on the CPU: the algorithmic byte model and
the lattice's spring count it is quoted on, the measured-traffic lookup in
the committed counter summary (used only while its kernel-source
fingerprint matches), and the refusal of more than one GPU."""
import os
import subprocess
import sys

import bench
from paper_1911_10274_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lattice_springs(n):
    """Springs of the n^3 lattice whose masses are joined to every neighbour
    within sqrt(3) spacings: axis edges, face diagonals (two per unit square)
    and body diagonals (four per unit cube)."""
    return 3 * n * n * (n - 1) + 6 * n * (n - 1) ** 2 + 4 * (n - 1) ** 3


def test_lattice_spring_count_closed_form():
    for n in (2, 3, 5, 7):
        assert scenes.lattice(n)["ends"].shape[0] == _lattice_springs(n)
    assert _lattice_springs(100) == 12_731_796


def test_algorithmic_bytes_of_the_benchmark_lattice():
    # 24 B per spring, 84 B per mass
    assert bench.algorithmic_bytes(1_000_000, _lattice_springs(100)) == 389_563_104
    assert bench.algorithmic_bytes(0, 0) == 0


def test_measured_traffic_follows_the_kernel_fingerprint(monkeypatch):
    t = bench.measured_traffic()
    assert t is not None and t > bench.algorithmic_bytes(1_000_000, _lattice_springs(100))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""
