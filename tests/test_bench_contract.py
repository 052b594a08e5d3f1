"""The benchmark's command-line contract on the CPU: a request for more than
one GPU exits at once with a message (the build runs on one GPU), and the
algorithmic FLOP counts used by the roofline are positive and ordered by the
window sizes of the four form spaces."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_mass_flop_counts():
    sys.path.insert(0, ROOT)
    import bench
    f = {sp: bench.mass_flops(3, 64, sp) for sp in ("B", "D", "E", "H")}
    assert all(v > 0 for v in f.values())
    # the primal spaces have the wider windows (degree p along or across)
    assert f["E"] > f["H"] and f["B"] > f["D"]
    # cost per tile times the tile count: 64^3 holds 8x the tiles of 32^3
    assert abs(bench.mass_flops(3, 64, "B") / bench.mass_flops(3, 32, "B") - 8.0) < 1e-12
