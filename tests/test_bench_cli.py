"""Host-side checks of bench.py: the one-GPU contract and the workload table."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workloads_tile_their_lattices():
    sys.path.insert(0, ROOT)
    import bench
    from oracle import sap as S
    for name, wl in bench.WORKLOADS.items():
        S.check_blocking(wl["L"], wl["block"])     # even block count per direction
        assert 0 <= wl["k"] < wl["m"] <= 48, name
        m0, src = bench.mass_for(wl["mass"])
        assert m0 == m0 and src, name
