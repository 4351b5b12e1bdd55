"""The bench measures one GPU: asked for more (a --gpus value above 1, or a
launcher's WORLD_SIZE above 1) it exits with status 2 and says so, before it
touches a device. Runs on the CPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [
    (["--gpus", "2"], {}),
    (["--gpus", "8", "--steps", "3", "--warmup", "1"], {}),
    (["--workload", "batch256_500to8000_d12", "--gpus", "4"], {}),
    (["--workload", "segmental_100000x100000_d12", "--gpus", "2"], {}),
    ([], {"WORLD_SIZE": "2"}),
])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT, env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, r.stderr
    assert "more than one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (3, 2), (7, 7), (9, 5), (100, 199), (100, 200), (333, 400),
                                 (700, 520), (1000, 1999), (1234, 987)])
def test_band_cell_counts(n, m):
    """The roofline's algorithmic cells: the closed forms used by the bench
    against cell-by-cell enumeration of the band masks."""
    sys.path.insert(0, ROOT)
    import bench
    from tests import parity
    assert bench.band_cells(n, m) == int(parity.band_mask(n, m).sum())
    assert bench.subseq_band_cells(n, m) == int(parity.subseq_band_mask(n, m).sum())


def test_band_cells_of_the_long_pair():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.band_cells(50000, 60000) == 933333334
