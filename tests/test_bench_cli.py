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


def test_path_deviation_by_hand():
    """The segmental accuracy report: a path's B position per row of A (mean
    over the row's cells, interpolated over skipped rows) and its deviation
    from a reference path, on small paths worked out by hand."""
    sys.path.insert(0, ROOT)
    import bench
    import numpy as np
    # rows 0..4; row 1 is skipped by a (2,1) step, row 3 holds two cells
    p = np.array([[0, 0], [2, 1], [3, 2], [3, 3], [4, 4]])
    np.testing.assert_allclose(bench.path_rows_position(p, 5), [0.0, 0.5, 1.0, 2.5, 4.0])
    # rows before the first and after the last visited row hold their neighbour
    q = np.array([[1, 3], [2, 5]])
    np.testing.assert_allclose(bench.path_rows_position(q, 4), [3.0, 3.0, 5.0, 5.0])
    ref = np.array([[0, 0], [1, 1], [2, 2], [3, 3], [4, 4]])
    d = bench.path_deviation(p, ref, 5)
    # |0-0|, |0.5-1|, |1-2|, |2.5-3|, |4-4|
    assert d["mean_dev_frames"] == round((0 + 0.5 + 1 + 0.5 + 0) / 5, 4)
    assert d["max_dev_frames"] == 1.0
    assert d["rows_within_1_frame"] == 1.0
    assert bench.path_deviation(ref, ref, 5)["mean_dev_frames"] == 0.0
