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
