"""bench.py's command line on the CPU: a run on more than one GPU is refused
with a message before anything touches a device (the path is one GPU's)."""
import os
import subprocess
import sys

BENCH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py")


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        res = subprocess.run([sys.executable, BENCH, "--gpus", n], capture_output=True,
                             text=True, timeout=300)
        assert res.returncode == 2, (res.returncode, res.stderr)
        assert "exactly one GPU" in res.stderr
        assert res.stdout == ""
