"""Host logic of bench.py (no GPU): a request for more than one GPU exits
with a message instead of measuring, whether it comes from --gpus or from a
distributed launcher's WORLD_SIZE."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _bench(["--gpus", "2"])
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""
    r = _bench(["--gpus", "1"], {"WORLD_SIZE": "4"})
    assert r.returncode == 2 and "one GPU only" in r.stderr
