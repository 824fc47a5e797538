"""Host-side checks of bench.py's command-line contract (no GPU): a run on
more than one GPU is refused before anything touches a device, with exit
code 2, a message on stderr and no JSON line on stdout."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        r = _bench("--gpus", n)
        assert r.returncode == 2, (r.returncode, r.stderr)
        assert r.stdout == ""
        assert "one GPU only" in r.stderr and f"--gpus {n}" in r.stderr


def test_help_lists_the_driver_options():
    r = _bench("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup"):
        assert opt in r.stdout
