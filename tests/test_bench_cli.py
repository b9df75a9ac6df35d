"""bench.py's command line on a host without a GPU: it parses, refuses more
than one GPU with a message, and exposes the slab set-up helper."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_help_parses():
    r = _run("--help")
    assert r.returncode == 0 and "--sort-every" in r.stdout


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_helpers_import():
    sys.path.insert(0, ROOT)
    import bench
    assert callable(bench.ionised_slab_simulation)
    b, per_ion, per_cell = bench.algorithmic_bytes(1, 0, True, 4, True)
    assert per_ion == 108 and b == 108
    _, per_el, _ = bench.algorithmic_bytes(1, 0, False, 4, False)
    assert per_el == 56
