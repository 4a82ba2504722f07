"""bench.py command-line contract on the CPU: more than one GPU is refused
with a message (the library has no multi-GPU path)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "8", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_missing_library_fails_loudly():
    """Without libcavity.so the binding raises ImportError on first use:
    there is no CPU fallback for any step of the path."""
    code = ("import paper_2006_02602_amd as C\n"
            "try:\n"
            "    C.cavity_state_elems(C.Grid.cube(16))\n"
            "except ImportError as e:\n"
            "    print('ImportError', e)\n")
    env = dict(os.environ, CAVITY_LIB=os.path.join(ROOT, "no_such_dir", "libcavity.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, env=env,
                       cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ImportError") and "libcavity.so" in r.stdout
