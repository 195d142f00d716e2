"""Host-side contract checks that need no GPU: the benchmark measures one GPU
only, and the binding refuses to run without the built HIP library (there is
no fallback path)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("args,env", [
    (["--gpus", "2"], {}),
    (["--gpus", "8"], {}),
    (["--gpus", "1"], {"WORLD_SIZE": "2"}),
], ids=["gpus2", "gpus8", "world_size2"])
def test_bench_refuses_more_than_one_gpu(args, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                       capture_output=True, text=True, timeout=120, cwd=ROOT, env=e)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_binding_fails_loudly_without_the_library():
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2405_07898_amd import md\n"
        "md.LIB_PATH = '/nonexistent/libmdeam.so'\n"
        "try:\n"
        "    md.lib()\n"
        "except ImportError as e:\n"
        "    print('refused:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(1)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "is missing" in r.stdout
