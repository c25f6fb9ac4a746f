"""Host-side checks of the product's contracts (no GPU): the package has no
fallback when the gfx950 library is missing, and the benchmark refuses a
multi-GPU run, which this implementation does not provide."""

import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2305_07026_amd")


def test_package_import_fails_without_the_library(tmp_path):
    # a copy of the Python package with no libdaba.so next to it
    dst = tmp_path / "paper_2305_07026_amd"
    dst.mkdir()
    for name in os.listdir(PKG):
        if name.endswith(".py"):
            shutil.copy(os.path.join(PKG, name), dst / name)
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "try:\n"
            "    import paper_2305_07026_amd\n"
            "except ImportError as e:\n"
            "    print('ImportError:', e); sys.exit(3)\n"
            "sys.exit(0)\n")
    r = subprocess.run([sys.executable, "-c", code, str(tmp_path)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 3, (r.returncode, r.stdout, r.stderr)
    assert "libdaba.so is not built" in r.stdout


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
