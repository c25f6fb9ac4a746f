"""The host layout code under UndefinedBehaviorSanitizer (host code only; the
device code is built as usual, and nothing here touches a GPU).

daba_workspace_bytes and daba_part_workspace_bytes build a problem's whole
layout on the host: partitions, the packed observation words (index in the
low bits, partition in the top six), slots, tiles, landmark blocks and the
workspace carve.  The library is rebuilt with -fsanitize=undefined on the
host side and called from a child process on problems with 64 partitions,
so that a partition index of 32 or more reaches the top bits; any undefined
behaviour aborts the child.  (Planting a shift of the partition index by one
bit too many in the packing makes it abort with "shift-out-of-bounds".)"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes as C, sys
import numpy as np
sys.path.insert(0, sys.argv[2])
from synth import make_problem
from paper_2305_07026_amd.binding import DabaProblem, DabaOptions
lib = C.CDLL(sys.argv[1])
for f in (lib.daba_workspace_bytes, lib.daba_part_workspace_bytes):
    f.argtypes = [C.POINTER(DabaProblem), C.POINTER(DabaOptions)]
    f.restype = C.c_size_t
def ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))
rng = np.random.default_rng(7)
for track in ("fixed8", "geom6"):
    prob = make_problem("cam50-lm5k", n_cameras=256, n_landmarks=3000, track=track, seed=11)
    M, N, K = prob["n_cameras"], prob["n_landmarks"], prob["n_obs"]
    cam = np.ascontiguousarray(prob["obs_camera"], np.int32)
    lm = np.ascontiguousarray(prob["obs_landmark"], np.int32)
    uv = np.ascontiguousarray(prob["obs_uv"], np.float64)
    cams = np.ascontiguousarray(prob["cameras"], np.float64)
    lms = np.ascontiguousarray(prob["landmarks"], np.float64)
    cp = np.ascontiguousarray(np.arange(M) % 64, np.int32)
    lp = np.ascontiguousarray(rng.integers(0, 64, N), np.int32)
    for maps in ((None, None), (cp, lp)):
        p = DabaProblem(M, N, K, ptr(cam, C.c_int32), ptr(lm, C.c_int32), ptr(uv, C.c_double),
                        ptr(cams, C.c_double), ptr(lms, C.c_double), 64,
                        None if maps[0] is None else ptr(maps[0], C.c_int32),
                        None if maps[1] is None else ptr(maps[1], C.c_int32), 512.0)
        for prec in (0, 1):  # FP64 and FP32-mixed (the device-level surrogate is FP64 only)
            o = DabaOptions(1, 1.0, 1e-9, 0.5, 1, 1, prec, 0)
            assert lib.daba_workspace_bytes(C.byref(p), C.byref(o)) > 0, (track, prec)
        o = DabaOptions(1, 1.0, 1e-9, 0.5, 1, 1, 0, 0)
        assert lib.daba_part_workspace_bytes(C.byref(p), C.byref(o)) > 0, track
print("layout ok")
"""


def _runtime_dir(hipcc):
    """Where the compiler's sanitizer runtimes are (hipcc's clang)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/lib/llvm/bin/clang"
    so = subprocess.run([clang, "-print-file-name=libclang_rt.ubsan_minimal-x86_64.so"], capture_output=True,
                        text=True, check=True).stdout.strip()
    if not os.path.isabs(so) or not os.path.exists(so):
        pytest.skip("no UBSan minimal runtime next to hipcc's clang")
    return os.path.dirname(so)


@pytest.mark.timeout(600)
def test_layout_has_no_undefined_behaviour(tmp_path):
    B = pytest.importorskip("paper_2305_07026_amd.build")
    if not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc")
    pytest.importorskip("paper_2305_07026_amd.binding")  # the structures; needs the regular build
    rt = _runtime_dir(B.HIPCC)
    lib = str(tmp_path / "libdaba_ubsan.so")
    cmd = [B.HIPCC, *B.FLAGS,
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fsanitize-minimal-runtime",
           "-Xarch_host", "-fno-sanitize-recover=all", "-shared-libsan", f"-Wl,-rpath,{rt}",
           *B.SOURCES, "-o", lib]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               LD_LIBRARY_PATH=os.pathsep.join(x for x in (rt, os.environ.get("LD_LIBRARY_PATH")) if x))
    r = subprocess.run([sys.executable, "-c", CHILD, lib, ROOT], capture_output=True, text=True, timeout=300,
                       env=env, cwd=ROOT)
    assert r.returncode == 0 and "layout ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
