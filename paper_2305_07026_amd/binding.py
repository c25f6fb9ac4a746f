"""ctypes binding of libdaba.so (include/daba.h).

Argument marshalling only: every step of the iteration runs in the library's
gfx950 kernels.  PyTorch supplies the device workspace and the stream.  If
the library has not been built this module raises on import; there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdaba.so")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")
HEADERS = (os.path.join(INCLUDE, "daba.h"), os.path.join(INCLUDE, "daba_part.h"))

DABA_OK = 0
ERRORS = {-1: "DABA_E_INVAL", -2: "DABA_E_NOMEM", -3: "DABA_E_HIP", -4: "DABA_E_NONFINITE", -5: "DABA_E_DEGENERATE"}
LOSS = {"trivial": 0, "huber": 1, "welsch": 2}
PRECISION = {"fp64": 0, "fp32_mixed": 1}
NEVER_RESTART = 1
ALWAYS_RESTART = 2
MAX_PARTITIONS = 64

_P = C.POINTER


class DabaProblem(C.Structure):
    _fields_ = [("n_cameras", C.c_int64), ("n_landmarks", C.c_int64), ("n_obs", C.c_int64),
                ("obs_camera", _P(C.c_int32)), ("obs_landmark", _P(C.c_int32)), ("obs_uv", _P(C.c_double)),
                ("cameras", _P(C.c_double)), ("landmarks", _P(C.c_double)),
                ("n_partitions", C.c_int32), ("camera_partition", _P(C.c_int32)),
                ("landmark_partition", _P(C.c_int32)), ("unit_scale", C.c_double)]


class DabaOptions(C.Structure):
    _fields_ = [("loss", C.c_int32), ("loss_delta", C.c_double), ("xi", C.c_double), ("eta", C.c_double),
                ("accelerate", C.c_int32), ("inner_steps", C.c_int32), ("precision", C.c_int32),
                ("debug_flags", C.c_uint64)]


class DabaError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {detail}")
        self.code = code


def header_symbols() -> list[str]:
    """Names of the functions the headers under include/ declare."""
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"\b(daba_[a-z_]+)\s*\(", text)))


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_2305_07026_amd/build.py")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one; load it first so that libdaba.so binds to the runtime that owns
    # the device memory and streams it is handed.
    import torch  # noqa: F401

    lib = C.CDLL(LIB_PATH)
    vp, d, i = C.c_void_p, C.c_double, C.c_int
    pd = _P(d)
    lib.daba_workspace_bytes.argtypes = [_P(DabaProblem), _P(DabaOptions)]
    lib.daba_workspace_bytes.restype = C.c_size_t
    lib.daba_create.argtypes = [_P(DabaProblem), _P(DabaOptions), vp, C.c_size_t, vp, _P(vp)]
    lib.daba_iterate.argtypes = [vp, i, pd]
    lib.daba_iterate_timed.argtypes = [vp, i, pd]
    lib.daba_objective.argtypes = [vp, vp, vp, vp, pd]
    lib.daba_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.daba_get_state.argtypes = [vp, pd, pd, pd, pd, pd, pd]
    lib.daba_set_state.argtypes = [vp, pd, pd, pd, pd, pd, pd]
    lib.daba_get_metrics.argtypes = [vp, pd]
    lib.daba_destroy.argtypes = [vp]
    lib.daba_stream_copy.argtypes = [vp, vp, C.c_size_t, i, vp]
    i64 = C.c_int64
    lib.daba_objective_noalloc.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, i, d, vp, vp]
    lib.daba_last_error.argtypes = [vp]
    lib.daba_last_error.restype = C.c_char_p
    # device-level surrogate (include/daba_part.h)
    lib.daba_part_workspace_bytes.argtypes = [_P(DabaProblem), _P(DabaOptions)]
    lib.daba_part_workspace_bytes.restype = C.c_size_t
    lib.daba_part_create.argtypes = [_P(DabaProblem), _P(DabaOptions), vp, C.c_size_t, vp, _P(vp)]
    lib.daba_part_iterate.argtypes = [vp, i, pd]
    lib.daba_part_iterate_timed.argtypes = [vp, i, pd]
    lib.daba_part_get_state.argtypes = [vp, pd, pd, pd]
    lib.daba_part_get_checkpoint.argtypes = [vp, pd, pd, pd, pd, pd]
    lib.daba_part_set_checkpoint.argtypes = [vp, pd, pd, pd, pd, pd]
    lib.daba_part_destroy.argtypes = [vp]
    lib.daba_part_last_error.argtypes = [vp]
    lib.daba_part_last_error.restype = C.c_char_p
    for name in ("daba_create", "daba_iterate", "daba_iterate_timed", "daba_objective", "daba_grad",
                 "daba_get_state", "daba_set_state", "daba_get_metrics", "daba_destroy", "daba_stream_copy",
                 "daba_objective_noalloc",
                 "daba_part_create", "daba_part_iterate", "daba_part_iterate_timed", "daba_part_get_state",
                 "daba_part_get_checkpoint", "daba_part_set_checkpoint", "daba_part_destroy"):
        getattr(lib, name).restype = C.c_int
    return lib


lib = _load()


def check(rc: int, where: str, handle=None):
    if rc != DABA_OK:
        detail = lib.daba_last_error(handle).decode()
        raise DabaError(rc, where, detail)


def check_part(rc: int, where: str, handle=None):
    if rc != DABA_OK:
        detail = lib.daba_part_last_error(handle).decode()
        raise DabaError(rc, where, detail)


def objective_noalloc(obs_camera, obs_landmark, obs_uv, cameras, landmarks, F_out, loss="huber", delta=1.0,
                      stream=None):
    """daba_objective_noalloc on torch device tensors (int32 observation
    lists, float64 pixels, cameras [M, 15], landmarks [N, 3], F_out one
    float64): enqueues on `stream` (default: torch's current stream) and
    returns; raises DabaError for a rejected argument."""
    import torch
    M, N, K = cameras.shape[0], landmarks.shape[0], obs_camera.shape[0]
    for t in (obs_camera, obs_landmark, obs_uv, cameras, landmarks, F_out):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("objective_noalloc takes contiguous device tensors")
    s = (stream or torch.cuda.current_stream()).cuda_stream
    rc = lib.daba_objective_noalloc(M, N, K, obs_camera.data_ptr(), obs_landmark.data_ptr(), obs_uv.data_ptr(),
                                    cameras.data_ptr(), landmarks.data_ptr(), LOSS[loss], float(delta),
                                    F_out.data_ptr(), s)
    if rc != DABA_OK:
        raise DabaError(rc, "daba_objective_noalloc", "argument rejected or launch failed")
