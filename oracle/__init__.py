"""ctypes wrapper of the plain CPU FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  It shares no code with the GPU path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

LOSS = {"trivial": 0, "huber": 1, "welsch": 2}
NEVER_RESTART = 1
ALWAYS_RESTART = 2

_lib = None
_P = C.POINTER


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # a variant build of the oracle (the pins' planted-mistake checks build
    # deliberately broken copies and run the pins against them)
    path = os.environ.get("DABA_ORACLE_LIB") or LIB
    if path == LIB and not os.path.exists(LIB):
        build()
    lib = C.CDLL(path)
    d, i64, i32, u64 = C.c_double, C.c_int64, C.c_int32, C.c_uint64
    pd, pi = _P(d), _P(i32)
    lib.orc_create.argtypes = [i64, i64, i64, pi, pi, pd, pd, pd, C.c_int, pi, pi, d, C.c_int, d, d, d,
                               C.c_int, C.c_int, u64, C.c_int, _P(C.c_void_p)]
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_iterate.argtypes = [C.c_void_p, C.c_int, pd, pd]
    lib.orc_objective.argtypes = [C.c_void_p, pd, pd, pd, pd]
    lib.orc_grad.argtypes = [C.c_void_p, pd, pd, pd, pd, pd, pd]
    lib.orc_get_state.argtypes = [C.c_void_p, pd, pd, pd, pd, pd, pd]
    lib.orc_set_state.argtypes = [C.c_void_p, pd, pd, pd, pd, pd, pd]
    lib.orc_extrapolation.argtypes = [C.c_void_p, pd, pd, pd]
    lib.orc_surrogate.argtypes = [C.c_void_p, pd, pd, pd, pd, pd, pd]
    lib.orc_obs_eval.argtypes = [C.c_void_p, pd, pd, pd, pd]
    lib.orc_PQ.argtypes = [C.c_void_p, pd, pd, pd, pd, pd, pd, pd]
    lib.orc_landmark_min.argtypes = [C.c_void_p, i64, pd, pd, pd]
    lib.orc_camera_min.argtypes = [C.c_void_p, i64, pd, pd, C.c_int, pd, _P(C.c_int)]
    lib.orc_camera_phi.argtypes = [C.c_void_p, i64, pd, pd, pd, pd]
    lib.orc_landmark_phi.argtypes = [C.c_void_p, i64, pd, pd, pd, pd]
    lib.orc_projrot3d.argtypes = [pd, pd]
    lib.orc_cams_to_internal.argtypes = [C.c_void_p, pd, pd, i64]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_num_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(_P(C.c_double))


def _ip(a):
    if a is None:
        return None
    return a.ctypes.data_as(_P(C.c_int32))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def projrot3d(M):
    lib = _load()
    M = _f64(np.asarray(M).reshape(9))
    R = np.empty(9)
    if lib.orc_projrot3d(_dp(M), _dp(R)) != 0:
        raise ValueError("rank-deficient matrix")
    return R.reshape(3, 3)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the OpenMP loops (n < 1: one per processor)."""
    _load().orc_set_num_threads(int(n))


class Oracle:
    """The oracle's state for one problem (see oracle.h for the meaning of
    each call).  Arrays are numpy float64 in caller units unless a method says
    internal units."""

    def __init__(self, prob: dict, *, n_partitions=None, cam_part=None, lm_part=None, unit_scale=512.0,
                 loss="huber", delta=1.0, xi=1e-9, eta=0.5, accelerate=True, inner_steps=1, flags=0,
                 frozen_partition=-1, cameras=None, landmarks=None, uv=None):
        lib = _load()
        self.M, self.N, self.K = int(prob["n_cameras"]), int(prob["n_landmarks"]), int(prob["n_obs"])
        self.S = int(n_partitions if n_partitions is not None else prob.get("n_partitions", 1))
        self.scale = float(unit_scale)
        self._cam = np.ascontiguousarray(prob["obs_camera"], dtype=np.int32)
        self._lm = np.ascontiguousarray(prob["obs_landmark"], dtype=np.int32)
        self._uv = _f64(prob["obs_uv"] if uv is None else uv)
        cams = _f64(prob["cameras"] if cameras is None else cameras)
        lms = _f64(prob["landmarks"] if landmarks is None else landmarks)
        cp = None if cam_part is None else np.ascontiguousarray(cam_part, dtype=np.int32)
        lp = None if lm_part is None else np.ascontiguousarray(lm_part, dtype=np.int32)
        h = C.c_void_p()
        rc = lib.orc_create(self.M, self.N, self.K, _ip(self._cam), _ip(self._lm), _dp(self._uv), _dp(cams),
                            _dp(lms), self.S, _ip(cp), _ip(lp), self.scale, LOSS[loss], float(delta),
                            float(xi), float(eta), int(bool(accelerate)), int(inner_steps), int(flags),
                            int(frozen_partition), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc})")
        self._h = h
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def _chk(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed ({rc})")

    def iterate(self, n: int):
        F = np.empty(n)
        mt = np.empty((n, self.S, 4))
        self._chk(self._lib.orc_iterate(self._h, n, _dp(F), _dp(mt)), "orc_iterate")
        return F, mt

    def objective(self, cams=None, lms=None, uv=None) -> float:
        out = np.empty(1)
        self._chk(self._lib.orc_objective(self._h, _dp(_f64(cams)), _dp(_f64(lms)), _dp(_f64(uv)), _dp(out)),
                  "orc_objective")
        return float(out[0])

    def grad(self, cams=None, lms=None, uv=None):
        gc, gl, gu = np.empty((self.M, 15)), np.empty((self.N, 3)), np.empty((self.K, 2))
        self._chk(self._lib.orc_grad(self._h, _dp(_f64(cams)), _dp(_f64(lms)), _dp(_f64(uv)), _dp(gc), _dp(gl),
                                     _dp(gu)), "orc_grad")
        return gc, gl, gu

    def get_state(self):
        c, l = np.empty((self.M, 15)), np.empty((self.N, 3))
        cp, lp = np.empty((self.M, 15)), np.empty((self.N, 3))
        p4, sc = np.empty((self.S, 4)), np.empty(2)
        self._chk(self._lib.orc_get_state(self._h, _dp(c), _dp(l), _dp(cp), _dp(lp), _dp(p4), _dp(sc)),
                  "orc_get_state")
        return dict(cams=c, lms=l, cams_prev=cp, lms_prev=lp, part=p4, s=sc[0], k=int(sc[1]))

    def set_state(self, st: dict):
        sc = np.array([st["s"], st["k"]], dtype=np.float64)
        self._chk(self._lib.orc_set_state(self._h, _dp(_f64(st["cams"])), _dp(_f64(st["lms"])),
                                          _dp(_f64(st["cams_prev"])), _dp(_f64(st["lms_prev"])),
                                          _dp(_f64(st["part"])), _dp(sc)), "orc_set_state")

    def extrapolation(self):
        """gamma^a(k) per partition and x-bar^(k) (caller units) that the next
        iteration would use; the state is not changed."""
        g, cb, lb = np.empty(self.S), np.empty((self.M, 15)), np.empty((self.N, 3))
        self._chk(self._lib.orc_extrapolation(self._h, _dp(g), _dp(cb), _dp(lb)), "orc_extrapolation")
        return g, cb, lb

    def surrogate(self, cams_x, lms_x, cams_y, lms_y):
        E, dE = np.empty(self.S), np.empty(self.S)
        self._chk(self._lib.orc_surrogate(self._h, _dp(_f64(cams_x)), _dp(_f64(lms_x)), _dp(_f64(cams_y)),
                                          _dp(_f64(lms_y)), _dp(E), _dp(dE)), "orc_surrogate")
        return E, dE

    # ---- internal-unit probes used by the pins
    def to_internal(self, cams):
        cams = _f64(cams)
        out = np.empty_like(cams)
        self._lib.orc_cams_to_internal(self._h, _dp(cams), _dp(out), cams.shape[0])
        return out

    def obs_eval(self, c15, l3, u2):
        out = np.empty(16)
        self._chk(self._lib.orc_obs_eval(self._h, _dp(_f64(c15)), _dp(_f64(l3)), _dp(_f64(u2)), _dp(out)),
                  "orc_obs_eval")
        return dict(p=out[0:3], lam=out[3], e=out[4:7], s=out[7], rho=out[8], w=out[9], a=out[10],
                    g=out[11:14], F=out[14])

    def PQ(self, u2, cy, ly, c, l):
        P, Q = np.empty(1), np.empty(1)
        self._chk(self._lib.orc_PQ(self._h, _dp(_f64(u2)), _dp(_f64(cy)), _dp(_f64(ly)), _dp(_f64(c)),
                                   _dp(_f64(l)), _dp(P), _dp(Q)), "orc_PQ")
        return float(P[0]), float(Q[0])

    def landmark_min(self, j, cams_y, lms_y):
        out = np.empty(3)
        self._chk(self._lib.orc_landmark_min(self._h, j, _dp(_f64(cams_y)), _dp(_f64(lms_y)), _dp(out)),
                  "orc_landmark_min")
        return out

    def camera_min(self, i, cams_y, lms_y, inner_steps=1):
        out = np.empty(15)
        ns = C.c_int()
        self._chk(self._lib.orc_camera_min(self._h, i, _dp(_f64(cams_y)), _dp(_f64(lms_y)), inner_steps,
                                           _dp(out), C.byref(ns)), "orc_camera_min")
        return out, ns.value

    def camera_phi(self, i, cams_y, lms_y, c):
        out = np.empty(1)
        self._chk(self._lib.orc_camera_phi(self._h, i, _dp(_f64(cams_y)), _dp(_f64(lms_y)), _dp(_f64(c)),
                                           _dp(out)), "orc_camera_phi")
        return float(out[0])

    def landmark_phi(self, j, cams_y, lms_y, l):
        out = np.empty(1)
        self._chk(self._lib.orc_landmark_phi(self._h, j, _dp(_f64(cams_y)), _dp(_f64(lms_y)), _dp(_f64(l)),
                                             _dp(out)), "orc_landmark_phi")
        return float(out[0])
