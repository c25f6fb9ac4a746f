"""Python face of the DABA library: a solver object over one problem and a
torch.autograd.Function for the robust objective.

PyTorch is used only for device memory (the workspace, inputs and outputs)
and for the stream; all computation runs in libdaba.so.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B

_P = C.POINTER


def _np(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, ctype):
    return None if a is None else a.ctypes.data_as(_P(ctype))


def _dev_ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("device arrays must be contiguous float64 CUDA tensors")
    return C.c_void_p(t.data_ptr())


class DabaSolver:
    """One problem on one GPU.

    prob: dict with obs_camera, obs_landmark (int [K]), obs_uv (float [K,2],
    pixels from the image centre), cameras (float [M,15] = R row-major | t |
    d), landmarks (float [N,3]) and n_cameras / n_landmarks / n_obs.
    """

    def __init__(self, prob: dict, *, n_partitions=None, camera_partition=None, landmark_partition=None,
                 unit_scale=512.0, loss="huber", delta=1.0, xi=1e-9, eta=0.5, accelerate=True, inner_steps=1,
                 precision="fp64", debug_flags=0, device="cuda", cameras=None, landmarks=None):
        if not torch.cuda.is_available():
            raise RuntimeError("DabaSolver needs a GPU (torch.cuda is not available)")
        self.device = torch.device(device)
        self.M, self.N, self.K = int(prob["n_cameras"]), int(prob["n_landmarks"]), int(prob["n_obs"])
        self.S = int(n_partitions if n_partitions is not None else prob.get("n_partitions", 1))
        self.scale = float(unit_scale)
        self.precision = precision
        self._keep = dict(
            cam=_np(prob["obs_camera"], np.int32), lm=_np(prob["obs_landmark"], np.int32),
            uv=_np(prob["obs_uv"], np.float64),
            cams=_np(prob["cameras"] if cameras is None else cameras, np.float64),
            lms=_np(prob["landmarks"] if landmarks is None else landmarks, np.float64),
            cp=_np(camera_partition, np.int32), lp=_np(landmark_partition, np.int32))
        k = self._keep
        self._prob = B.DabaProblem(self.M, self.N, self.K, _ptr(k["cam"], C.c_int32), _ptr(k["lm"], C.c_int32),
                                   _ptr(k["uv"], C.c_double), _ptr(k["cams"], C.c_double),
                                   _ptr(k["lms"], C.c_double), self.S, _ptr(k["cp"], C.c_int32),
                                   _ptr(k["lp"], C.c_int32), self.scale)
        self._opt = B.DabaOptions(B.LOSS[loss], float(delta), float(xi), float(eta), int(bool(accelerate)),
                                  int(inner_steps), B.PRECISION[precision], int(debug_flags))
        nbytes = B.lib.daba_workspace_bytes(C.byref(self._prob), C.byref(self._opt))
        if nbytes == 0:
            h = C.c_void_p()
            rc = B.lib.daba_create(C.byref(self._prob), C.byref(self._opt), None, 0, None, C.byref(h))
            B.check(rc, "daba_create")
        self.workspace_bytes = int(nbytes)
        with torch.cuda.device(self.device):
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            self.stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            rc = B.lib.daba_create(C.byref(self._prob), C.byref(self._opt), C.c_void_p(aligned), nbytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        B.check(rc, "daba_create")
        self._h = h

    # -- lifetime
    def close(self):
        h = getattr(self, "_h", None)
        if h and B is not None and getattr(B, "lib", None) is not None:
            B.lib.daba_destroy(h)
        self._h = None

    def __del__(self):
        self.close()

    def _chk(self, rc, where):
        B.check(rc, where, self._h)

    # -- Algorithm 1
    def iterate(self, n: int, trace: bool = True):
        """n iterations; returns F after each (pixels^2) when trace is set."""
        if trace:
            F = np.empty(n)
            self._chk(B.lib.daba_iterate(self._h, n, _ptr(F, C.c_double)), "daba_iterate")
            return F
        self._chk(B.lib.daba_iterate(self._h, n, None), "daba_iterate")
        return None

    def iterate_timed(self, n: int):
        """n iterations; returns summed GPU ms of (camera tiles, landmark
        passes, camera solves, restart tests and the closing store of the
        iterate)."""
        ms = np.zeros(4)
        self._chk(B.lib.daba_iterate_timed(self._h, n, _ptr(ms, C.c_double)), "daba_iterate_timed")
        return ms

    def objective(self, cams=None, lms=None, uv=None) -> float:
        out = np.empty(1)
        self._chk(B.lib.daba_objective(self._h, _dev_ptr(cams), _dev_ptr(lms), _dev_ptr(uv),
                                       _ptr(out, C.c_double)), "daba_objective")
        return float(out[0])

    def grad(self, cams=None, lms=None, uv=None, want=(True, True, True)):
        """Euclidean gradient of F (caller units) as float64 device tensors
        (cams [M,15], lms [N,3], uv [K,2]); the stream is synchronized."""
        dev = self.device
        gc = torch.empty((self.M, 15), dtype=torch.float64, device=dev) if want[0] else None
        gl = torch.empty((self.N, 3), dtype=torch.float64, device=dev) if want[1] else None
        gu = torch.empty((self.K, 2), dtype=torch.float64, device=dev) if want[2] else None
        self._chk(B.lib.daba_grad(self._h, _dev_ptr(cams), _dev_ptr(lms), _dev_ptr(uv), _dev_ptr(gc),
                                  _dev_ptr(gl), _dev_ptr(gu)), "daba_grad")
        self.stream.synchronize()
        return gc, gl, gu

    def get_state(self) -> dict:
        c, l = np.empty((self.M, 15)), np.empty((self.N, 3))
        cp, lp = np.empty((self.M, 15)), np.empty((self.N, 3))
        p4, sc = np.empty((self.S, 4)), np.empty(2)
        self._chk(B.lib.daba_get_state(self._h, _ptr(c, C.c_double), _ptr(l, C.c_double), _ptr(cp, C.c_double),
                                       _ptr(lp, C.c_double), _ptr(p4, C.c_double), _ptr(sc, C.c_double)),
                  "daba_get_state")
        return dict(cams=c, lms=l, cams_prev=cp, lms_prev=lp, part=p4, s=float(sc[0]), k=int(sc[1]))

    def set_state(self, st: dict):
        sc = np.array([st["s"], st["k"]], dtype=np.float64)
        arrs = [_np(st.get(n), np.float64) for n in ("cams", "lms", "cams_prev", "lms_prev", "part")]
        self._chk(B.lib.daba_set_state(self._h, *[_ptr(a, C.c_double) for a in arrs], _ptr(sc, C.c_double)),
                  "daba_set_state")

    def metrics(self) -> np.ndarray:
        m = np.empty((self.S, 4))
        self._chk(B.lib.daba_get_metrics(self._h, _ptr(m, C.c_double)), "daba_get_metrics")
        return m


class DabaPartSolver:
    """One problem on one GPU with the device-level surrogate of eq. Ealpha
    (include/daba_part.h): pairs inside a partition exact, pairs between
    partitions majorized, one Levenberg-Marquardt solve per partition.  Same
    problem dict and options as DabaSolver; FP64 only, inner_steps >= 1."""

    def __init__(self, prob: dict, *, n_partitions=None, camera_partition=None, landmark_partition=None,
                 unit_scale=512.0, loss="huber", delta=1.0, xi=1e-9, eta=0.5, accelerate=True, inner_steps=1,
                 debug_flags=0, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("DabaPartSolver needs a GPU (torch.cuda is not available)")
        self.device = torch.device(device)
        self.M, self.N, self.K = int(prob["n_cameras"]), int(prob["n_landmarks"]), int(prob["n_obs"])
        self.S = int(n_partitions if n_partitions is not None else prob.get("n_partitions", 1))
        self.scale = float(unit_scale)
        self._keep = dict(
            cam=_np(prob["obs_camera"], np.int32), lm=_np(prob["obs_landmark"], np.int32),
            uv=_np(prob["obs_uv"], np.float64), cams=_np(prob["cameras"], np.float64),
            lms=_np(prob["landmarks"], np.float64),
            cp=_np(camera_partition, np.int32), lp=_np(landmark_partition, np.int32))
        k = self._keep
        self._prob = B.DabaProblem(self.M, self.N, self.K, _ptr(k["cam"], C.c_int32), _ptr(k["lm"], C.c_int32),
                                   _ptr(k["uv"], C.c_double), _ptr(k["cams"], C.c_double),
                                   _ptr(k["lms"], C.c_double), self.S, _ptr(k["cp"], C.c_int32),
                                   _ptr(k["lp"], C.c_int32), self.scale)
        self._opt = B.DabaOptions(B.LOSS[loss], float(delta), float(xi), float(eta), int(bool(accelerate)),
                                  int(inner_steps), B.PRECISION["fp64"], int(debug_flags))
        nbytes = B.lib.daba_part_workspace_bytes(C.byref(self._prob), C.byref(self._opt))
        if nbytes == 0:
            h = C.c_void_p()
            rc = B.lib.daba_part_create(C.byref(self._prob), C.byref(self._opt), None, 0, None, C.byref(h))
            B.check_part(rc, "daba_part_create")
        self.workspace_bytes = int(nbytes)
        with torch.cuda.device(self.device):
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self._ws.data_ptr() + 255) // 256 * 256
            self.stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            rc = B.lib.daba_part_create(C.byref(self._prob), C.byref(self._opt), C.c_void_p(aligned), nbytes,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h))
        B.check_part(rc, "daba_part_create")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h and B is not None and getattr(B, "lib", None) is not None:
            B.lib.daba_part_destroy(h)
        self._h = None

    def __del__(self):
        self.close()

    def _chk(self, rc, where):
        B.check_part(rc, where, self._h)

    def iterate(self, n: int, trace: bool = True):
        """n iterations; returns F after each (pixels^2) when trace is set."""
        F = np.empty(n) if trace else None
        self._chk(B.lib.daba_part_iterate(self._h, n, _ptr(F, C.c_double)), "daba_part_iterate")
        return F

    def iterate_timed(self, n: int) -> dict:
        """n iterations with every launch group timed; returns ms per group
        and the LM attempts and Cholesky launches made."""
        ms = np.zeros(8)
        self._chk(B.lib.daba_part_iterate_timed(self._h, n, _ptr(ms, C.c_double)), "daba_part_iterate_timed")
        keys = ("eval", "normal_eq", "schur", "cholesky", "solve", "rest")
        out = {k: float(v) for k, v in zip(keys, ms[:6])}
        out.update(lm_attempts=int(ms[6]), cholesky_launches=int(ms[7]))
        return out

    def get_state(self) -> dict:
        c, l, m = np.empty((self.M, 15)), np.empty((self.N, 3)), np.empty((self.S, 4))
        self._chk(B.lib.daba_part_get_state(self._h, _ptr(c, C.c_double), _ptr(l, C.c_double), _ptr(m, C.c_double)),
                  "daba_part_get_state")
        return dict(cams=c, lms=l, metrics=m)

    def checkpoint(self) -> dict:
        """x^k, x^(k-1) and per partition (Fbar^a(k-1), E^a(k), s^a(k))."""
        c, l = np.empty((self.M, 15)), np.empty((self.N, 3))
        cp, lp, p3 = np.empty((self.M, 15)), np.empty((self.N, 3)), np.empty((self.S, 3))
        self._chk(B.lib.daba_part_get_checkpoint(self._h, *[_ptr(a, C.c_double) for a in (c, l, cp, lp, p3)]),
                  "daba_part_get_checkpoint")
        return dict(cams=c, lms=l, cams_prev=cp, lms_prev=lp, part3=p3)

    def restore(self, ck: dict):
        """Continue from a checkpoint of a solver of the same problem and options."""
        arrs = [_np(ck.get(n), np.float64) for n in ("cams", "lms", "cams_prev", "lms_prev", "part3")]
        self._chk(B.lib.daba_part_set_checkpoint(self._h, *[_ptr(a, C.c_double) for a in arrs]),
                  "daba_part_set_checkpoint")


class DabaObjective(torch.autograd.Function):
    """F(cams, lms, uv) of Problem 1 with the hand-written adjoint of App. D.

    Inputs are float64 CUDA tensors in caller units: cams [M,15] (R row-major,
    t, d = (f, f k1, f k2)), lms [N,3], uv [K,2].  Gradients flow to all three;
    build d from (f, k1, k2) with torch ops to get gradients in those."""

    @staticmethod
    def forward(ctx, solver: DabaSolver, cams, lms, uv):
        cams, lms, uv = cams.contiguous(), lms.contiguous(), uv.contiguous()
        F = solver.objective(cams, lms, uv)
        ctx.solver = solver
        ctx.save_for_backward(cams, lms, uv)
        return torch.tensor(F, dtype=torch.float64, device=cams.device)

    @staticmethod
    def backward(ctx, gF):
        cams, lms, uv = ctx.saved_tensors
        want = ctx.needs_input_grad[1:4]
        gc, gl, gu = ctx.solver.grad(cams, lms, uv, want=want)
        scale = gF.to(torch.float64)
        return (None, None if gc is None else gc * scale, None if gl is None else gl * scale,
                None if gu is None else gu * scale)


def daba_objective(solver: DabaSolver, cams, lms, uv):
    return DabaObjective.apply(solver, cams, lms, uv)
