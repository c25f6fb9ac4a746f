"""Problems in the Bundle Adjustment in the Large (BAL) text format, converted
to this library's problem dictionary (the one `DabaSolver` takes).

BAL file layout (whitespace-separated text):
    n_cameras n_points n_observations
    camera_index point_index x y          (n_observations lines)
    9 numbers per camera: Rodrigues vector w (3), t (3), f, k1, k2
    3 numbers per point
BAL camera model: P = R(w) X + t; p = -P_xy / P_z; the observed pixel (from
the image centre) is u = f (1 + k1 |p|^2 + k2 |p|^4) p.

This library's camera (Sec. III):
- the camera frame is X_c = R^T (X - t), with +z the optical axis;
- the ray through pixel u is (u, d1 + d2 |u|^2 + d3 |u|^4);
- a point projects where u / (d1 + d2 |u|^2 + d3 |u|^4) = X_c,xy / X_c,z.

The paper uses BAL scenes, but does not say how it converts BAL's forward
distortion into its undistortion model. This module reads it as follows.

- Frames. X_c = D P with D = diag(1, -1, -1), a rotation, so
  R = (D R(w))^T and t = -R(w)^T t_BAL. D turns the image's y axis, so the
  observed y is negated.
- Intrinsics. BAL maps the normalised radius rho to the pixel radius
  r = f (1 + k1 rho^2 + k2 rho^4) rho, so r / rho = f (1 + k1 rho^2 + k2 rho^4).
  d is the least-squares fit of d1 + d2 r^2 + d3 r^4 to r / rho over radii
  from 0 to the camera's largest observed radius. With k1 = k2 = 0 the fit
  is exact: d = (f, 0, 0).
"""

from __future__ import annotations

import io

import numpy as np

_D = np.diag([1.0, -1.0, -1.0])


def read_bal(src) -> dict:
    """The raw arrays of a BAL file (a path or a text stream): obs_camera,
    obs_point (int [K]), obs_xy (float [K, 2]), cameras (float [M, 9]) and
    points (float [N, 3])."""
    text = open(src).read() if isinstance(src, str) else src.read()
    tok = text.split()
    if len(tok) < 3:
        raise ValueError("not a BAL file: no header")
    M, N, K = int(tok[0]), int(tok[1]), int(tok[2])
    need = 3 + 4 * K + 9 * M + 3 * N
    if M < 1 or N < 1 or K < 0 or len(tok) < need:
        raise ValueError(f"not a BAL file: header ({M}, {N}, {K}) needs {need} numbers, found {len(tok)}")
    o = np.array(tok[3:3 + 4 * K], dtype=np.float64).reshape(K, 4)
    cams = np.array(tok[3 + 4 * K:3 + 4 * K + 9 * M], dtype=np.float64).reshape(M, 9)
    pts = np.array(tok[3 + 4 * K + 9 * M:need], dtype=np.float64).reshape(N, 3)
    ci, pi = o[:, 0].astype(np.int64), o[:, 1].astype(np.int64)
    if K and (ci.min() < 0 or ci.max() >= M or pi.min() < 0 or pi.max() >= N):
        raise ValueError("observation index out of range")
    return dict(obs_camera=ci, obs_point=pi, obs_xy=o[:, 2:4].copy(), cameras=cams, points=pts)


def write_bal(dst, raw: dict) -> None:
    """Writes raw arrays (as read_bal returns them) in the BAL text format to
    a path or a text stream."""
    out = io.StringIO()
    K = raw["obs_camera"].size
    out.write(f"{raw['cameras'].shape[0]} {raw['points'].shape[0]} {K}\n")
    for c, p, (x, y) in zip(raw["obs_camera"], raw["obs_point"], raw["obs_xy"]):
        out.write(f"{int(c)} {int(p)} {x:.17g} {y:.17g}\n")
    for v in np.asarray(raw["cameras"]).reshape(-1):
        out.write(f"{v:.17g}\n")
    for v in np.asarray(raw["points"]).reshape(-1):
        out.write(f"{v:.17g}\n")
    if isinstance(dst, str):
        with open(dst, "w") as f:
            f.write(out.getvalue())
    else:
        dst.write(out.getvalue())


def rodrigues(w: np.ndarray) -> np.ndarray:
    """Rotation matrices R = exp([w]x) for axis-angle vectors w (..., 3)."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w, axis=-1)[..., None, None]
    K = np.zeros(w.shape[:-1] + (3, 3))
    K[..., 0, 1], K[..., 0, 2], K[..., 1, 2] = -w[..., 2], w[..., 1], -w[..., 0]
    K[..., 1, 0], K[..., 2, 0], K[..., 2, 1] = w[..., 2], -w[..., 1], w[..., 0]
    small = th < 1e-8
    ths = np.where(small, 1.0, th)
    A = np.where(small, 1.0, np.sin(ths) / ths)
    B = np.where(small, 0.5, (1.0 - np.cos(ths)) / (ths * ths))
    return np.eye(3) + A * K + B * (K @ K)


def fit_intrinsics(f: float, k1: float, k2: float, r_max: float, samples: int = 64):
    """d = (d1, d2, d3) with d1 + d2 r^2 + d3 r^4 ~ r / rho(r) on [0, r_max],
    where BAL's model gives r = f (1 + k1 rho^2 + k2 rho^4) rho; returns d and
    the largest relative error of the fit on the samples."""
    if k1 == 0.0 and k2 == 0.0:
        return np.array([f, 0.0, 0.0]), 0.0
    r_max = max(float(r_max), 1.0)
    # rho up to the one that reaches r_max (BAL's radius is increasing there)
    rho_max = r_max / f
    for _ in range(60):
        g = f * (1 + k1 * rho_max ** 2 + k2 * rho_max ** 4) * rho_max - r_max
        dg = f * (1 + 3 * k1 * rho_max ** 2 + 5 * k2 * rho_max ** 4)
        if dg <= 0:
            raise ValueError("BAL distortion is not monotone over the observed radii")
        rho_max -= g / dg
    rho = np.linspace(0.0, rho_max, samples)
    y = f * (1 + k1 * rho ** 2 + k2 * rho ** 4)  # r / rho
    r = y * rho
    s = r / r_max  # scaled radius for conditioning
    A = np.stack([np.ones_like(s), s ** 2, s ** 4], axis=1)
    c, *_ = np.linalg.lstsq(A, y, rcond=None)
    d = np.array([c[0], c[1] / r_max ** 2, c[2] / r_max ** 4])
    err = np.max(np.abs(A @ c - y) / y)
    return d, float(err)


def bal_to_problem(raw: dict) -> dict:
    """The BAL scene as this library's problem dictionary: obs_camera,
    obs_landmark (int32), obs_uv (pixels, y negated), cameras (R row-major,
    t, d) and landmarks, plus intrinsics_fit_error (per camera)."""
    cams = np.asarray(raw["cameras"], dtype=np.float64)
    M = cams.shape[0]
    Rb = rodrigues(cams[:, 0:3])
    tb = cams[:, 3:6]
    R = np.transpose(_D @ Rb, (0, 2, 1))  # camera axes as columns
    t = -np.einsum("nji,nj->ni", Rb, tb)  # camera centre -R_BAL^T t_BAL
    uv = np.asarray(raw["obs_xy"], dtype=np.float64) * np.array([1.0, -1.0])
    ci = np.asarray(raw["obs_camera"], dtype=np.int64)
    rad = np.zeros(M)
    if ci.size:
        np.maximum.at(rad, ci, np.linalg.norm(uv, axis=1))
    d = np.zeros((M, 3))
    err = np.zeros(M)
    for i in range(M):
        f, k1, k2 = cams[i, 6:9]
        if not f > 0:
            raise ValueError(f"camera {i}: focal length {f} is not positive")
        d[i], err[i] = fit_intrinsics(f, k1, k2, rad[i])
    cameras = np.concatenate([R.reshape(M, 9), t, d], axis=1)
    return dict(
        n_cameras=M, n_landmarks=int(np.asarray(raw["points"]).shape[0]), n_obs=int(ci.size),
        obs_camera=np.ascontiguousarray(ci, dtype=np.int32),
        obs_landmark=np.ascontiguousarray(raw["obs_point"], dtype=np.int32),
        obs_uv=np.ascontiguousarray(uv), cameras=np.ascontiguousarray(cameras),
        landmarks=np.ascontiguousarray(raw["points"], dtype=np.float64),
        intrinsics_fit_error=err)


def load_bal(src) -> dict:
    """read_bal followed by bal_to_problem."""
    return bal_to_problem(read_bal(src))
