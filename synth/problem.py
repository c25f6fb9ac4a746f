"""Synthetic problems shaped like the paper's large BAL / 1DSfM scenes.

The paper evaluates on public datasets (Table II) that are not available
here; these seeded problems stand in for them at matching shapes.  Recipe:

* cameras on a sphere of radius 10 around the origin, optical axis (+z of the
  camera frame) pointing at the origin, uniform random roll;
* R_i holds the camera axes as columns (a point l is at X = R_i^T (l - t_i)
  in the camera frame) and t_i is the camera centre;
* focal length f = 500 px, radial coefficients kappa1, kappa2 ~ N(0, 1e-3)
  (the 1e-3 is a variance) on the normalised radius |u|/f, so the paper's
  intrinsics d = (f, f k1, f k2) are (f, kappa1/f, kappa2/f^3) in pixels;
* 640 x 480 image, pixels measured from the image centre;
* landmarks ~ N(0, I3);
* each landmark is seen by a set of distinct, uniformly drawn cameras in
  whose image it falls: min(8, #visible) of them, or 2 + Geometric(1/5)
  (mean 6) for the largest configuration;
* pixel noise N(0, 1 px^2) per coordinate, and 5 % of observations replaced
  by a uniform draw over the image (outliers);
* the initial guess is the ground truth with each rotation turned by
  0.05 rad about a uniform random axis, camera centres and landmarks moved by
  N(0, 0.1^2 I3); intrinsics start at their true values.

The observed pixel of a landmark is found by inverting the undistortion model
of Sec. III: with X the point in the camera frame and rho = |X_xy| / X_z, the
distorted radius r solves r = rho (d1 + d2 r^2 + d3 r^4), and u = r X_xy/|X_xy|.
"""

from __future__ import annotations

import math

import numpy as np

IMAGE_HALF = (320.0, 240.0)

# name -> (cameras, landmarks, track model, partitions, iterations, precision)
CONFIGS = {
    # 50 cameras, 5,000 landmarks, ~40k observations
    "cam50-lm5k": dict(n_cameras=50, n_landmarks=5_000, track="fixed8", n_partitions=1,
                       iterations=100, precision="fp64"),
    # 1,000 cameras, 200,000 landmarks, ~1.6M observations
    "cam1k-lm200k": dict(n_cameras=1_000, n_landmarks=200_000, track="fixed8", n_partitions=8,
                         iterations=200, precision="fp64"),
    # 5,000 cameras, 2,000,000 landmarks, ~16M observations
    "cam5k-lm2m": dict(n_cameras=5_000, n_landmarks=2_000_000, track="fixed8", n_partitions=16,
                       iterations=200, precision="fp32_mixed"),
    # the 1.6M-observation shape with another seed (gradient checks)
    "cam1k-lm200k-grad": dict(n_cameras=1_000, n_landmarks=200_000, track="fixed8", n_partitions=8,
                              iterations=0, precision="fp64"),
    # 20,000 cameras, 10,000,000 landmarks, ~60M observations (tracks 2 + Geometric(1/5))
    "cam20k-lm10m": dict(n_cameras=20_000, n_landmarks=10_000_000, track="geom6", n_partitions=64,
                         iterations=300, precision="fp32_mixed"),
}

_CONFIG_SEED = {"cam50-lm5k": 1, "cam1k-lm200k": 2, "cam5k-lm2m": 3, "cam1k-lm200k-grad": 4, "cam20k-lm10m": 5}


def _rotation_exp(w: np.ndarray) -> np.ndarray:
    """Rotation matrices exp([w]x) for an array of axis-angle vectors (..., 3)."""
    th = np.linalg.norm(w, axis=-1, keepdims=True)
    k = np.where(th > 0, w / np.where(th > 0, th, 1.0), 0.0)
    kx, ky, kz = k[..., 0], k[..., 1], k[..., 2]
    zero = np.zeros_like(kx)
    K = np.stack([np.stack([zero, -kz, ky], -1),
                  np.stack([kz, zero, -kx], -1),
                  np.stack([-ky, kx, zero], -1)], -2)
    s = np.sin(th)[..., None]
    c = np.cos(th)[..., None]
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + s * K + (1.0 - c) * (K @ K)


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _make_cameras(rng: np.random.Generator, m: int):
    centre = 10.0 * _unit_vectors(rng, m)
    z = -centre / np.linalg.norm(centre, axis=1, keepdims=True)
    a = rng.standard_normal((m, 3))
    x = a - np.sum(a * z, axis=1, keepdims=True) * z
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=2)  # columns are the camera axes
    f = np.full(m, 500.0)
    kappa = rng.normal(0.0, math.sqrt(1e-3), size=(m, 2))
    d = np.stack([f, kappa[:, 0] / f, kappa[:, 1] / f ** 3], axis=1)
    return R, centre, d


def _project(R, t, d, lm):
    """Distorted pixel of points lm seen by cameras (R, t, d); all arrays are
    broadcast per row.  Returns (u, ok) where ok marks points in front of the
    camera, inside the image and with a converged radius."""
    X = np.einsum("nji,nj->ni", R, lm - t)
    z = X[:, 2]
    front = z > 1e-9
    zs = np.where(front, z, 1.0)
    xy = X[:, :2]
    nxy = np.linalg.norm(xy, axis=1)
    rho = nxy / zs
    d1, d2, d3 = d[:, 0], d[:, 1], d[:, 2]
    r = rho * d1
    # 30 Newton steps; an entry whose step is exactly zero stays where it is
    # for every later step, so only the others are iterated further
    act = np.arange(r.size)
    for _ in range(30):
        ra, pa = r[act], rho[act]
        a1, a2, a3 = d1[act], d2[act], d3[act]
        r2 = ra * ra
        g = ra - pa * (a1 + a2 * r2 + a3 * r2 * r2)
        dg = 1.0 - pa * (2.0 * a2 * ra + 4.0 * a3 * r2 * ra)
        rn = ra - g / dg
        r[act] = rn
        act = act[rn != ra]
        if act.size == 0:
            break
    r2 = r * r
    conv = np.abs(r - rho * (d1 + d2 * r2 + d3 * r2 * r2)) <= 1e-11 * np.maximum(1.0, r)
    safe = np.where(nxy > 0, nxy, 1.0)
    u = np.where((nxy > 0)[:, None], xy * (r / safe)[:, None], 0.0)
    inside = (np.abs(u[:, 0]) <= IMAGE_HALF[0]) & (np.abs(u[:, 1]) <= IMAGE_HALF[1])
    return u, front & inside & conv & (r >= 0)


def _choose_tracks(rng, R, t, d, lm, want):
    """For each landmark j pick want[j] distinct uniformly drawn cameras that
    see it (fewer if not enough do).  Returns (cam, lmk, uv_clean) arrays."""
    m = R.shape[0]
    n = lm.shape[0]
    cams, lmks, uvs = [], [], []
    chunk = 200_000 if m > 256 else max(1, 2_000_000 // max(m, 1))
    for s0 in range(0, n, chunk):
        s1 = min(n, s0 + chunk)
        ids = np.arange(s0, s1)
        w = want[s0:s1]
        if m <= 256:
            # exhaustive: a random permutation of all cameras per landmark
            keys = rng.random((s1 - s0, m))
            order = np.argsort(keys, axis=1)
            jj = np.repeat(ids, m)
            cc = order.reshape(-1)
            u, ok = _project(R[cc], t[cc], d[cc], lm[jj])
            ok = ok.reshape(s1 - s0, m)
            rank = np.cumsum(ok, axis=1) - 1
            take = ok & (rank < w[:, None])
            sel = take.reshape(-1)
            cams.append(cc[sel]); lmks.append(jj[sel]); uvs.append(u[sel])
            continue
        # large camera sets: sample candidates with replacement, drop
        # repeats and invisible ones, keep the first want[j] in draw order;
        # repeat for landmarks still short of cameras.
        need = w.copy()
        pend = np.arange(s1 - s0)
        have = np.zeros(s1 - s0, np.int64)
        seen_pairs = []
        for _round in range(20):
            if pend.size == 0:
                break
            ncand = np.ceil(1.3 * need[pend]).astype(np.int64) + 4
            jj_local = np.repeat(pend, ncand)
            cc = rng.integers(0, m, size=jj_local.size)
            if seen_pairs:
                prev = np.concatenate(seen_pairs)
            else:
                prev = np.empty((0, 2), np.int64)
            key_new = np.stack([jj_local, cc], 1)
            allk = np.concatenate([prev, key_new])
            # pairs ordered by (landmark, camera), draw order among equal
            # pairs (a stable sort of one combined key)
            ks = allk[:, 0] * m + allk[:, 1]
            o = np.argsort(ks, kind="stable")
            ks = ks[o]
            dup_sorted = np.zeros(ks.shape[0], bool)
            dup_sorted[1:] = ks[1:] == ks[:-1]
            dup = np.empty_like(dup_sorted)
            dup[o] = dup_sorted
            dup = dup[prev.shape[0]:]
            u, ok = _project(R[cc], t[cc], d[cc], lm[s0 + jj_local])
            valid = ok & ~dup
            # rank of each valid candidate within its landmark, in draw order
            csum = np.cumsum(valid)
            start = np.concatenate([[0], np.cumsum(ncand)[:-1]])
            base = np.where(start > 0, csum[start - 1], 0)
            rank = csum - 1 - np.repeat(base, ncand) + np.repeat(have[pend], ncand)
            take = valid & (rank < np.repeat(w[pend], ncand))
            cams.append(cc[take]); lmks.append(s0 + jj_local[take]); uvs.append(u[take])
            seen_pairs.append(key_new[valid])
            add = np.bincount(jj_local[take], minlength=s1 - s0)
            have += add
            short = have[pend] < w[pend]
            pend = pend[short]
            need = np.maximum(w - have, 0)
    return (np.concatenate(cams).astype(np.int64), np.concatenate(lmks).astype(np.int64),
            np.concatenate(uvs))


def make_problem(config: str = "cam50-lm5k", seed: int | None = None, *, n_cameras=None,
                 n_landmarks=None, track=None, n_partitions=None, outlier_rate=0.05,
                 pixel_sigma=1.0, rot_perturb=0.05, trans_perturb=0.1,
                 point_perturb=0.1, shuffle=True):
    """Draw one problem.  Size keywords override the named configuration so
    that tests can make small problems of the same kind.

    Returns a dict of numpy arrays:
      obs_camera, obs_landmark (int32 [K]), obs_uv (float64 [K,2], pixels from
      the image centre), obs_uv_clean (same without noise or outliers),
      cameras (float64 [M,15] = R row-major | t | d), landmarks (float64 [N,3])
      as the perturbed initial guess, cameras_gt / landmarks_gt, is_outlier,
      plus the scalars n_cameras, n_landmarks, n_obs, n_partitions, seed.
    """
    cfg = dict(CONFIGS[config])
    if n_cameras is not None:
        cfg["n_cameras"] = n_cameras
    if n_landmarks is not None:
        cfg["n_landmarks"] = n_landmarks
    if track is not None:
        cfg["track"] = track
    if n_partitions is not None:
        cfg["n_partitions"] = n_partitions
    if seed is None:
        seed = _CONFIG_SEED[config]
    rng = np.random.Generator(np.random.PCG64(seed))
    m, n = cfg["n_cameras"], cfg["n_landmarks"]

    R, t, d = _make_cameras(rng, m)
    lm = rng.standard_normal((n, 3))
    if cfg["track"] == "fixed8":
        want = np.full(n, 8, np.int64)
    elif cfg["track"] == "geom6":
        want = 1 + rng.geometric(0.2, size=n).astype(np.int64)
    elif cfg["track"].startswith("fixed"):
        want = np.full(n, int(cfg["track"][5:]), np.int64)
    else:
        raise ValueError(cfg["track"])
    want = np.minimum(want, m)

    cam, lmk, uv_clean = _choose_tracks(rng, R, t, d, lm, want)
    k = cam.size
    uv = uv_clean + pixel_sigma * rng.standard_normal((k, 2))
    outl = rng.random(k) < outlier_rate
    n_out = int(outl.sum())
    uv[outl, 0] = rng.uniform(-IMAGE_HALF[0], IMAGE_HALF[0], n_out)
    uv[outl, 1] = rng.uniform(-IMAGE_HALF[1], IMAGE_HALF[1], n_out)

    if shuffle:
        perm = rng.permutation(k)
        cam, lmk, uv, uv_clean, outl = cam[perm], lmk[perm], uv[perm], uv_clean[perm], outl[perm]

    # perturbed initial guess
    axis = _unit_vectors(rng, m)
    R0 = R @ _rotation_exp(rot_perturb * axis)
    t0 = t + trans_perturb * rng.standard_normal((m, 3))
    lm0 = lm + point_perturb * rng.standard_normal((n, 3))

    def pack(Rm, tm, dm):
        return np.ascontiguousarray(np.concatenate([Rm.reshape(-1, 9), tm, dm], axis=1))

    return dict(
        n_cameras=m, n_landmarks=n, n_obs=int(k), n_partitions=cfg["n_partitions"],
        seed=seed, config=config,
        obs_camera=np.ascontiguousarray(cam, dtype=np.int32),
        obs_landmark=np.ascontiguousarray(lmk, dtype=np.int32),
        obs_uv=np.ascontiguousarray(uv, dtype=np.float64),
        obs_uv_clean=np.ascontiguousarray(uv_clean, dtype=np.float64),
        is_outlier=outl,
        cameras=pack(R0, t0, d), landmarks=np.ascontiguousarray(lm0),
        cameras_gt=pack(R, t, d), landmarks_gt=np.ascontiguousarray(lm),
    )


def subproblem(prob: dict, n_cameras: int, n_landmarks: int, seed: int = 0) -> dict:
    """The sub-problem on the first n_cameras cameras and the n_landmarks
    landmarks among those seen most by them (ties by id), keeping every
    observation between the two sets; ids are renumbered densely."""
    cam_keep = np.arange(n_cameras)
    inc = prob["obs_camera"] < n_cameras
    cnt = np.bincount(prob["obs_landmark"][inc], minlength=prob["n_landmarks"])
    order = np.lexsort((np.arange(cnt.size), -cnt))
    lm_keep = np.sort(order[:n_landmarks])
    lm_new = -np.ones(prob["n_landmarks"], np.int64)
    lm_new[lm_keep] = np.arange(lm_keep.size)
    sel = inc & (lm_new[prob["obs_landmark"]] >= 0)
    out = dict(prob)
    out.update(
        n_cameras=n_cameras, n_landmarks=int(lm_keep.size), n_obs=int(sel.sum()),
        obs_camera=np.ascontiguousarray(prob["obs_camera"][sel]),
        obs_landmark=np.ascontiguousarray(lm_new[prob["obs_landmark"][sel]].astype(np.int32)),
        obs_uv=np.ascontiguousarray(prob["obs_uv"][sel]),
        obs_uv_clean=np.ascontiguousarray(prob["obs_uv_clean"][sel]),
        is_outlier=prob["is_outlier"][sel],
        cameras=np.ascontiguousarray(prob["cameras"][cam_keep]),
        cameras_gt=np.ascontiguousarray(prob["cameras_gt"][cam_keep]),
        landmarks=np.ascontiguousarray(prob["landmarks"][lm_keep]),
        landmarks_gt=np.ascontiguousarray(prob["landmarks_gt"][lm_keep]),
    )
    return out
