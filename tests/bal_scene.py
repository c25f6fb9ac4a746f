"""A scene drawn in BAL's own convention (P = R(w) X + t, p = -P_xy / P_z,
u = f (1 + k1 |p|^2 + k2 |p|^4) p): cameras on a sphere looking at the
origin, points ~ N(0, I), every point observed by each camera that sees it
in front and inside a 640 x 480 image (so track lengths vary).  Shared by the
BAL reader's tests and the GPU run of a converted scene."""

import numpy as np

from paper_2305_07026_amd import bal


def scene(rng, M=6, N=400, k_sigma=0.05):
    # cameras on a sphere of radius 8 looking at the origin, BAL convention:
    # the camera looks down its -z axis
    C = rng.standard_normal((M, 3))
    C = 8.0 * C / np.linalg.norm(C, axis=1, keepdims=True)
    w = []
    for c in C:
        back = c / np.linalg.norm(c)  # BAL +z points away from the scene
        a = rng.standard_normal(3)
        x = a - a.dot(back) * back
        x /= np.linalg.norm(x)
        y = np.cross(back, x)
        Rb = np.stack([x, y, back])  # rows: camera axes in world coordinates
        # Rodrigues vector of Rb
        th = np.arccos(np.clip((np.trace(Rb) - 1) / 2, -1, 1))
        v = np.array([Rb[2, 1] - Rb[1, 2], Rb[0, 2] - Rb[2, 0], Rb[1, 0] - Rb[0, 1]])
        w.append(v / (2 * np.sin(th)) * th)
    w = np.array(w)
    Rb = bal.rodrigues(w)
    tb = -np.einsum("nij,nj->ni", Rb, C)
    f = rng.uniform(400, 600, M)
    k = rng.normal(0, k_sigma, (M, 2))
    X = rng.standard_normal((N, 3))
    ci, pi, xy = [], [], []
    for i in range(M):
        P = X @ Rb[i].T + tb[i]
        p = -P[:, :2] / P[:, 2:3]
        r2 = np.sum(p * p, axis=1)
        u = f[i] * (1 + k[i, 0] * r2 + k[i, 1] * r2 * r2)[:, None] * p
        ok = (P[:, 2] < -0.5) & (np.abs(u[:, 0]) < 320) & (np.abs(u[:, 1]) < 240)
        ci.append(np.full(ok.sum(), i)), pi.append(np.nonzero(ok)[0]), xy.append(u[ok])
    raw = dict(obs_camera=np.concatenate(ci), obs_point=np.concatenate(pi), obs_xy=np.concatenate(xy),
               cameras=np.concatenate([w, tb, f[:, None], k], axis=1), points=X)
    return raw
