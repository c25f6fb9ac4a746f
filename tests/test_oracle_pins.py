"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
generator's independent forward camera model, brute force on tiny inputs,
closed forms, library routines (numpy SVD) and the propositions and lemmas
of the paper.  None of these needs a GPU.
"""

import numpy as np
import pytest

from oracle import ALWAYS_RESTART, Oracle, projrot3d
from synth import make_problem

S_UNIT = 512.0


def _exp(w):
    w = np.asarray(w, float)
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K


@pytest.fixture(scope="module")
def small():
    return make_problem("cam50-lm5k", n_landmarks=400, seed=11)


@pytest.fixture(scope="module")
def tiny():
    return make_problem("cam50-lm5k", n_cameras=6, n_landmarks=40, seed=12)


# --------------------------------------------------------------- Sec. III


def test_zero_objective_at_ground_truth_noise_free(small):
    """eq. error: |e| = 0 iff the ray is parallel to the camera-frame point
    (eq. err0).  The generator places pixels with its own inversion of the
    undistortion model, so F(x_gt) = 0 pins the ray, the rotation convention
    and the residual of the oracle."""
    o = Oracle(small, cameras=small["cameras_gt"], landmarks=small["landmarks_gt"], uv=small["obs_uv_clean"],
               loss="trivial")
    F = o.objective()
    assert F < 1e-18 * small["n_obs"], F
    # and not zero once the pixels carry noise
    o2 = Oracle(small, cameras=small["cameras_gt"], landmarks=small["landmarks_gt"], loss="trivial")
    assert o2.objective() > 1.0


def test_residual_is_the_least_squares_projection(tiny):
    """eq. error_opt / eq. lambdaij / eq. error: lambda minimises
    |p - lambda R^T (l - t)|^2 (brute-force scan), e is orthogonal to
    R^T (l - t), |e|^2 = |p x n|^2 for the unit direction n, and |e| <= |p|."""
    o = Oracle(tiny, loss="trivial")
    ci = o.to_internal(tiny["cameras"])
    rng = np.random.default_rng(0)
    for o_id in rng.choice(tiny["n_obs"], 20, replace=False):
        i, j = tiny["obs_camera"][o_id], tiny["obs_landmark"][o_id]
        c, l, u = ci[i], tiny["landmarks"][j], tiny["obs_uv"][o_id] / S_UNIT
        q = o.obs_eval(c, l, u)
        R = c[:9].reshape(3, 3)
        n = R.T @ (l - c[9:12])
        p = q["p"]
        lam_grid = q["lam"] + np.linspace(-1e-3, 1e-3, 2001) * abs(q["lam"])
        vals = [np.sum((p - lg * n) ** 2) for lg in lam_grid]
        assert abs(lam_grid[int(np.argmin(vals))] - q["lam"]) <= 2e-6 * abs(q["lam"])
        assert abs(np.dot(q["e"], n)) <= 1e-12 * np.linalg.norm(n) * np.linalg.norm(p)
        nh = n / np.linalg.norm(n)
        assert np.isclose(q["s"], np.sum(np.cross(p, nh) ** 2), rtol=1e-9, atol=1e-22)
        assert np.linalg.norm(q["e"]) <= np.linalg.norm(p) * (1 + 1e-15)
        # the ray is linear in d and its first two entries are the pixel
        assert np.allclose(p[:2], u, rtol=0, atol=0)


def test_ray_matches_undistortion_model(tiny):
    """eq. ray with d = (f, f k1, f k2) reproduces the undistortion model of
    eq. reprojection1 scaled by f: third entry f (1 + k1 |u|^2 + k2 |u|^4)."""
    o = Oracle(tiny, loss="trivial", unit_scale=1.0)
    c = tiny["cameras"][0].copy()
    f, fk1, fk2 = c[12:15]
    k1, k2 = fk1 / f, fk2 / f
    u = np.array([123.0, -77.0])
    q = o.obs_eval(c, tiny["landmarks"][0], u)
    r2 = u @ u
    assert np.isclose(q["p"][2], f * (1 + k1 * r2 + k2 * r2 * r2), rtol=1e-14)


# --------------------------------------------------------------- losses


@pytest.mark.parametrize("loss", ["trivial", "huber", "welsch"])
def test_loss_assumption_1(tiny, loss):
    """Assumption 1: rho(0)=0, 0 <= rho' <= 1, rho'(0)=1, rho concave; w is
    rho' (finite differences of the oracle's own rho) and a >= 0; the trivial
    loss has w = 1, a = 0, and Huber equals the trivial loss below delta."""
    o = Oracle(tiny, loss=loss, delta=1.0)
    ci = o.to_internal(tiny["cameras"])
    i, j = tiny["obs_camera"][0], tiny["obs_landmark"][0]
    base = o.obs_eval(ci[i], tiny["landmarks"][j], tiny["obs_uv"][0] / S_UNIT)
    # walk the pixel along the residual direction to sweep s = |e|^2
    vals = []
    for t in np.linspace(-4, 4, 161):
        u = tiny["obs_uv"][0] / S_UNIT + t * base["e"][:2] / max(np.linalg.norm(base["e"][:2]), 1e-30) / S_UNIT
        vals.append(o.obs_eval(ci[i], tiny["landmarks"][j], u))
    s = np.array([v["s"] for v in vals])
    rho = np.array([v["rho"] for v in vals])
    w = np.array([v["w"] for v in vals])
    a = np.array([v["a"] for v in vals])
    assert np.all((w >= 0) & (w <= 1 + 1e-15))
    assert np.all(a >= -1e-18)
    order = np.argsort(s)
    s, rho, w = s[order], rho[order], w[order]
    keep = np.concatenate([[True], np.diff(s) > 1e-3 * s.max()])
    s, rho, w = s[keep], rho[keep], w[keep]
    slope = np.diff(rho) / np.diff(s)
    mid_w = 0.5 * (w[1:] + w[:-1])
    assert np.allclose(slope, mid_w, rtol=2e-2, atol=1e-6)
    assert np.all(np.diff(slope) <= 1e-9)  # concave
    if loss == "trivial":
        assert np.all(w == 1.0) and np.all(a == 0.0)
    if loss == "huber":
        dl = 1.0 / S_UNIT
        small_s = s <= dl * dl
        assert np.allclose(rho[small_s], s[small_s], rtol=1e-15)


# --------------------------------------------------------------- Prop. 1


@pytest.mark.parametrize("loss", ["trivial", "huber", "welsch"])
def test_majorizer_prop1(tiny, loss):
    """Prop. 1: F_ij <= P_ij + Q_ij for any (c_i, l_j), with equality at y;
    at y P = Q = F/2 and |R p + lambda t - g| = |e| / 2 (eq. approx0)."""
    o = Oracle(tiny, loss=loss, delta=1.0)
    ci = o.to_internal(tiny["cameras"])
    rng = np.random.default_rng(1)
    for o_id in rng.choice(tiny["n_obs"], 25, replace=False):
        i, j = tiny["obs_camera"][o_id], tiny["obs_landmark"][o_id]
        cy, ly, u = ci[i], tiny["landmarks"][j], tiny["obs_uv"][o_id] / S_UNIT
        qy = o.obs_eval(cy, ly, u)
        P, Q = o.PQ(u, cy, ly, cy, ly)
        assert np.isclose(P + Q, qy["F"], rtol=1e-9, atol=1e-20)
        assert np.isclose(P, qy["F"] / 2, rtol=1e-8, atol=1e-20)
        assert np.isclose(Q, qy["F"] / 2, rtol=1e-8, atol=1e-20)
        R = cy[:9].reshape(3, 3)
        v = R @ qy["p"] + qy["lam"] * cy[9:12] - qy["g"]
        assert np.isclose(np.linalg.norm(v), 0.5 * np.sqrt(qy["s"]), rtol=1e-7, atol=1e-16)
        for scale in (1e-3, 1e-2, 0.1, 0.5):
            c = cy.copy()
            c[:9] = (R @ _exp(scale * rng.standard_normal(3))).reshape(9)
            c[9:12] += scale * rng.standard_normal(3)
            c[12:15] *= 1 + scale * 0.1 * rng.standard_normal(3)
            l = ly + scale * rng.standard_normal(3)
            q = o.obs_eval(c, l, u)
            P, Q = o.PQ(u, cy, ly, c, l)
            assert q["F"] <= P + Q + 1e-15 * (P + Q) + 1e-22


# --------------------------------------------------------------- gradients


def _fd_objective(o, cams, lms, uv, which, idx, h):
    def f(delta):
        c, l, u = cams.copy(), lms.copy(), uv.copy()
        arr = {"c": c, "l": l, "u": u}[which]
        arr.reshape(-1)[idx] += delta
        return o.objective(c, l, u)
    return (f(h) - f(-h)) / (2 * h)


@pytest.mark.parametrize("loss", ["trivial", "huber"])
def test_gradient_vs_central_differences(tiny, loss):
    """App. D, eq. DFij (intrinsics row transposed back) and the pixel
    gradient, against central differences of the oracle objective."""
    o = Oracle(tiny, loss=loss, delta=1.0)
    cams, lms, uv = tiny["cameras"].copy(), tiny["landmarks"].copy(), tiny["obs_uv"].copy()
    gc, gl, gu = o.grad()
    rng = np.random.default_rng(2)
    # rotation entries, translation, landmarks: h = 1e-6 (world units)
    for i in rng.choice(tiny["n_cameras"], 3, replace=False):
        for k in list(range(12)):
            fd = _fd_objective(o, cams, lms, uv, "c", 15 * i + k, 1e-6)
            assert np.isclose(fd, gc[i, k], rtol=2e-5, atol=1e-4 * np.abs(gc[i, :12]).max()), (i, k)
        # intrinsics: h = 1e-6 in the well-scaled coordinates (f/f0, kappa1,
        # kappa2) with d = (f, kappa1/f, kappa2/f^3), f0 = 500 px
        f0 = cams[i, 12]
        for k, h in zip(range(12, 15), (1e-6 * f0, 1e-6 / f0, 1e-6 / f0 ** 3)):
            fd = _fd_objective(o, cams, lms, uv, "c", 15 * i + k, h)
            assert np.isclose(fd, gc[i, k], rtol=1e-4, atol=1e-6 * abs(gc[i, k]) + 1e-12), (i, k)
    for j in rng.choice(tiny["n_landmarks"], 4, replace=False):
        for k in range(3):
            fd = _fd_objective(o, cams, lms, uv, "l", 3 * j + k, 1e-6)
            assert np.isclose(fd, gl[j, k], rtol=2e-5, atol=1e-4 * np.abs(gl[j]).max()), (j, k)
    for q in rng.choice(tiny["n_obs"], 6, replace=False):
        for k in range(2):
            fd = _fd_objective(o, cams, lms, uv, "u", 2 * q + k, 1e-4)
            assert np.isclose(fd, gu[q, k], rtol=2e-5, atol=1e-6 * np.abs(gu[q]).max() + 1e-9), (q, k)


def test_surrogate_gradient_touches_objective(tiny):
    """eq. gradFij: the surrogate P + Q has the objective's Riemannian
    gradient at the touching point: directional derivatives along R Exp(.)
    and along t, d, l agree."""
    o = Oracle(tiny, loss="huber", delta=1.0)
    ci = o.to_internal(tiny["cameras"])
    rng = np.random.default_rng(3)
    for o_id in rng.choice(tiny["n_obs"], 8, replace=False):
        i, j = tiny["obs_camera"][o_id], tiny["obs_landmark"][o_id]
        cy, ly, u = ci[i], tiny["landmarks"][j], tiny["obs_uv"][o_id] / S_UNIT
        R = cy[:9].reshape(3, 3)
        for _ in range(3):
            dth, dt, dd, dl = (rng.standard_normal(3) for _ in range(4))
            dd *= np.array([1.0, 0.1, 0.1])

            def at(h):
                c = cy.copy()
                c[:9] = (R @ _exp(h * dth)).reshape(9)
                c[9:12] += h * dt
                c[12:15] += h * dd
                return c, ly + h * dl

            h = 1e-6
            cp, lp = at(h)
            cm, lm_ = at(-h)
            dF = (o.obs_eval(cp, lp, u)["F"] - o.obs_eval(cm, lm_, u)["F"]) / (2 * h)
            dE = (sum(o.PQ(u, cy, ly, cp, lp)) - sum(o.PQ(u, cy, ly, cm, lm_))) / (2 * h)
            assert np.isclose(dF, dE, rtol=1e-5, atol=1e-12), (dF, dE)


# --------------------------------------------------------------- minimizers


def test_landmark_minimizer(tiny):
    """The landmark closed form zeroes the gradient of sum Q + prox and no
    coordinate move decreases it."""
    o = Oracle(tiny, loss="huber", delta=1.0, xi=1e-3)
    ci = o.to_internal(tiny["cameras"])
    lms = tiny["landmarks"]
    for j in range(0, tiny["n_landmarks"], 7):
        l = o.landmark_min(j, ci, lms)
        phi0 = o.landmark_phi(j, ci, lms, l)
        for k in range(3):
            for h in (1e-5, 1e-3):
                e = np.zeros(3)
                e[k] = h
                assert o.landmark_phi(j, ci, lms, l + e) >= phi0 - 1e-16 * abs(phi0)
                assert o.landmark_phi(j, ci, lms, l - e) >= phi0 - 1e-16 * abs(phi0)
            e = np.zeros(3)
            e[k] = 1e-6
            g = (o.landmark_phi(j, ci, lms, l + e) - o.landmark_phi(j, ci, lms, l - e)) / 2e-6
            assert abs(g) <= 1e-6 * (1 + abs(phi0)) + 1e-9


def test_camera_minimizer_converged_is_stationary(tiny):
    """Assumption 4 realised by the converged LM mode: along every tangent
    direction of SO(3) x R^3 x R^3 the surrogate does not decrease and its
    central-difference gradient vanishes."""
    o = Oracle(tiny, loss="huber", delta=1.0, xi=1e-6)
    ci = o.to_internal(tiny["cameras"])
    lms = tiny["landmarks"]
    for i in range(tiny["n_cameras"]):
        c, ns = o.camera_min(i, ci, lms, inner_steps=0)
        assert ns >= 1
        phi0 = o.camera_phi(i, ci, lms, c)
        phi_y = o.camera_phi(i, ci, lms, ci[i])
        assert phi0 < phi_y
        R = c[:9].reshape(3, 3)
        for k in range(9):
            def move(h):
                cc = c.copy()
                if k < 3:
                    e = np.zeros(3)
                    e[k] = h
                    cc[:9] = (R @ _exp(e)).reshape(9)
                else:
                    cc[9 + k - 3] += h
                return o.camera_phi(i, ci, lms, cc)
            for h in (1e-4, -1e-4):
                assert move(h) >= phi0 - 1e-12 * abs(phi0)
            g = (move(1e-6) - move(-1e-6)) / 2e-6
            # gradient is tiny compared with its size at the start point
            assert abs(g) <= 1e-4 * phi_y + 1e-12


def test_camera_one_step_decreases(tiny):
    """One successful inner LM step strictly decreases the camera surrogate."""
    o = Oracle(tiny, loss="huber", delta=1.0)
    ci = o.to_internal(tiny["cameras"])
    for i in range(tiny["n_cameras"]):
        c, ns = o.camera_min(i, ci, tiny["landmarks"], inner_steps=1)
        assert ns == 1
        assert o.camera_phi(i, ci, tiny["landmarks"], c) < o.camera_phi(i, ci, tiny["landmarks"], ci[i])
        R = c[:9].reshape(3, 3)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14) and np.isclose(np.linalg.det(R), 1.0, atol=1e-14)


# --------------------------------------------------------------- ProjRot3D


def _umeyama_numpy(M):
    U, _, Vt = np.linalg.svd(M)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
    return U @ D @ Vt


def test_projrot3d_matches_library_svd():
    """eq. proj_rot3d: equals the numpy-SVD closed form, fixes rotations, is
    invariant to positive scaling and handles det(M) < 0."""
    rng = np.random.default_rng(4)
    for trial in range(200):
        M = rng.standard_normal((3, 3))
        if trial % 3 == 0:
            M = _exp(rng.standard_normal(3)) + 0.05 * rng.standard_normal((3, 3))
        R = projrot3d(M)
        assert np.allclose(R, _umeyama_numpy(M), atol=1e-10)
        assert np.isclose(np.linalg.det(R), 1.0)
        assert np.allclose(projrot3d(3.7 * M), R, atol=1e-10)
        Q = _exp(rng.standard_normal(3))
        assert np.allclose(projrot3d(Q), Q, atol=1e-14)
        # brute-force optimality against nearby rotations
        best = np.sum((R - M) ** 2)
        for _ in range(5):
            R2 = R @ _exp(1e-3 * rng.standard_normal(3))
            assert np.sum((R2 - M) ** 2) >= best - 1e-12


# --------------------------------------------------------------- Sec. V


def test_nesterov_scalars(tiny):
    """eq. nesterov_scalar: s(0) = 1, s(1) = golden ratio, s(k) ~ (k+2)/2;
    gamma(0) = 0, so the first accelerated step equals the MM step."""
    o = Oracle(tiny, loss="huber")
    assert o.get_state()["s"] == 1.0
    o.iterate(1)
    assert np.isclose(o.get_state()["s"], (1 + 5 ** 0.5) / 2, rtol=1e-15)
    o.iterate(99)
    st = o.get_state()
    assert st["k"] == 100
    assert abs(st["s"] - 51.0) < np.log(100)
    a = Oracle(tiny, loss="huber")
    b = Oracle(tiny, loss="huber", accelerate=False)
    a.iterate(1)
    b.iterate(1)
    # equal up to the rounding of projecting an exact rotation onto SO(3)
    assert np.allclose(a.get_state()["cams"], b.get_state()["cams"], rtol=1e-12, atol=1e-13)
    assert np.allclose(a.get_state()["lms"], b.get_state()["lms"], rtol=0, atol=1e-12)


# gamma^(k) for k = 0..3, worked by hand from eq. nesterov_scalar
# (s^(0) = 1, s^(k) = (sqrt(4 s^(k-1)^2 + 1) + 1) / 2, gamma^(k) = (s^(k) - 1) / s^(k+1)):
# s = 1, 1.618034, 2.193527, 2.749791, 3.294881 to six places.
GAMMA_0_3 = (0.0, 0.281754, 0.434043, 0.531064)


def test_nesterov_gamma_sequence(tiny):
    """eq. nesterov_scalar: gamma^(0..3) = 0, 0.281754, 0.434043, 0.531064 on
    every partition; eq. gamma_bnd: 0 <= gamma^(k) <= (s^(k) - 1) / s^(k) < 1;
    without acceleration gamma = 0."""
    o = Oracle(tiny, loss="huber", n_partitions=2)
    for k, want in enumerate(GAMMA_0_3):
        g, _, _ = o.extrapolation()
        assert g.shape == (2,)
        assert np.all(np.abs(g - want) <= 5e-7), (k, g, want)
        o.iterate(1)
    for _ in range(40):
        g, _, _ = o.extrapolation()
        s = o.get_state()["s"]
        assert np.all((g >= 0) & (g <= (s - 1) / s + 1e-15) & (g < 1))
        o.iterate(1)
    d = Oracle(tiny, loss="huber", accelerate=False)
    d.iterate(3)
    assert np.all(d.extrapolation()[0] == 0.0)


def test_nesterov_extrapolation_by_hand(tiny):
    """eq. nesterov_x with eq. proj_rot3d, computed here from the oracle's
    x^k and x^(k-1) at k = 3: R-bar = numpy-SVD projection of
    R + gamma (R - R^(k-1)); t, d and l extrapolated linearly (d in caller
    units: the unit conversion is linear per component)."""
    o = Oracle(tiny, loss="huber", n_partitions=2)
    o.iterate(3)
    st = o.get_state()
    g, cb, lb = o.extrapolation()
    gam = GAMMA_0_3[3]
    assert np.allclose(g, gam, atol=5e-7)
    gam = float(g[0])
    c, cp = st["cams"], st["cams_prev"]
    # the iterates have moved, so a sign or factor mistake shows
    assert np.max(np.abs(c[:, :9] - cp[:, :9])) > 1e-5 and np.max(np.abs(st["lms"] - st["lms_prev"])) > 1e-5
    for i in range(c.shape[0]):
        R, Rp = c[i, :9].reshape(3, 3), cp[i, :9].reshape(3, 3)
        assert np.allclose(cb[i, :9], _umeyama_numpy(R + gam * (R - Rp)).ravel(), rtol=0, atol=2e-14)
        want = c[i, 9:] + gam * (c[i, 9:] - cp[i, 9:])
        assert np.allclose(cb[i, 9:], want, rtol=1e-14, atol=1e-15)
    want = st["lms"] + gam * (st["lms"] - st["lms_prev"])
    assert np.allclose(lb, want, rtol=1e-14, atol=1e-15)
    # the probe changes nothing: the next iteration is the one without it
    a = Oracle(tiny, loss="huber", n_partitions=2)
    a.iterate(3)
    assert np.array_equal(o.iterate(2)[0], a.iterate(2)[0])


# Textbook closed forms with delta = 1 px, at |e| = 0.5, 1 and 3 px:
# Huber   rho(s) = s (|e| <= delta), 2 delta |e| - delta^2 (above); w = rho'(s) = 1 or delta / |e|;
# Welsch  rho(s) = delta^2 (1 - exp(-s / delta^2)); w = exp(-s / delta^2).
LOSS_CLOSED_FORMS = {
    "huber": {0.5: (0.25, 1.0), 1.0: (1.0, 1.0), 3.0: (5.0, 1.0 / 3.0)},
    "welsch": {0.5: (0.22119921692859512, 0.7788007830714049),
               1.0: (0.6321205588285577, 0.36787944117144233),
               3.0: (0.9998765901959134, 1.2340980408667956e-4)},
}


@pytest.mark.parametrize("unit_scale", [512.0, 1.0])
@pytest.mark.parametrize("loss", ["huber", "welsch"])
def test_loss_closed_forms_in_pixels(loss, unit_scale):
    """Assumption 1 with readings R7 and R9: rho and w of Huber and Welsch
    at |e| = 0.5, 1 and 3 px for delta = 1 px, through the objective (F in
    px^2 = sum rho / 2, eq. Fij) and through one observation's evaluation in
    internal units, at two unit scales (delta becomes delta / s inside).  A
    camera at the origin looking down +z with f = 500 px sees a point on its
    axis; the pixel (|e|, 0) then has residual exactly |e| px."""
    errs = sorted(LOSS_CLOSED_FORMS[loss])
    prob = dict(n_cameras=1, n_landmarks=len(errs), n_obs=len(errs),
                obs_camera=np.zeros(len(errs), np.int32), obs_landmark=np.arange(len(errs), dtype=np.int32),
                obs_uv=np.array([[e, 0.0] for e in errs]),
                cameras=np.concatenate([np.eye(3).ravel(), np.zeros(3), [500.0, 0.0, 0.0]])[None, :],
                landmarks=np.tile([0.0, 0.0, 10.0], (len(errs), 1)))
    o = Oracle(prob, loss=loss, delta=1.0, unit_scale=unit_scale)
    want_rho = np.array([LOSS_CLOSED_FORMS[loss][e][0] for e in errs])
    want_w = np.array([LOSS_CLOSED_FORMS[loss][e][1] for e in errs])
    assert np.isclose(o.objective(), 0.5 * want_rho.sum(), rtol=1e-13, atol=0)
    ci = o.to_internal(prob["cameras"])[0]
    for q, e in enumerate(errs):
        v = o.obs_eval(ci, prob["landmarks"][q], prob["obs_uv"][q] / unit_scale)
        assert np.isclose(np.sqrt(v["s"]) * unit_scale, e, rtol=1e-14)
        assert np.isclose(v["rho"] * unit_scale ** 2, want_rho[q], rtol=1e-13, atol=0), (loss, e)
        assert np.isclose(v["w"], want_w[q], rtol=1e-13, atol=0), (loss, e)
        assert np.isclose(v["F"] * unit_scale ** 2, 0.5 * want_rho[q], rtol=1e-13, atol=0)


def test_mm_monotone_without_acceleration(small):
    """Sec. IV: F(x^{k+1}) <= E(x^{k+1} | x^k) <= E(x^k | x^k) = F(x^k)."""
    o = Oracle(small, loss="huber", accelerate=False, n_partitions=3)
    F_prev = o.objective()
    for _ in range(12):
        st0 = o.get_state()
        o.iterate(1)
        st1 = o.get_state()
        E_next, _ = o.surrogate(st1["cams"], st1["lms"], st0["cams"], st0["lms"])
        E_cur, _ = o.surrogate(st0["cams"], st0["lms"], st0["cams"], st0["lms"])
        F = o.objective()
        assert np.isclose(E_cur.sum(), F_prev, rtol=1e-10)
        assert F <= E_next.sum() * (1 + 1e-12)
        assert E_next.sum() <= E_cur.sum() * (1 + 1e-12)
        F_prev = F


@pytest.mark.parametrize("eta", [0.5, 1.0])
def test_restart_metrics_lemma2(small, eta):
    """Lemma 2 and the induction of App. C.3: sum_a F^a(k) = F(x^k);
    sum_a Fbar^a(k) follows the exponential average of F; F^a(k) <= E^a(k);
    F^a(k) <= Fbar^a(k) <= Fbar^a(k-1)."""
    o = Oracle(small, loss="huber", n_partitions=5, eta=eta)
    F0 = o.objective()
    F, mt = o.iterate(40)
    Fx = np.concatenate([[F0], F])  # F(x^k), k = 0..40
    assert np.allclose(mt[:, :, 0].sum(1), Fx[:-1], rtol=1e-9)
    Fbar = F0
    for k in range(40):
        Fbar = (1 - eta) * Fbar + eta * Fx[k]
        assert np.isclose(mt[k, :, 1].sum(), Fbar, rtol=1e-9)
    E_k = np.concatenate([mt[:1, :, 0], mt[:-1, :, 2]])  # E^a(k): E^a(0) = F^a(-1) = F^a(0)
    tol = 1e-9 * F0
    assert np.all(mt[:, :, 0] <= E_k + tol)
    assert np.all(mt[:, :, 0] <= mt[:, :, 1] + tol)
    assert np.all(np.diff(mt[:, :, 1], axis=0) <= tol)
    assert np.all(np.diff(Fx) <= 0.05 * Fx[:-1])  # F itself may rise slightly; Fbar may not
    assert mt[:, :, 3].sum() > 0  # the run exercises the restart branch


def test_restart_triggers_and_falls_back(small):
    """Forcing the restart on every iteration reproduces the MM (DUBA)
    iterates exactly; with eta = 1 restarts occur in the free run and the
    metrics invariants still hold."""
    a = Oracle(small, loss="huber", n_partitions=2, flags=ALWAYS_RESTART)
    b = Oracle(small, loss="huber", n_partitions=2, accelerate=False)
    Fa, _ = a.iterate(8)
    Fb, _ = b.iterate(8)
    assert np.array_equal(Fa, Fb)


def test_duba_independent_of_partitions(small):
    """With every observation majorized, the MM iterates do not depend on
    how cameras and landmarks are split into partitions."""
    a = Oracle(small, loss="huber", accelerate=False, n_partitions=1)
    rng = np.random.default_rng(5)
    b = Oracle(small, loss="huber", accelerate=False, n_partitions=6,
               cam_part=rng.integers(0, 6, small["n_cameras"]), lm_part=rng.integers(0, 6, small["n_landmarks"]))
    Fa, _ = a.iterate(10)
    Fb, _ = b.iterate(10)
    assert np.allclose(Fa, Fb, rtol=1e-12)
    assert np.allclose(a.get_state()["lms"], b.get_state()["lms"], rtol=0, atol=1e-12)


def test_frozen_partition_keeps_guarantees(small):
    """A stalled device (its variables frozen) still satisfies
    E^a(x^{k+1} | x^k) <= E^a(x^k | x^k), so the MM objective stays
    monotone and Lemma 2 still holds."""
    o = Oracle(small, loss="huber", accelerate=False, n_partitions=4, frozen_partition=2)
    st0 = o.get_state()
    F0 = o.objective()
    F, mt = o.iterate(10)
    assert np.all(np.diff(np.concatenate([[F0], F])) <= 1e-12 * F0)
    st = o.get_state()
    blk = -(-small["n_cameras"] // 4)
    frozen = np.arange(small["n_cameras"]) // blk == 2
    assert np.array_equal(st["cams"][frozen], st0["cams"][frozen])
    assert np.allclose(mt[:, :, 0].sum(1), np.concatenate([[F0], F[:-1]]), rtol=1e-9)


def test_state_roundtrip_resumes_identically(small):
    """Checkpoint at k, restore into a fresh oracle, continue: identical to an
    uninterrupted run."""
    a = Oracle(small, loss="huber", n_partitions=3)
    a.iterate(5)
    st = a.get_state()
    Fa, _ = a.iterate(5)
    b = Oracle(small, loss="huber", n_partitions=3)
    b.set_state(st)
    Fb, _ = b.iterate(5)
    assert np.array_equal(Fa, Fb)
