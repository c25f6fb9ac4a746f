"""Pins of the partition-level oracle (oracle/partition.py) against what the
paper and the mathematics fix, independently of its own formulas:

- Jacobians against central finite differences on the manifold;
- the model gradient against finite differences of E^a;
- eq. Ealpha + eq. DEalpha summing to F of the C oracle (independent code);
- Prop. 2 (majorization, equality at x = y);
- with every pair split between devices, E^a and DeltaE^a equal the entity
  surrogate of the C oracle;
- with one device nothing is majorized: the iteration is LM on full bundle
  adjustment and drives a noise-free problem to zero residual;
- MM descent without acceleration, and sum_a F^a(k) = F(x^k) (eq. Fak).
"""

import numpy as np
import pytest

import oracle as O
from oracle.partition import PartOracle, so3_exp
from synth import make_problem


@pytest.fixture(scope="module")
def prob():
    return make_problem("cam50-lm5k", seed=7, n_cameras=12, n_landmarks=150)


def _perturbed(prob, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    c = prob["cameras"].copy()
    R = c[:, :9].reshape(-1, 3, 3) @ so3_exp(0.02 * scale * rng.standard_normal((c.shape[0], 3)))
    c[:, :9] = R.reshape(-1, 9)
    c[:, 9:12] += 0.05 * scale * rng.standard_normal((c.shape[0], 3))
    c[:, 12] *= 1 + 0.01 * scale * rng.standard_normal(c.shape[0])
    c[:, 13:15] += 1e-9 * scale * rng.standard_normal((c.shape[0], 2))
    l = prob["landmarks"] + 0.05 * scale * rng.standard_normal(prob["landmarks"].shape)
    return c, l


def _state(po, c, l):
    return (*po._cams_in(c), l.copy())


def test_residual_jacobian_matches_finite_differences(prob):
    po = PartOracle(prob, n_partitions=3, loss="trivial")
    x = po.x
    sel = np.arange(0, po.K, max(1, po.K // 25))
    _, Jc, Jl = po.residual_jacobian(x, sel)
    h = 1e-6
    for k, o in enumerate(sel):
        i, j = po.cam[o], po.lmk[o]
        num = np.zeros((3, 12))
        for c in range(12):
            xs = []
            for sg in (1.0, -1.0):
                R, t, d, l = (a.copy() for a in x)
                dv = np.zeros(12)
                dv[c] = sg * h
                R[i] = R[i] @ so3_exp(dv[0:3])
                t[i] += dv[3:6]
                d[i] += dv[6:9]
                l[j] += dv[9:12]
                xs.append(po.obs((R, t, d, l), np.array([o]))["e"][0])
            num[:, c] = (xs[0] - xs[1]) / (2 * h)
        ana = np.concatenate([Jc[k], Jl[k]], axis=1)
        np.testing.assert_allclose(ana, num, rtol=1e-5, atol=1e-7 * np.abs(ana).max())


def test_P_jacobian_matches_finite_differences(prob):
    po = PartOracle(prob, n_partitions=3, loss="huber")
    c, l = _perturbed(prob, 1)
    x = _state(po, c, l)
    lin = po.linearize(po.x)
    sel = np.arange(3, po.K, max(1, po.K // 20))
    r0, J = po.P_jacobian(lin, x, sel)
    h = 1e-6
    for k, o in enumerate(sel):
        i = po.cam[o]
        num = np.zeros((3, 9))
        for cc in range(9):
            vals = []
            for sg in (1.0, -1.0):
                R, t, d, lm = (a.copy() for a in x)
                dv = np.zeros(9)
                dv[cc] = sg * h
                R[i] = R[i] @ so3_exp(dv[0:3])
                t[i] += dv[3:6]
                d[i] += dv[6:9]
                vals.append(po.P_jacobian(lin, (R, t, d, lm), np.array([o]))[0][0])
            num[:, cc] = (vals[0] - vals[1]) / (2 * h)
        np.testing.assert_allclose(J[k], num, rtol=1e-5, atol=1e-7 * np.abs(J[k]).max())


def test_surrogate_and_gap_sum_to_the_objective(prob):
    """eq. Ealpha and eq. DEalpha: sum_a E^a(x | y) + DeltaE^a(x | y) = F(x),
    with F from the C oracle."""
    po = PartOracle(prob, n_partitions=3, loss="huber", xi=0.5)
    cy, ly = _perturbed(prob, 2)
    cx, lx = _perturbed(prob, 3)
    y, x = _state(po, cy, ly), _state(po, cx, lx)
    lin = po.linearize(y)
    tot = np.sum(po.surrogate(x, y, lin) + po.gap(x, y, lin)) * po.s_unit ** 2
    F = O.Oracle(prob, n_partitions=1, loss="huber").objective(cx, lx)
    assert tot == pytest.approx(F, rel=1e-12)
    assert po.objective(x) == pytest.approx(F, rel=1e-12)


def test_majorization_prop2(prob):
    po = PartOracle(prob, n_partitions=4, loss="huber", xi=1e-9)
    cy, ly = _perturbed(prob, 4)
    y = _state(po, cy, ly)
    lin = po.linearize(y)
    F_y = po.objective(y) / po.s_unit ** 2
    assert np.sum(po.surrogate(y, y, lin)) == pytest.approx(F_y, rel=1e-12)
    for s in range(5):
        cx, lx = _perturbed({**prob, "cameras": cy, "landmarks": ly}, 10 + s, scale=0.5)
        x = _state(po, cx, lx)
        assert po.objective(x) / po.s_unit ** 2 <= np.sum(po.surrogate(x, y, lin)) * (1 + 1e-12)


def test_every_pair_split_reduces_to_entity_surrogate(prob):
    """Each camera its own device and every landmark on a device none of its
    cameras is on: E' is empty and E^a, DeltaE^a are the entity surrogate's."""
    M = prob["n_cameras"]
    seen = np.zeros((prob["n_landmarks"], M), bool)
    seen[prob["obs_landmark"], prob["obs_camera"]] = True
    assert not seen.all(axis=1).any()
    lm_part = np.argmin(seen, axis=1).astype(np.int32)  # first device that does not observe j
    cam_part = np.arange(M, dtype=np.int32)
    po = PartOracle(prob, n_partitions=M, cam_part=cam_part, lm_part=lm_part, loss="huber", xi=0.3)
    assert not po.intra.any()
    orc = O.Oracle(prob, n_partitions=M, cam_part=cam_part, lm_part=lm_part, loss="huber", xi=0.3)
    cy, ly = _perturbed(prob, 5)
    cx, lx = _perturbed(prob, 6)
    E_ent, dE_ent = orc.surrogate(cx, lx, cy, ly)
    y, x = _state(po, cy, ly), _state(po, cx, lx)
    lin = po.linearize(y)
    s2 = po.s_unit ** 2
    np.testing.assert_allclose(po.surrogate(x, y, lin) * s2, E_ent, rtol=1e-11, atol=1e-9 * np.abs(E_ent).max())
    np.testing.assert_allclose(po.gap(x, y, lin) * s2, dE_ent, rtol=1e-9, atol=1e-9 * np.abs(E_ent).max())


def test_model_gradient_matches_finite_differences(prob):
    po = PartOracle(prob, n_partitions=3, loss="huber", xi=0.3)
    cy, ly = _perturbed(prob, 7)
    cx, lx = _perturbed({**prob, "cameras": cy, "landmarks": ly}, 8, scale=0.3)
    y, x = _state(po, cy, ly), _state(po, cx, lx)
    lin = po.linearize(y)
    a = 1
    H, g, cams, lms = po.system(a, x, y, lin)
    assert np.allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())
    n = g.size
    rng = np.random.default_rng(0)
    lm_coords = np.arange(9 * cams.size, n)
    assert lm_coords.size > 0
    idx = np.concatenate([np.arange(9 * cams.size), rng.choice(lm_coords, min(12, lm_coords.size), replace=False)])
    for c in idx:
        h = 1e-6
        dv = np.zeros(n)
        dv[c] = h
        Ep = po.surrogate(po.retract(x, cams, lms, dv), y, lin)[a]
        Em = po.surrogate(po.retract(x, cams, lms, -dv), y, lin)[a]
        num = (Ep - Em) / (2 * h)
        assert num == pytest.approx(g[c], rel=2e-5, abs=1e-6 * np.abs(g).max()), c


def test_one_device_is_full_bundle_adjustment(prob):
    """S = 1: no pair is majorized, so each iteration is one successful LM
    step on F (plus a vanishing prox); noise-free data converge to zero."""
    clean = dict(prob, obs_uv=prob["obs_uv_clean"])
    po = PartOracle(clean, n_partitions=1, loss="trivial", accelerate=False, xi=1e-12)
    assert po.intra.all()
    F0 = po.objective()
    F, _ = po.iterate(25)
    assert np.all(np.diff(F) <= 1e-12 * F0)
    assert F[-1] < 1e-12 * F0


def test_mm_descent_and_partition_metrics_sum_to_F(prob):
    po = PartOracle(prob, n_partitions=3, loss="huber", accelerate=False)
    F0 = po.objective()
    F, mt = po.iterate(8)
    Fs = np.concatenate([[F0], F])
    assert np.all(np.diff(Fs) <= 1e-12 * F0)
    np.testing.assert_allclose(mt[:, :, 0].sum(axis=1), Fs[:-1], rtol=1e-11)
    assert np.all(mt[:, :, 3] == 1)


def test_daba_bookkeeping_and_restart_flags(prob):
    po = PartOracle(prob, n_partitions=3, loss="huber", accelerate=True)
    F0 = po.objective()
    F, mt = po.iterate(10)
    Fs = np.concatenate([[F0], F])
    np.testing.assert_allclose(mt[:, :, 0].sum(axis=1), Fs[:-1], rtol=1e-11)
    assert F[-1] < F0
    never = PartOracle(prob, n_partitions=3, loss="huber", flags=1)
    assert not never.iterate(3)[1][:, :, 3].any()
    always = PartOracle(prob, n_partitions=3, loss="huber", flags=2)
    duba = PartOracle(prob, n_partitions=3, loss="huber", accelerate=False)
    np.testing.assert_allclose(always.iterate(3)[0], duba.iterate(3)[0], rtol=1e-12)


def test_converged_lm_with_every_pair_split_matches_entity_minimizers(prob):
    """With E' empty, E^a is a sum of independent camera and landmark terms;
    LM run to convergence must reach the landmark closed form and the
    converged camera solve of the C oracle."""
    M = prob["n_cameras"]
    seen = np.zeros((prob["n_landmarks"], M), bool)
    seen[prob["obs_landmark"], prob["obs_camera"]] = True
    lm_part = np.argmin(seen, axis=1).astype(np.int32)
    cam_part = np.arange(M, dtype=np.int32)
    kw = dict(n_partitions=M, cam_part=cam_part, lm_part=lm_part, loss="huber", xi=0.3)
    po = PartOracle(prob, inner_steps=60, **kw)
    orc = O.Oracle(prob, **kw)
    cy, ly = _perturbed(prob, 9)
    y = _state(po, cy, ly)
    lin = po.linearize(y)
    cy_int = orc.to_internal(cy)  # the C oracle's probes work in internal units
    for a in (0, 5):
        xa, succ = po.lm_partition(a, y, lin)
        assert succ >= 3
        cams, lms = po.unknowns(a)
        c_int = np.concatenate([xa[0][cams].reshape(-1, 9), xa[1][cams], xa[2][cams]], axis=1)
        for k, i in enumerate(cams):
            ref, _ = orc.camera_min(int(i), cy_int, ly, inner_steps=0)
            # both solves stop at the rounding floor of a flat minimum: ~sqrt(eps) in x
            np.testing.assert_allclose(c_int[k], ref, rtol=1e-6, atol=1e-8)
        for j in lms[:20]:
            np.testing.assert_allclose(xa[3][j], orc.landmark_min(int(j), cy_int, ly), rtol=1e-9, atol=1e-10)
