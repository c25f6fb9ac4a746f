"""GPU (gfx950) path against the CPU oracle, element by element, on the same
seeded inputs, through the C ABI.

Tolerances: the FP64 path matches the oracle's objective to 1e-10 relative
after every iteration (the requirement for this path); single evaluations
(objective, gradient, one iteration from a common state) agree to rounding,
checked at 1e-12 / 1e-10.  The FP32-mixed path matches the FP64 oracle to
1e-4 relative after 100 iterations.
"""

import numpy as np
import pytest

from compare import assert_state_close, state_errs
from oracle import ALWAYS_RESTART, Oracle
from synth import make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_2305_07026_amd")


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def nrel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c1():
    # the small configuration: 50 cameras, 5000 landmarks, ~40k observations
    return make_problem("cam50-lm5k")


@pytest.fixture(scope="module")
def tiled():
    # few cameras with many observations each (several tiles per camera and a
    # ragged tail) and geometric track lengths (many landmark groups)
    return make_problem("cam50-lm5k", n_cameras=7, n_landmarks=2500, track="geom6", seed=31)


def both(prob, **kw):
    return P.DabaSolver(prob, **kw), Oracle(prob, **kw)


@pytest.mark.parametrize("loss", ["trivial", "huber", "welsch"])
def test_objective_parity(tiled, loss):
    g, o = both(tiled, loss=loss, n_partitions=3)
    assert rel(g.objective(), o.objective()) <= 1e-12
    st_g, st_o = g.get_state(), o.get_state()
    # F^a(-1) = E^a(x^0 | x^0) per partition
    assert rel(st_g["part"][:, 1], st_o["part"][:, 1]) <= 1e-12


@pytest.mark.parametrize("S,acc", [(1, True), (4, True), (4, False), (8, True)])
def test_free_running_parity_fp64(c1, S, acc):
    """F after each of 100 iterations within 1e-10 relative of the oracle."""
    g, o = both(c1, n_partitions=S, accelerate=acc, loss="huber")
    Fg = g.iterate(100)
    Fo, mo = o.iterate(100)
    r = np.abs(Fg - Fo) / Fo
    assert r.max() <= 1e-10, (r.argmax(), r.max())
    mg = g.metrics()
    assert rel(mg[:, :3], mo[-1, :, :3]) <= 1e-9
    assert np.array_equal(mg[:, 3], mo[-1, :, 3])
    if acc and S > 1:
        assert mo[:, :, 3].sum() > 0  # the restart branch was exercised


def test_free_running_parity_tiled(tiled):
    g, o = both(tiled, n_partitions=5, loss="huber", eta=1.0)
    Fg = g.iterate(60)
    Fo, _ = o.iterate(60)
    assert (np.abs(Fg - Fo) / Fo).max() <= 1e-10


@pytest.mark.parametrize("xi,scale", [(0.05, 256.0), (2.0, 512.0)])
def test_free_running_parity_large_prox(tiled, xi, scale):
    """A proximal weight that shapes every camera and landmark solve (the
    rotation prox of the camera LM, the xi terms of the landmark closed
    form), with another unit scale."""
    g, o = both(tiled, n_partitions=3, loss="huber", xi=xi, unit_scale=scale)
    Fg = g.iterate(40)
    Fo, mo = o.iterate(40)
    assert (np.abs(Fg - Fo) / Fo).max() <= 1e-10
    mg = g.metrics()
    assert rel(mg[:, :3], mo[-1, :, :3]) <= 1e-9
    assert np.array_equal(mg[:, 3], mo[-1, :, 3])


@pytest.mark.parametrize("loss", ["trivial", "welsch"])
def test_free_running_parity_other_losses(tiled, loss):
    """The other two losses of Assumption 1 (Welsch is non-convex): F after
    each of 60 iterations within 1e-10 relative, same restart decisions."""
    g, o = both(tiled, n_partitions=4, loss=loss)
    Fg = g.iterate(60)
    Fo, mo = o.iterate(60)
    r = np.abs(Fg - Fo) / Fo
    assert r.max() <= 1e-10, (r.argmax(), r.max())
    assert np.array_equal(g.metrics()[:, 3], mo[-1, :, 3])


def test_metrics_and_restart_decisions_each_iteration(c1):
    g, o = both(c1, n_partitions=6, loss="huber", eta=0.7)
    Fo, mo = o.iterate(40)
    for k in range(40):
        g.iterate(1)
        mg = g.metrics()
        assert np.array_equal(mg[:, 3], mo[k, :, 3]), k
        assert rel(mg[:, :3], mo[k, :, :3]) <= 1e-9, k


def test_state_after_iterations(c1):
    g, o = both(c1, n_partitions=4, loss="huber")
    g.iterate(30, trace=False)
    o.iterate(30)
    sg, so = g.get_state(), o.get_state()
    assert_state_close(sg, so, 1e-10, "x^30")
    assert_state_close(sg, so, 1e-10, "x^29", cams_key="cams_prev", lms_key="lms_prev")
    assert sg["k"] == so["k"] == 30 and sg["s"] == so["s"]
    assert rel(sg["part"], so["part"]) <= 1e-9


def test_one_step_parity_from_common_state(c1):
    """The oracle continues from the GPU's state: one iteration each."""
    g = P.DabaSolver(c1, n_partitions=4, loss="huber")
    g.iterate(25, trace=False)
    st = g.get_state()
    o = Oracle(c1, n_partitions=4, loss="huber")
    o.set_state(st)
    Fg = g.iterate(1)
    Fo, mo = o.iterate(1)
    assert rel(Fg, Fo) <= 1e-12
    sg, so = g.get_state(), o.get_state()
    assert_state_close(sg, so, 1e-11, "one step")
    assert np.array_equal(g.metrics()[:, 3], mo[0, :, 3])


@pytest.mark.parametrize("loss", ["trivial", "huber", "welsch"])
def test_gradient_parity(tiled, loss):
    g, o = both(tiled, loss=loss, n_partitions=2)
    gc, gl, gu = (t.cpu().numpy() for t in g.grad())
    oc, ol, ou = o.grad()
    assert nrel(gc[:, :12], oc[:, :12]) <= 1e-10
    for k in range(12, 15):
        assert nrel(gc[:, k], oc[:, k]) <= 1e-10
    assert nrel(gl, ol) <= 1e-10
    assert nrel(gu, ou) <= 1e-10


def test_objective_and_gradient_at_caller_point(tiled):
    g, o = both(tiled, loss="huber")
    rng = np.random.default_rng(7)
    lms = tiled["landmarks"] + 0.01 * rng.standard_normal(tiled["landmarks"].shape)
    uv = tiled["obs_uv"] + 0.3 * rng.standard_normal(tiled["obs_uv"].shape)
    cams = tiled["cameras_gt"]
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    assert rel(g.objective(dev(cams), dev(lms), dev(uv)), o.objective(cams, lms, uv)) <= 1e-12
    gc, gl, gu = (t.cpu().numpy() for t in g.grad(dev(cams), dev(lms), dev(uv)))
    oc, ol, ou = o.grad(cams, lms, uv)
    assert nrel(gl, ol) <= 1e-10 and nrel(gu, ou) <= 1e-10 and nrel(gc[:, :12], oc[:, :12]) <= 1e-10
    for k in range(12, 15):
        assert nrel(gc[:, k], oc[:, k]) <= 1e-10
    # the stored point is untouched
    assert rel(g.objective(), o.objective()) <= 1e-12


def test_determinism_and_resume(c1):
    a = P.DabaSolver(c1, n_partitions=4, loss="huber")
    b = P.DabaSolver(c1, n_partitions=4, loss="huber")
    Fa = a.iterate(20)
    Fb = b.iterate(20)
    assert np.array_equal(Fa, Fb)
    st = a.get_state()
    Fa2 = a.iterate(13)
    c = P.DabaSolver(c1, n_partitions=4, loss="huber")
    c.set_state(st)
    Fc = c.iterate(13)
    assert np.array_equal(Fa2, Fc)


def test_duba_monotone_and_partition_independent(c1):
    a = P.DabaSolver(c1, n_partitions=1, loss="huber", accelerate=False)
    b = P.DabaSolver(c1, n_partitions=8, loss="huber", accelerate=False)
    F0 = a.objective()
    Fa = a.iterate(30)
    Fb = b.iterate(30)
    assert np.all(np.diff(np.concatenate([[F0], Fa])) <= 1e-12 * F0)
    assert rel(Fa, Fb) <= 1e-12


def test_forced_restart_equals_mm(c1):
    a = P.DabaSolver(c1, n_partitions=3, loss="huber", debug_flags=ALWAYS_RESTART)
    b = P.DabaSolver(c1, n_partitions=3, loss="huber", accelerate=False)
    assert rel(a.iterate(10), b.iterate(10)) <= 1e-12


def test_converged_inner_solver(tiled):
    g, o = both(tiled, n_partitions=2, loss="huber", inner_steps=0, xi=1e-6)
    Fg = g.iterate(5)
    Fo, _ = o.iterate(5)
    assert rel(Fg, Fo) <= 1e-10


def test_fp32_mixed_within_1e4_after_100(c1):
    """FP32-mixed against the FP64 oracle, per result: the objective after
    100 iterations within 1e-4 (the requirement), and, stated and bounded,
    the objective on every iteration, the iterate per column group and the
    restart decisions."""
    g = P.DabaSolver(c1, n_partitions=4, loss="huber", precision="fp32_mixed")
    o = Oracle(c1, n_partitions=4, loss="huber")
    Fo, mo = o.iterate(100)
    Fg = np.empty(100)
    flags = np.empty((100, 4))
    for k in range(100):
        Fg[k] = g.iterate(1)[0]
        flags[k] = g.metrics()[:, 3]
    r = np.abs(Fg - Fo) / Fo
    agree = float(np.mean(flags == mo[:, :, 3]))
    print(f"FP32-mixed vs oracle: F after 100 {r[-1]:.1e}, worst iteration {r.max():.1e}, "
          f"restart decisions equal on {100 * agree:.1f}% of (iteration, partition) pairs", flush=True)
    assert r[-1] <= 1e-4, r[-1]
    assert r.max() <= 1e-3
    assert agree >= 0.9
    assert_state_close(g.get_state(), o.get_state(), 5e-3, "FP32-mixed iterate after 100")


@pytest.mark.parametrize("loss", ["trivial", "welsch"])
def test_fp32_mixed_other_losses(c1, loss):
    g = P.DabaSolver(c1, n_partitions=4, loss=loss, precision="fp32_mixed")
    o = Oracle(c1, n_partitions=4, loss=loss)
    Fg = g.iterate(100)
    Fo, _ = o.iterate(100)
    r = np.abs(Fg - Fo) / Fo
    assert r[-1] <= 1e-4, r[-1]


def test_edge_cases_empty_entities():
    """A landmark nobody observes, a camera with no observations, more
    partitions than non-empty camera blocks, and a problem with no
    observations at all."""
    prob = make_problem("cam50-lm5k", n_cameras=9, n_landmarks=200, seed=41)
    keep = prob["obs_camera"] != 4
    prob2 = dict(prob)
    prob2["obs_camera"] = prob["obs_camera"][keep]
    prob2["obs_landmark"] = prob["obs_landmark"][keep]
    prob2["obs_uv"] = prob["obs_uv"][keep]
    prob2["n_obs"] = int(keep.sum())
    prob2["n_landmarks"] = prob["n_landmarks"] + 1
    prob2["landmarks"] = np.vstack([prob["landmarks"], [[0.3, -0.2, 0.1]]])
    g, o = both(prob2, n_partitions=12, loss="huber")
    Fg = g.iterate(15)
    Fo, _ = o.iterate(15)
    assert rel(Fg, Fo) <= 1e-10
    sg, so = g.get_state(), o.get_state()
    assert nrel(sg["lms"], so["lms"]) <= 1e-10
    empty = dict(prob2, obs_camera=prob2["obs_camera"][:0], obs_landmark=prob2["obs_landmark"][:0],
                 obs_uv=prob2["obs_uv"][:0], n_obs=0)
    e = P.DabaSolver(empty, n_partitions=2, loss="huber")
    assert e.objective() == 0.0
    assert np.all(e.iterate(3) == 0.0)


def test_degenerate_point_is_reported(c1):
    g = P.DabaSolver(c1, n_partitions=2, loss="huber")
    st = g.get_state()
    j, i = c1["obs_landmark"][0], c1["obs_camera"][0]
    st["lms"][j] = st["cams"][i, 9:12]
    g.set_state({k: v for k, v in st.items() if k != "part"})
    with pytest.raises(P.binding.DabaError) as ei:
        g.iterate(1)
    assert ei.value.code == -5


def test_rejected_set_state_changes_nothing(c1):
    """A state with one camera that is not a rotation (and a new iteration
    counter) is rejected before anything is written: the handle continues
    exactly like an untouched one."""
    a = P.DabaSolver(c1, n_partitions=4, loss="huber")
    b = P.DabaSolver(c1, n_partitions=4, loss="huber")
    a.iterate(5, trace=False)
    b.iterate(5, trace=False)
    bad = a.get_state()
    bad["cams"] = bad["cams"].copy()
    bad["cams"][3, :9] *= 1.5
    bad["k"] = bad["k"] + 7
    with pytest.raises(P.binding.DabaError):
        a.set_state(bad)
    assert np.array_equal(a.iterate(6), b.iterate(6))
    assert np.array_equal(a.get_state()["cams"], b.get_state()["cams"])
