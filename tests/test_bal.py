"""The BAL reader and its conversion to this library's camera model.  A scene
is drawn in BAL's own convention (P = R(w) X + t, p = -P_xy / P_z,
u = f (1 + k1 |p|^2 + k2 |p|^4) p), written as a BAL file, read back and
converted; the converted cameras, projected with the synthetic generator's
(independent) implementation of the paper's model, must land on the BAL
pixels with y negated.  No GPU."""

import io

import numpy as np
import pytest

from bal_scene import scene as _scene
from synth.problem import _project

bal = pytest.importorskip("paper_2305_07026_amd.bal")


def _reprojection_error(prob):
    cams = prob["cameras"]
    o_c, o_l = prob["obs_camera"].astype(np.int64), prob["obs_landmark"].astype(np.int64)
    R = cams[o_c, :9].reshape(-1, 3, 3)
    u, ok = _project(R, cams[o_c, 9:12], cams[o_c, 12:15], prob["landmarks"][o_l])
    assert ok.all()
    return np.max(np.abs(u - prob["obs_uv"]))


def test_file_round_trip():
    raw = _scene(np.random.default_rng(1))
    buf = io.StringIO()
    bal.write_bal(buf, raw)
    back = bal.read_bal(io.StringIO(buf.getvalue()))
    for key in raw:
        assert np.array_equal(np.asarray(raw[key]), back[key]), key


def test_undistorted_cameras_convert_exactly():
    raw = _scene(np.random.default_rng(2), k_sigma=0.0)
    prob = bal.bal_to_problem(raw)
    assert np.allclose(prob["cameras"][:, 12], raw["cameras"][:, 6]) and np.all(prob["cameras"][:, 13:] == 0)
    assert _reprojection_error(prob) < 1e-9


def test_distorted_cameras_convert_to_subpixel():
    raw = _scene(np.random.default_rng(3), k_sigma=0.05)
    prob = bal.bal_to_problem(raw)
    assert prob["n_obs"] > 300
    assert np.max(prob["intrinsics_fit_error"]) < 1e-4
    assert _reprojection_error(prob) < 0.05
    # rotations are rotations
    R = prob["cameras"][:, :9].reshape(-1, 3, 3)
    assert np.allclose(R @ np.transpose(R, (0, 2, 1)), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0)


def test_rejects_bad_files():
    with pytest.raises(ValueError):
        bal.read_bal(io.StringIO("2 3"))
    with pytest.raises(ValueError):
        bal.read_bal(io.StringIO("1 1 1\n0 5 1.0 2.0\n" + "0\n" * 9 + "0\n" * 3))


def test_converted_scene_runs_plain_mm_downhill():
    """The converted problem (with 1 px pixel noise and perturbed points) is
    a valid input: the oracle's plain MM descends monotonically on it."""
    from oracle import Oracle
    rng = np.random.default_rng(4)
    raw = _scene(rng)
    raw["obs_xy"] = raw["obs_xy"] + rng.standard_normal(raw["obs_xy"].shape)
    raw["points"] = raw["points"] + 0.05 * rng.standard_normal(raw["points"].shape)
    prob = bal.bal_to_problem(raw)
    o = Oracle(prob, n_partitions=2, loss="huber", accelerate=False)
    F0 = o.objective()
    F, _ = o.iterate(20)
    assert F[0] < F0 and np.all(np.diff(F) <= 1e-12 * F0)
