"""The real-data path on the GPU: a scene in BAL's convention (variable track
lengths, radial distortion in BAL's forward model) is written as a BAL file,
read back and converted by paper_2305_07026_amd.bal, and run through both GPU
solvers against their oracles on the same converted problem: the
entity-level iteration (objective within 1e-10 after each of 50 iterations,
restart decisions, the iterate per column group) and the device-level
surrogate (objective within 1e-10 after each of 6 iterations)."""

import io

import numpy as np
import pytest

from bal_scene import scene
from compare import assert_state_close
from oracle import Oracle
from oracle.partition import PartOracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_2305_07026_amd")
bal = P.bal


@pytest.fixture(scope="module")
def converted():
    rng = np.random.default_rng(11)
    raw = scene(rng, M=9, N=700, k_sigma=0.05)
    # 1 px pixel noise, perturbed points (the converted scene is then a
    # problem with a nonzero optimum, like a real one)
    raw["obs_xy"] = raw["obs_xy"] + rng.standard_normal(raw["obs_xy"].shape)
    raw["points"] = raw["points"] + 0.05 * rng.standard_normal(raw["points"].shape)
    buf = io.StringIO()
    bal.write_bal(buf, raw)
    prob = bal.load_bal(io.StringIO(buf.getvalue()))
    tracks = np.bincount(prob["obs_landmark"], minlength=prob["n_landmarks"])
    print(f"BAL scene: {prob['n_cameras']} cameras, {prob['n_landmarks']} points, {prob['n_obs']} observations, "
          f"track lengths {tracks.min()}..{tracks.max()}", flush=True)
    assert tracks.max() > tracks.min()
    return prob


def test_bal_scene_entity_level(converted):
    opts = dict(n_partitions=3, loss="huber", delta=1.0, xi=1e-9, eta=0.5)
    g = P.DabaSolver(converted, **opts)
    o = Oracle(converted, **opts)
    assert abs(g.objective() - o.objective()) <= 1e-12 * o.objective()
    Fo, mo = o.iterate(50)
    Fg = np.empty(50)
    for k in range(50):
        Fg[k] = g.iterate(1)[0]
        assert np.array_equal(g.metrics()[:, 3], mo[k, :, 3]), k
    r = np.abs(Fg - Fo) / Fo
    print(f"BAL scene, entity level: worst relative F over 50 iterations {r.max():.1e}", flush=True)
    assert r.max() <= 1e-10, (r.argmax(), r.max())
    assert Fo[-1] < Fo[0]
    assert_state_close(g.get_state(), o.get_state(), 1e-9, "BAL scene x^50")


def test_bal_scene_device_level(converted):
    g = P.DabaPartSolver(converted, n_partitions=3, loss="huber")
    o = PartOracle(converted, n_partitions=3, loss="huber")
    Fg = g.iterate(6)
    Fo, mo = o.iterate(6)
    r = np.abs(Fg - Fo) / Fo
    print(f"BAL scene, device level: worst relative F over 6 iterations {r.max():.1e}", flush=True)
    assert r.max() <= 1e-10
    np.testing.assert_array_equal(g.get_state()["metrics"][:, 3], mo[-1, :, 3])
