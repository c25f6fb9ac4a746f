"""The 1,000-camera configuration at full size (200,000 landmarks, ~1.6M
observations, 8 partitions, Huber), in the launch configuration the
benchmark uses: the objective at x^0 and one iteration from a common state,
then a 200-iteration free run from x^0, compared with the oracle after
every iteration (objective, per-partition metrics, restart decisions) and
on the final iterate per column group."""

import numpy as np
import pytest

from compare import assert_state_close
from oracle import Oracle
from synth import make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_2305_07026_amd")


@pytest.fixture(scope="module")
def c2():
    return make_problem("cam1k-lm200k")


def test_fullsize_objective_and_one_step(c2):
    opts = dict(n_partitions=8, loss="huber", delta=1.0, xi=1e-9, eta=0.5)
    g = P.DabaSolver(c2, **opts)
    o = Oracle(c2, **opts)
    assert abs(g.objective() - o.objective()) <= 1e-12 * o.objective()
    g.iterate(12, trace=False)
    st = g.get_state()
    o.set_state(st)
    Fg = g.iterate(1)
    Fo, mo = o.iterate(1)
    assert abs(Fg[0] - Fo[0]) <= 1e-11 * Fo[0]
    mg = g.metrics()
    assert np.array_equal(mg[:, 3], mo[0, :, 3])
    assert np.max(np.abs(mg[:, :3] - mo[0, :, :3]) / np.abs(mo[0, :, :3])) <= 1e-9
    assert_state_close(g.get_state(), o.get_state(), 1e-10, "one step at 1.6M observations")


@pytest.mark.timeout(600)
def test_fullsize_free_run_200_iterations(c2):
    opts = dict(n_partitions=8, loss="huber", delta=1.0, xi=1e-9, eta=0.5)
    o = Oracle(c2, **opts)
    Fo, mo = o.iterate(200)
    print("oracle: 200 iterations done", flush=True)
    g = P.DabaSolver(c2, **opts)
    worst = 0.0
    for k in range(200):
        Fg = g.iterate(1)[0]
        r = abs(Fg - Fo[k]) / Fo[k]
        worst = max(worst, r)
        assert r <= 1e-10, (k, r)
        mg = g.metrics()
        assert np.array_equal(mg[:, 3], mo[k, :, 3]), k
        assert np.max(np.abs(mg[:, :3] - mo[k, :, :3]) / np.abs(mo[k, :, :3])) <= 1e-9, k
    print(f"200 iterations: worst relative F difference {worst:.1e}, restarts {int(mo[:, :, 3].sum())}", flush=True)
    assert mo[:, :, 3].sum() > 0  # the restart branch was taken
    assert_state_close(g.get_state(), o.get_state(), 1e-9, "x^200 at 1.6M observations")
