"""The headline configuration at full size (1,000 cameras, 200,000
landmarks, ~1.6M observations, 8 partitions, Huber), in the launch
configuration the benchmark times: objective and per-partition shares at
x^0, then one iteration from a common state, compared with the oracle."""

import numpy as np
import pytest

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
    sg, so = g.get_state(), o.get_state()
    for key in ("cams", "lms"):
        assert np.linalg.norm(sg[key] - so[key]) <= 1e-11 * np.linalg.norm(so[key])
