"""Parity at the two largest configurations, at full size:

* 5,000 cameras, 2,000,000 landmarks, ~16M observations, 16 partitions
  (the precision form);
* 20,000 cameras, 10,000,000 landmarks, ~60M observations, 64 partitions,
  track lengths 2 + Geometric(1/5) (up to ~70 observations per landmark, so
  the landmark pass takes records in several rounds).

At each: the objective at x^0 and one FP64 iteration from a common state
against the oracle (objective after the step, per-partition metrics and
restart decisions, the new iterate), then FP32-mixed against FP64 on the GPU
after 100 iterations (the FP64 path itself being pinned to the oracle)."""

import time

import numpy as np
import pytest

from oracle import Oracle
from synth import CONFIGS, make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_2305_07026_amd")


def say(msg):
    print(msg, flush=True)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("wl", ["cam5k-lm2m", "cam20k-lm10m"])
def test_large_fullsize(wl):
    t0 = time.time()
    prob = make_problem(wl)
    S = CONFIGS[wl]["n_partitions"]
    say(f"{wl}: {prob['n_obs']} observations generated in {time.time() - t0:.0f} s")
    opts = dict(n_partitions=S, loss="huber", delta=1.0, xi=1e-9, eta=0.5)
    g = P.DabaSolver(prob, **opts)
    o = Oracle(prob, **opts)
    assert abs(g.objective() - o.objective()) <= 1e-12 * o.objective()
    g.iterate(3, trace=False)
    o.set_state(g.get_state())
    Fg = g.iterate(1)
    Fo, mo = o.iterate(1)
    say(f"{wl}: one step compared, {time.time() - t0:.0f} s")
    assert abs(Fg[0] - Fo[0]) <= 1e-11 * Fo[0]
    mg = g.metrics()
    assert np.array_equal(mg[:, 3], mo[0, :, 3])
    assert np.max(np.abs(mg[:, :3] - mo[0, :, :3]) / np.abs(mo[0, :, :3])) <= 1e-9
    sg, so = g.get_state(), o.get_state()
    for key in ("cams", "lms"):
        assert np.linalg.norm(sg[key] - so[key]) <= 1e-11 * np.linalg.norm(so[key])
    del o, g

    F64 = P.DabaSolver(prob, **opts).iterate(100)
    F32 = P.DabaSolver(prob, precision="fp32_mixed", **opts).iterate(100)
    say(f"{wl}: FP32-mixed vs FP64 after 100 iterations: {abs(F32[-1] - F64[-1]) / F64[-1]:.2e}")
    assert abs(F32[-1] - F64[-1]) <= 1e-4 * F64[-1]
    assert F64[-1] < F64[0]
