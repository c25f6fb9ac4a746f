"""The time-to-target harness on the GPU path against the same harness
driven by the oracle: on small problems, every run's F_init, F_ref, target
and each method's iterations to target agree."""

import numpy as np
import pytest

from oracle import Oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
T = pytest.importorskip("paper_2305_07026_amd.time_to_target")


def _oracle_runner(prob, accelerate, loss, S, budget):
    o = Oracle(prob, n_partitions=S, loss=loss, delta=1.0, accelerate=accelerate)
    return o.objective(), o.iterate(budget)[0]


def test_gpu_and_oracle_suites_agree():
    problems = [T.Problem("cam50-lm5k", 12, 400, s) for s in (31, 32)]
    kw = dict(losses=("trivial", "huber"), partitions=(1, 3), budget=60, delta=1e-4, ks=[5, 20, 60])
    g = T.run(problems, runner=T.gpu_runner, **kw)
    o = T.run(problems, runner=_oracle_runner, **kw)
    assert len(g["records"]) == len(o["records"]) == 8
    for a, b in zip(g["records"], o["records"]):
        for key in ("F_init", "F_ref", "F_target"):
            assert abs(a[key] - b[key]) <= 1e-10 * abs(b[key]), (a, b)
        assert a["iterations"] == b["iterations"], (a, b)
    assert g["profiles"] == o["profiles"]
    # DUBA (plain MM) never increases F, so it reaches the target in the end
    # whenever DABA's lower objective is the reference
    for r in g["records"]:
        assert r["F_final"]["DUBA"] >= r["F_ref"] * (1 - 1e-12)
