"""The time-to-target arithmetic (eq. Fdelta, iterations to target, the
performance profile of Fig. 3's methodology) on hand-computed cases, and the
suite runner on traces with known crossings.  No GPU."""

import math

import pytest

T = pytest.importorskip("paper_2305_07026_amd.time_to_target")


def test_f_delta_closed_form():
    # F_ref + Delta (F_init - F_ref)
    assert T.f_delta(10.0, 2.0, 0.25) == 4.0
    assert T.f_delta(7.0, 7.0, 1e-4) == 7.0
    assert T.f_delta(3.0, 1.0) == pytest.approx(1.0002)


def test_iterations_to_target():
    tr = [5.0, 4.0, 3.0, 2.0]
    assert T.iterations_to_target(tr, 3.0) == 3  # ties count as reached
    assert T.iterations_to_target(tr, 5.0) == 1
    assert T.iterations_to_target(tr, 1.0) is None
    assert T.iterations_to_target([], 1.0) is None


def test_performance_profile_by_hand():
    assert T.performance_profile([1, 3, None, 10], [1, 2, 3, 10, 100]) == [0.25, 0.25, 0.5, 0.75, 0.75]
    assert T.performance_profile([], [1, 5]) == [0.0, 0.0]


class _Fake:
    """A stand-in problem whose runs follow F_k = F0 r^k (r per method)."""

    def __init__(self, seed):
        self.seed = seed
        self.name = f"fake{seed}"

    def make(self):
        return dict(n_cameras=10, seed=self.seed)


def _runner(prob, accelerate, loss, S, budget):
    F0 = 100.0 + prob["seed"]
    r = 0.5 if accelerate else 0.8
    return F0, [F0 * r ** k for k in range(1, budget + 1)]


def _runner_S(prob, accelerate, loss, S, budget):
    # as _runner, with the plain method slower on more partitions
    F0 = 100.0 + prob["seed"]
    r = 0.5 if accelerate else 0.8 + 0.001 * S
    return F0, [F0 * r ** k for k in range(1, budget + 1)]


def test_reference_is_shared_across_partitions():
    res = T.run([_Fake(1)], losses=("huber",), partitions=(2, 6), budget=40, delta=1e-3, runner=_runner_S,
                ks=[40])
    a, b = res["records"]
    assert a["F_ref"] == b["F_ref"] == 101.0 * 0.5 ** 40
    assert a["iterations"]["DUBA"] <= b["iterations"]["DUBA"]


def test_run_with_known_traces():
    budget, delta = 60, 1e-3
    res = T.run([_Fake(1), _Fake(2)], losses=("huber",), partitions=(4, 32), budget=budget, delta=delta,
                runner=_runner, ks=[1, 10, 20, 40, 60])
    assert len(res["records"]) == 4
    assert sorted(r["partitions"] for r in res["records"]) == [4, 4, 10, 10]  # capped at the camera count
    for rec in res["records"]:
        F0 = rec["F_init"]
        F_ref = F0 * 0.5 ** budget
        assert rec["F_ref"] == F_ref
        target = F_ref + delta * (F0 - F_ref)
        # first k with F0 r^k <= target, by direct search
        for m, r in (("DABA", 0.5), ("DUBA", 0.8)):
            k = next((k for k in range(1, budget + 1) if F0 * r ** k <= target), None)
            assert rec["iterations"][m] == k
        assert rec["iterations"]["DABA"] == math.ceil(math.log(target / F0) / math.log(0.5))
    prof = res["profiles"]["huber/S=4"]
    assert prof["DABA"] == [0.0, 1.0, 1.0, 1.0, 1.0]
    assert prof["DUBA"] == [0.0, 0.0, 0.0, 1.0, 1.0]
