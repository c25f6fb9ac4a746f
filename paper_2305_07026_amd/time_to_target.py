"""Time to target and performance profiles for DABA against DUBA (Sec. VII).

The paper uses two measures. One is the target objective of eq. Fdelta,
F_delta(p) = F_ref + Delta (F_init - F_ref). The other is the performance
profile of Dolan and More: the share of problems whose objective reaches
F_delta(p) within k iterations, plotted over k (Fig. 3, Delta = 1e-4).

Here these run over seeded synthetic problems and compare two methods:
DABA (Nesterov extrapolation with adaptive restart) and DUBA (the same
iteration without acceleration).

The paper takes F_ref from a centralized solver, per problem and loss and
independent of the device count; that solver is not part of this library.
Here F_ref(p) for a loss is the lowest objective that any run on p with that
loss reaches within the iteration budget, over every partition count and
both methods.

    python -m paper_2305_07026_amd.time_to_target [--budget 2000] [--out FILE] [--surrogate device]
"""

from __future__ import annotations

import argparse
import json
import time
from dataclasses import dataclass

import numpy as np

METHODS = {"DABA": True, "DUBA": False}  # method -> Nesterov acceleration with adaptive restart


def f_delta(F_init: float, F_ref: float, delta: float = 1e-4) -> float:
    """eq. Fdelta: the target objective with suboptimality tolerance delta."""
    return F_ref + delta * (F_init - F_ref)


def iterations_to_target(trace, target: float):
    """Iterations needed to reach the target: the 1-based index of the first
    entry <= target (trace[i] is F after iteration i + 1), or None if no
    entry is."""
    hit = np.nonzero(np.asarray(trace, dtype=np.float64) <= target)[0]
    return int(hit[0]) + 1 if hit.size else None


def performance_profile(iters, ks):
    """Share of problems solved within k iterations, for each k in ks.
    iters holds the iterations to target per problem (None: not reached)."""
    n = len(iters)
    if n == 0:
        return [0.0 for _ in ks]
    return [sum(1 for x in iters if x is not None and x <= k) / n for k in ks]


@dataclass(frozen=True)
class Problem:
    """One synthetic problem of the suite: a generator configuration, its
    sizes and a seed."""
    config: str
    n_cameras: int
    n_landmarks: int
    seed: int

    @property
    def name(self) -> str:
        return f"{self.n_cameras}cam-{self.n_landmarks}lm-seed{self.seed}"

    def make(self) -> dict:
        from synth import make_problem
        return make_problem(self.config, seed=self.seed, n_cameras=self.n_cameras, n_landmarks=self.n_landmarks)


def default_suite(seeds=(11, 12, 13, 14, 15)):
    """Ten problems: 50 cameras / 5,000 landmarks and 200 cameras / 20,000
    landmarks (about 8 observations per landmark), five seeds each."""
    return [Problem("cam50-lm5k", m, n, s) for (m, n) in ((50, 5_000), (200, 20_000)) for s in seeds]


def gpu_runner(prob: dict, accelerate: bool, loss: str, S: int, budget: int):
    """(F at x^0, F after each of `budget` iterations) on the GPU path with
    the entity-level surrogate."""
    from .solver import DabaSolver
    sol = DabaSolver(prob, n_partitions=S, loss=loss, delta=1.0, accelerate=accelerate)
    F0 = sol.objective()
    trace = sol.iterate(budget)
    sol.close()
    return F0, trace


def gpu_runner_device(prob: dict, accelerate: bool, loss: str, S: int, budget: int):
    """The same with the device-level surrogate of eq. Ealpha (intra-partition
    pairs exact, one LM solve per partition)."""
    from .solver import DabaPartSolver, DabaSolver
    F0 = DabaSolver(prob, n_partitions=S, loss=loss, delta=1.0).objective()
    sol = DabaPartSolver(prob, n_partitions=S, loss=loss, delta=1.0, accelerate=accelerate)
    trace = sol.iterate(budget)
    sol.close()
    return F0, trace


def run(problems, *, losses=("trivial", "huber"), partitions=(4, 8, 16, 32), budget=2000, delta=1e-4,
        runner=gpu_runner, ks=None, log=None):
    """Runs every method on every (problem, loss, partition count).

    Returns a dict with one record per (problem, loss, partitions). Each
    record holds F_init, the F_ref shared by all runs of that problem and
    loss, the target and each method's iterations to target. The dict also
    holds the performance profiles per (loss, partitions, method) at the
    iteration counts ks."""
    if ks is None:
        ks = sorted({int(round(x)) for x in np.geomspace(1, budget, 25)})
    records = []
    for pr in problems:
        prob = pr.make()
        for loss in losses:
            runs = []  # (S, F_init, {method: trace})
            for S in partitions:
                S_eff = min(S, prob["n_cameras"])
                F0, traces = None, {}
                for name, acc in METHODS.items():
                    f0, tr = runner(prob, acc, loss, S_eff, budget)
                    F0 = f0 if F0 is None else F0
                    traces[name] = np.asarray(tr, dtype=np.float64)
                runs.append((S_eff, F0, traces))
            F_ref = min(float(t.min()) for _, _, tr in runs for t in tr.values())
            for S_eff, F0, traces in runs:
                target = f_delta(F0, F_ref, delta)
                rec = dict(problem=pr.name, loss=loss, partitions=S_eff, F_init=F0, F_ref=F_ref, F_target=target,
                           iterations={m: iterations_to_target(t, target) for m, t in traces.items()},
                           F_final={m: float(t[-1]) for m, t in traces.items()})
                records.append(rec)
                if log:
                    log(f"{pr.name} {loss} S={S_eff}: " +
                        ", ".join(f"{m} {rec['iterations'][m]}" for m in METHODS))
    profiles = {}
    for loss in losses:
        for S in sorted({r["partitions"] for r in records}):
            sel = [r for r in records if r["loss"] == loss and r["partitions"] == S]
            if not sel:
                continue
            profiles[f"{loss}/S={S}"] = {m: performance_profile([r["iterations"][m] for r in sel], ks)
                                         for m in METHODS}
    return dict(delta=delta, budget=budget, ks=ks, records=records, profiles=profiles,
                reference="F_ref per problem and loss = lowest objective any run reaches within the budget")


def summary(result) -> str:
    """A text table: per (loss, partitions), the share of problems each
    method solves within the budget and its median iterations to target."""
    lines = [f"{'loss/partitions':18s} " + " ".join(f"{m + ' solved':>12s} {m + ' median':>12s}" for m in METHODS)]
    for key in result["profiles"]:
        loss, S = key.split("/S=")
        sel = [r for r in result["records"] if r["loss"] == loss and r["partitions"] == int(S)]
        cells = []
        for m in METHODS:
            it = [r["iterations"][m] for r in sel]
            done = [x for x in it if x is not None]
            med = float(np.median(done)) if done else float("nan")
            cells.append(f"{len(done) / len(it):12.2f} {med:12.1f}")
        lines.append(f"{key:18s} " + " ".join(cells))
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--budget", type=int, default=2000)
    ap.add_argument("--delta", type=float, default=1e-4)
    ap.add_argument("--out", default=None, help="write the full result as JSON")
    ap.add_argument("--surrogate", default="entity", choices=["entity", "device"],
                    help="entity: every pair majorized; device: the surrogate of eq. Ealpha (include/daba_part.h)")
    args = ap.parse_args()
    t0 = time.time()
    runner = gpu_runner_device if args.surrogate == "device" else gpu_runner
    res = run(default_suite(), budget=args.budget, delta=args.delta, runner=runner,
              log=lambda s: print(s, flush=True))
    print(summary(res))
    print(f"({len(res['records'])} comparisons in {time.time() - t0:.0f} s)")
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
