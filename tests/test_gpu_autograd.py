"""The hand-written adjoint behind torch.autograd.Function (App. D, eq.
DFij with the intrinsics row transposed back, plus the pixel gradient):
central finite differences (h = 1e-6 in well-scaled coordinates) on a
10-camera / 200-point sub-problem, torch.autograd.gradcheck on a tiny one,
and the oracle's gradient on the full differentiation-form problem."""

import numpy as np
import pytest

from oracle import Oracle
from synth import make_problem, subproblem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
P = pytest.importorskip("paper_2305_07026_amd")

DEV = "cuda"


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device=DEV)


def to_params(cams):
    """(R 9 | t 3 | f, kappa1, kappa2) with d = (f, kappa1 / f, kappa2 / f^3)."""
    f = cams[:, 12]
    return np.concatenate([cams[:, :12], f[:, None], (cams[:, 13] * f)[:, None], (cams[:, 14] * f ** 3)[:, None]], 1)


def from_params(q):
    f = q[:, 12:13]
    return torch.cat([q[:, :12], f, q[:, 13:14] / f, q[:, 14:15] / f ** 3], dim=1)


@pytest.fixture(scope="module")
def sub():
    big = make_problem("cam1k-lm200k-grad", n_cameras=40, n_landmarks=3000, seed=44)
    return subproblem(big, 10, 200)


@pytest.mark.parametrize("loss", ["trivial", "huber"])
def test_autograd_matches_central_differences(sub, loss):
    sol = P.DabaSolver(sub, loss=loss, n_partitions=1)
    q = dev(to_params(sub["cameras"])).requires_grad_(True)
    l = dev(sub["landmarks"]).requires_grad_(True)
    u = dev(sub["obs_uv"]).requires_grad_(True)
    F = P.daba_objective(sol, from_params(q), l, u)
    F.backward()
    rng = np.random.default_rng(3)

    def F_at(qq, ll, uu):
        with torch.no_grad():
            return sol.objective(from_params(qq).contiguous(), ll.contiguous(), uu.contiguous())

    checks = []
    f0 = float(sub["cameras"][0, 12])
    # h = 1e-6 in world units for R entries, t and l, in pixels for u, and in
    # the well-scaled (f / f0, kappa1, kappa2) for the intrinsics
    for _ in range(40):
        which = rng.integers(0, 3)
        if which == 0:
            i, c = rng.integers(0, sub["n_cameras"]), rng.integers(0, 15)
            h = 1e-6 * f0 if c == 12 else 1e-6
            base, grad, idx = q, q.grad, (i, c)
        elif which == 1:
            j, c = rng.integers(0, sub["n_landmarks"]), rng.integers(0, 3)
            h, base, grad, idx = 1e-6, l, l.grad, (j, c)
        else:
            o, c = rng.integers(0, sub["n_obs"]), rng.integers(0, 2)
            h, base, grad, idx = 1e-6, u, u.grad, (o, c)
        plus, minus = base.detach().clone(), base.detach().clone()
        plus[idx] += h
        minus[idx] -= h
        args_p = [q.detach(), l.detach(), u.detach()]
        args_m = [q.detach(), l.detach(), u.detach()]
        args_p[which] = plus
        args_m[which] = minus
        fd = (F_at(*args_p) - F_at(*args_m)) / (2 * h)
        checks.append((fd, float(grad[idx])))
    fd = np.array([c[0] for c in checks])
    an = np.array([c[1] for c in checks])
    scale = np.abs(an).max()
    assert np.all(np.abs(fd - an) <= 1e-4 * np.abs(an) + 1e-6 * scale), np.max(np.abs(fd - an) / scale)


def test_gradcheck_tiny():
    big = make_problem("cam50-lm5k", n_cameras=3, n_landmarks=20, seed=45)
    sol = P.DabaSolver(big, loss="huber", n_partitions=1)
    # pixels in units of 1/512 px so every input is O(1)-scaled for gradcheck
    q = dev(to_params(big["cameras"])).requires_grad_(True)
    l = dev(big["landmarks"]).requires_grad_(True)
    un = dev(big["obs_uv"] / 512.0).requires_grad_(True)

    def fn(qq, ll, uu):
        return P.daba_objective(sol, from_params(qq), ll, uu * 512.0) / 1e4

    assert torch.autograd.gradcheck(fn, (q, l, un), eps=1e-6, atol=1e-5, rtol=1e-4, nondet_tol=1e-10)


def test_fp32_gradient_error(sub):
    g64 = P.DabaSolver(sub, loss="huber", n_partitions=1)
    g32 = P.DabaSolver(sub, loss="huber", n_partitions=1, precision="fp32_mixed")
    a = [t.cpu().numpy() for t in g64.grad()]
    b = [t.cpu().numpy() for t in g32.grad()]
    for x, y in zip(a, b):
        # FP32 residuals carry ~1e-7 relative error on O(1) quantities, which
        # the cancellation e = R p - lambda m amplifies to ~1e-4 on e
        assert np.linalg.norm(x - y) <= 2e-3 * np.linalg.norm(x)
    assert abs(g64.objective() - g32.objective()) <= 1e-4 * g64.objective()


def test_gradient_parity_differentiation_form():
    """Full differentiation-form size: 1,000 cameras, 200,000 landmarks,
    ~1.6M observations, against the oracle's gradient, in FP64 and in the
    FP32-mixed form."""
    prob = make_problem("cam1k-lm200k-grad")
    g = P.DabaSolver(prob, loss="huber", n_partitions=8)
    o = Oracle(prob, loss="huber", n_partitions=8)
    gc, gl, gu = (t.cpu().numpy() for t in g.grad())
    oc, ol, ou = o.grad()
    for a, b in ((gc[:, :12], oc[:, :12]), (gl, ol), (gu, ou)):
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
    for k in range(12, 15):
        assert np.linalg.norm(gc[:, k] - oc[:, k]) <= 1e-10 * np.linalg.norm(oc[:, k])
    assert abs(g.objective() - o.objective()) <= 1e-12 * o.objective()
    # the FP32-mixed adjoint at the same size (FP32 residuals: ~1e-4 on e)
    g32 = P.DabaSolver(prob, loss="huber", n_partitions=8, precision="fp32_mixed")
    fc, fl, fu = (t.cpu().numpy() for t in g32.grad())
    for a, b in ((fc, oc), (fl, ol), (fu, ou)):
        assert np.linalg.norm(a - b) <= 2e-3 * np.linalg.norm(b)
    assert abs(g32.objective() - o.objective()) <= 1e-4 * o.objective()
