"""Plain CPU FP64 oracle of DABA with the paper's device-level surrogate.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the GPU library never loads it, and it shares
no code with the GPU path.  numpy, vectorised over observations, with a dense
linear solve per partition: slow, and meant for small problems.

Sec. IV splits the observations into E' (camera and point on the same device)
and E'' (on different devices).  The device surrogate E^a(x^a | y) of
eq. Ealpha keeps every pair of E' exact and majorizes every pair of E'' by
Prop. 1:

    E^a(x^a | y) = xi/2 |x^a - y^a|^2 + sum_{(i,j) in E', i, j in a} F_ij(c_i, l_j)
                   + sum_{(i,j) in E'', i in a} P_ij(c_i | y)
                   + sum_{(i,j) in E'', j in a} Q_ij(l_j | y),

and the gap of eq. DEalpha charges half of F_ij - P_ij - Q_ij of each pair of
E'' to each of its two devices, so that sum_a (E^a + DeltaE^a) = F.

Readings where the paper is silent (the partitions, Nesterov scalars, restart
test and units follow the entity-level oracle, oracle.c):
  P1  Devices are the S camera partitions; camera i is in partition
      floor(i / ceil(M/S)) and landmark j in the partition of the lowest
      camera id observing it, unless given.
  P2  E^a is minimised by Levenberg-Marquardt over all of a's cameras and
      landmarks together (Sec. VII-B names LM and one successful inner step):
      tangent coordinates (dtheta, dt, dd) per camera with R <- R Exp(dtheta)
      and dl per landmark; model Hessian = Gauss-Newton with the robust
      weight rho'(|e|^2) for pairs of E' (iteratively reweighted), 2 w J^T J
      for P_ij and 2 w lambda^2 I for Q_ij, plus xi I; damping mu diag(H),
      mu0 = 1e-4; a step is accepted iff E^a strictly decreases (then
      mu /= 10), else mu *= 10 and retry, giving up after 10 rejects in a
      row; stop after inner_steps accepted steps (>= 1).  A damped system
      that is not positive definite counts as a rejected step.
  P3  The linear system of each step is solved exactly (here by a dense
      Cholesky factorisation; the paper does not say how).
  P4  The rotation part of the proximal gradient is that of
      xi/2 |R Exp(dtheta) - R^y|_F^2 at dtheta = 0; its model Hessian is
      xi I, as for t and d (as in the entity-level camera solve).
  P5  The restart test and the bookkeeping of eq. Fak, lFak, Eak are those
      of the entity-level oracle with E^a and DeltaE^a above.
"""

from __future__ import annotations

import numpy as np

LOSSES = ("trivial", "huber", "welsch")
NEVER_RESTART = 1
ALWAYS_RESTART = 2


# ------------------------------------------------------------ small helpers

def skew(w):
    """[w]x for w (..., 3)."""
    w = np.asarray(w, dtype=np.float64)
    K = np.zeros(w.shape[:-1] + (3, 3))
    K[..., 0, 1], K[..., 0, 2], K[..., 1, 2] = -w[..., 2], w[..., 1], -w[..., 0]
    K[..., 1, 0], K[..., 2, 0], K[..., 2, 1] = w[..., 2], -w[..., 1], w[..., 0]
    return K


def so3_exp(w):
    """Exp([w]x) by Rodrigues' formula, Taylor coefficients for tiny angles."""
    w = np.asarray(w, dtype=np.float64)
    th2 = np.sum(w * w, axis=-1)[..., None, None]
    th = np.sqrt(th2)
    tiny = th < 1e-8
    ths = np.where(tiny, 1.0, th)
    A = np.where(tiny, 1.0, np.sin(ths) / ths)
    B = np.where(tiny, 0.5, (1.0 - np.cos(ths)) / (ths * ths))
    K = skew(w)
    return np.eye(3) + A * K + B * (K @ K)


def projrot3d(M):
    """eq. proj_rot3d: the rotation nearest to M in Frobenius norm,
    U diag(1, 1, det(U V^T)) V^T from the SVD M = U S V^T (Umeyama)."""
    U, _, Vt = np.linalg.svd(M)
    D = np.ones(M.shape[:-2] + (3,))
    D[..., 2] = np.sign(np.linalg.det(U @ Vt))
    return U @ (D[..., :, None] * Vt)


def ray(d, u):
    """eq. ray: p = [u; d1 + d2 |u|^2 + d3 |u|^4]."""
    r2 = np.sum(u * u, axis=-1)
    return np.stack([u[..., 0], u[..., 1], d[..., 0] + d[..., 1] * r2 + d[..., 2] * r2 * r2], axis=-1)


# ------------------------------------------------------------------ oracle

class PartOracle:
    """State of partition-level DABA for one problem.  Public arrays are in
    caller units (pixels); everything inside is in pixels / unit_scale."""

    def __init__(self, prob: dict, *, n_partitions=None, cam_part=None, lm_part=None, unit_scale=512.0,
                 loss="huber", delta=1.0, xi=1e-9, eta=0.5, accelerate=True, inner_steps=1, flags=0,
                 cameras=None, landmarks=None, uv=None):
        if loss not in LOSSES:
            raise ValueError(loss)
        if inner_steps < 1:
            raise ValueError("inner_steps must be >= 1")
        self.M, self.N, self.K = int(prob["n_cameras"]), int(prob["n_landmarks"]), int(prob["n_obs"])
        self.S = int(n_partitions if n_partitions is not None else prob.get("n_partitions", 1))
        self.s_unit = float(unit_scale)
        self.loss, self.delta = loss, float(delta) / self.s_unit
        self.xi, self.eta = float(xi), float(eta)
        self.accelerate, self.inner_steps, self.flags = bool(accelerate), int(inner_steps), int(flags)
        self.cam = np.asarray(prob["obs_camera"], dtype=np.int64)
        self.lmk = np.asarray(prob["obs_landmark"], dtype=np.int64)
        self.u = np.asarray(prob["obs_uv"] if uv is None else uv, dtype=np.float64) / self.s_unit
        c = np.asarray(prob["cameras"] if cameras is None else cameras, dtype=np.float64)
        lms = np.asarray(prob["landmarks"] if landmarks is None else landmarks, dtype=np.float64)
        self.x = (*self._cams_in(c), lms.copy())
        self.x_prev = tuple(a.copy() for a in self.x)
        # partitions (P1)
        if cam_part is None:
            blk = -(-self.M // self.S)
            self.cpart = np.arange(self.M) // blk
        else:
            self.cpart = np.asarray(cam_part, dtype=np.int64)
        if lm_part is None:
            first = np.full(self.N, self.M, np.int64)
            np.minimum.at(first, self.lmk, self.cam)
            self.lpart = np.where(first < self.M, self.cpart[np.minimum(first, self.M - 1)], 0)
        else:
            self.lpart = np.asarray(lm_part, dtype=np.int64)
        if (self.cpart.min(initial=0) < 0 or self.cpart.max(initial=0) >= self.S or
                self.lpart.min(initial=0) < 0 or self.lpart.max(initial=0) >= self.S):
            raise ValueError("partition index out of range")
        self.oc = self.cpart[self.cam]  # partition of each observation's camera
        self.ol = self.lpart[self.lmk]  # ... and of its landmark
        self.intra = self.oc == self.ol  # E'
        # eq. Fainit
        lin0 = self.linearize(self.x)
        E0 = self.surrogate(self.x, self.x, lin0)
        self.Fprev = E0.copy()
        self.Fbar = E0.copy()
        self.E = E0.copy()
        self.s_nes = np.ones(self.S)
        self.k = 0

    # ---- units
    def _cams_in(self, c):
        s = self.s_unit
        R = c[:, 0:9].reshape(-1, 3, 3).copy()
        t = c[:, 9:12].copy()
        d = np.stack([c[:, 12] / s, c[:, 13] * s, c[:, 14] * s ** 3], axis=1)
        return R, t, d

    def _cams_out(self, R, t, d):
        s = self.s_unit
        dd = np.stack([d[:, 0] * s, d[:, 1] / s, d[:, 2] / s ** 3], axis=1)
        return np.concatenate([R.reshape(-1, 9), t, dd], axis=1)

    # ---- robust loss (Assumption 1; Huber and Welsch widths as in oracle.c)
    def rho(self, s):
        dl = self.delta
        if self.loss == "huber":
            big = s > dl * dl
            ss = np.where(big, s, 1.0)
            return np.where(big, 2.0 * dl * np.sqrt(ss) - dl * dl, s), np.where(big, dl / np.sqrt(ss), 1.0)
        if self.loss == "welsch":
            ex = np.exp(-s / (dl * dl))
            return dl * dl * (1.0 - ex), ex
        return s.copy(), np.ones_like(s)

    # ---- per observation quantities (Sec. III, Prop. 1)
    def obs(self, x, sel=slice(None)):
        """Residual and majorizer quantities of the observations `sel` at x."""
        R, t, d, l = x
        ci, lj, u = self.cam[sel], self.lmk[sel], self.u[sel]
        Ri, ti, di, lm = R[ci], t[ci], d[ci], l[lj]
        m = lm - ti
        r2 = np.sum(m * m, axis=1)
        if np.any(~(r2 > 1e-24)):
            raise FloatingPointError("Assumption 2 violated")
        p = ray(di, u)
        Rp = np.einsum("kab,kb->ka", Ri, p)
        n = np.einsum("kba,kb->ka", Ri, m)  # R^T (l - t)
        lam = np.sum(m * Rp, axis=1) / r2  # eq. lambdaij
        e = p - n * (np.sum(n * p, axis=1) / r2)[:, None]  # eq. error
        sq = np.sum(e * e, axis=1)
        rho, w = self.rho(sq)
        a = 0.5 * rho - 0.5 * w * sq  # eq. a
        g = 0.5 * Rp + 0.5 * lam[:, None] * ti + 0.5 * lam[:, None] * lm  # eq. g
        return dict(p=p, n=n, r2=r2, lam=lam, e=e, sq=sq, rho=rho, w=w, a=a, g=g, F=0.5 * rho)

    def linearize(self, y):
        q = self.obs(y)
        return dict(w=q["w"], lam=q["lam"], g=q["g"], a=q["a"])

    def P_val(self, lin, x):
        """eq. P for every observation, camera from x, frozen quantities lin."""
        R, t, d, _ = x
        p = ray(d[self.cam], self.u)
        v = np.einsum("kab,kb->ka", R[self.cam], p) + lin["lam"][:, None] * t[self.cam] - lin["g"]
        return lin["w"] * np.sum(v * v, axis=1) + 0.5 * lin["a"]

    def Q_val(self, lin, x):
        """eq. Q for every observation."""
        v = lin["lam"][:, None] * x[3][self.lmk] - lin["g"]
        return lin["w"] * np.sum(v * v, axis=1) + 0.5 * lin["a"]

    def _prox_parts(self, x, y):
        R, t, d, l = x
        Ry, ty, dy, ly = y
        pc = (np.sum((R - Ry) ** 2, axis=(1, 2)) + np.sum((t - ty) ** 2, axis=1) + np.sum((d - dy) ** 2, axis=1))
        pl = np.sum((l - ly) ** 2, axis=1)
        out = np.bincount(self.cpart, weights=pc, minlength=self.S)
        return out + np.bincount(self.lpart, weights=pl, minlength=self.S)

    # ---- eq. Ealpha and eq. DEalpha
    def surrogate(self, x, y, lin_y):
        """E^a(x | y) for every partition a (x: full state; only a's part
        of x enters E^a)."""
        F = self.obs(x)["F"]
        P, Q = self.P_val(lin_y, x), self.Q_val(lin_y, x)
        cut = ~self.intra
        E = 0.5 * self.xi * self._prox_parts(x, y)
        E += np.bincount(self.oc[self.intra], weights=F[self.intra], minlength=self.S)
        E += np.bincount(self.oc[cut], weights=P[cut], minlength=self.S)
        E += np.bincount(self.ol[cut], weights=Q[cut], minlength=self.S)
        return E

    def gap(self, x, y, lin_y):
        """DeltaE^a(x | y) of eq. DEalpha for every partition a."""
        F = self.obs(x)["F"]
        P, Q = self.P_val(lin_y, x), self.Q_val(lin_y, x)
        cut = ~self.intra
        half = 0.5 * (F - P - Q)
        dE = -0.5 * self.xi * self._prox_parts(x, y)
        dE += np.bincount(self.oc[cut], weights=half[cut], minlength=self.S)
        dE += np.bincount(self.ol[cut], weights=half[cut], minlength=self.S)
        return dE

    # ---- Jacobians
    def residual_jacobian(self, x, sel):
        """e of the observations `sel` at x, and its Jacobians with respect
        to the camera's (dtheta, dt, dd) [K,3,9] and the landmark's dl [K,3,3]
        for R <- R Exp(dtheta), t <- t + dt, d <- d + dd, l <- l + dl."""
        q = self.obs(x, sel)
        R = x[0][self.cam[sel]]
        n, p, r2 = q["n"], q["p"], q["r2"]
        npv = np.sum(n * p, axis=1)
        I = np.eye(3)
        # e = (I - n n^T / |n|^2) p; De = de/dn
        De = (-(npv[:, None, None] * I + n[:, :, None] * p[:, None, :]) / r2[:, None, None]
              + 2.0 * npv[:, None, None] * n[:, :, None] * n[:, None, :] / (r2 * r2)[:, None, None])
        Pperp = I - n[:, :, None] * n[:, None, :] / r2[:, None, None]
        u = self.u[sel]
        r2u = np.sum(u * u, axis=1)
        b = np.stack([np.ones_like(r2u), r2u, r2u * r2u], axis=1)
        Rt = np.transpose(R, (0, 2, 1))
        Jc = np.concatenate([De @ skew(n),                              # n = R^T m, dn = [n]x dtheta
                             -De @ Rt,                                  # dn = -R^T dt
                             Pperp[:, :, 2:3] * b[:, None, :]], axis=2)  # dp = e3 b^T dd
        Jl = De @ Rt
        return q, Jc, Jl

    def P_jacobian(self, lin, x, sel):
        """r = R p + lambda t - g of eq. P and dr / d(dtheta, dt, dd)."""
        R, t, d, _ = x
        ci = self.cam[sel]
        u = self.u[sel]
        p = ray(d[ci], u)
        Rp = np.einsum("kab,kb->ka", R[ci], p)
        lam = lin["lam"][sel]
        r = Rp + lam[:, None] * t[ci] - lin["g"][sel]
        r2u = np.sum(u * u, axis=1)
        b = np.stack([np.ones_like(r2u), r2u, r2u * r2u], axis=1)
        J = np.concatenate([-R[ci] @ skew(p),                            # d(R Exp(w) p) = -R [p]x w
                            lam[:, None, None] * np.eye(3),
                            R[ci][:, :, 2:3] * b[:, None, :]], axis=2)
        return r, J

    # ---- Levenberg-Marquardt on one partition (P2, P3, P4)
    def unknowns(self, a):
        cams = np.nonzero(self.cpart == a)[0]
        lms = np.nonzero(self.lpart == a)[0]
        return cams, lms

    def system(self, a, x, y, lin_y):
        """Model Hessian H and gradient g of E^a(. | y) at x in a's tangent
        coordinates: cameras of a (9 each, ascending id) then landmarks of a
        (3 each, ascending id)."""
        cams, lms = self.unknowns(a)
        nc, nl = cams.size, lms.size
        n = 9 * nc + 3 * nl
        cpos = -np.ones(self.M, np.int64)
        cpos[cams] = 9 * np.arange(nc)
        lpos = -np.ones(self.N, np.int64)
        lpos[lms] = 9 * nc + 3 * np.arange(nl)
        H = np.zeros((n, n))
        g = np.zeros(n)
        # pairs of E' inside a: F_ij = rho(|e|^2) / 2, gradient rho' J^T e, model rho' J^T J
        sel = np.nonzero(self.intra & (self.oc == a))[0]
        if sel.size:
            q, Jc, Jl = self.residual_jacobian(x, sel)
            J = np.concatenate([Jc, Jl], axis=2)
            idx = np.concatenate([cpos[self.cam[sel]][:, None] + np.arange(9),
                                  lpos[self.lmk[sel]][:, None] + np.arange(3)], axis=1)
            w = q["w"]
            np.add.at(H, (idx[:, :, None], idx[:, None, :]), w[:, None, None] * np.einsum("kra,krb->kab", J, J))
            np.add.at(g, idx, w[:, None] * np.einsum("kra,kr->ka", J, q["e"]))
        # cameras of a in pairs of E'': P_ij
        sel = np.nonzero(~self.intra & (self.oc == a))[0]
        if sel.size:
            r, J = self.P_jacobian(lin_y, x, sel)
            idx = cpos[self.cam[sel]][:, None] + np.arange(9)
            w2 = 2.0 * lin_y["w"][sel]
            np.add.at(H, (idx[:, :, None], idx[:, None, :]), w2[:, None, None] * np.einsum("kra,krb->kab", J, J))
            np.add.at(g, idx, w2[:, None] * np.einsum("kra,kr->ka", J, r))
        # landmarks of a in pairs of E'': Q_ij
        sel = np.nonzero(~self.intra & (self.ol == a))[0]
        if sel.size:
            lam, gg, w = lin_y["lam"][sel], lin_y["g"][sel], lin_y["w"][sel]
            idx = lpos[self.lmk[sel]][:, None] + np.arange(3)
            v = lam[:, None] * x[3][self.lmk[sel]] - gg
            np.add.at(H, (idx, idx), (2.0 * w * lam * lam)[:, None] * np.ones(3))
            np.add.at(g, idx, (2.0 * w * lam)[:, None] * v)
        # proximal term (P4)
        H[np.arange(n), np.arange(n)] += self.xi
        R, t, d, l = x
        Ry, ty, dy, ly = y
        A = np.transpose(Ry[cams], (0, 2, 1)) @ R[cams]  # Y^T R
        grot = -self.xi * np.stack([A[:, 1, 2] - A[:, 2, 1], A[:, 2, 0] - A[:, 0, 2], A[:, 0, 1] - A[:, 1, 0]],
                                   axis=1)
        gc = np.concatenate([grot, self.xi * (t[cams] - ty[cams]), self.xi * (d[cams] - dy[cams])], axis=1)
        g[:9 * nc] += gc.reshape(-1)
        g[9 * nc:] += (self.xi * (l[lms] - ly[lms])).reshape(-1)
        return H, g, cams, lms

    def retract(self, x, cams, lms, delta):
        """x with a's cameras and landmarks moved by the tangent step delta."""
        R, t, d, l = (a.copy() for a in x)
        nc = cams.size
        dc = delta[:9 * nc].reshape(nc, 9)
        R[cams] = R[cams] @ so3_exp(dc[:, 0:3])
        t[cams] += dc[:, 3:6]
        d[cams] += dc[:, 6:9]
        l[lms] += delta[9 * nc:].reshape(-1, 3)
        return R, t, d, l

    def lm_partition(self, a, y, lin_y):
        """argmin of E^a(. | y) by P2's Levenberg-Marquardt from y; returns
        the new state (only a's entities differ from y) and the accepted step
        count."""
        x = y
        phi = self.surrogate(x, y, lin_y)[a]
        mu, succ, rej = 1e-4, 0, 0
        while succ < self.inner_steps:
            H, g, cams, lms = self.system(a, x, y, lin_y)
            Ad = H + mu * np.diag(np.diag(H))
            try:
                L = np.linalg.cholesky(Ad)
                step = -np.linalg.solve(L.T, np.linalg.solve(L, g))
                ok = True
            except np.linalg.LinAlgError:
                ok = False
            if ok:
                cand = self.retract(x, cams, lms, step)
                phic = self.surrogate(cand, y, lin_y)[a]
            if ok and phic < phi:
                x, phi = cand, phic
                mu /= 10.0
                succ += 1
                rej = 0
            else:
                mu *= 10.0
                rej += 1
                if rej >= 10:
                    break
        return x, succ

    def minimize(self, y, lin_y):
        """eq. update_mm / update_amm: every partition's LM from y."""
        R, t, d, l = (a.copy() for a in y)
        for a in range(self.S):
            xa, _ = self.lm_partition(a, y, lin_y)
            cams, lms = self.unknowns(a)
            R[cams], t[cams], d[cams], l[lms] = xa[0][cams], xa[1][cams], xa[2][cams], xa[3][lms]
        return R, t, d, l

    # ---- Algorithm 1
    def objective(self, x=None) -> float:
        """F in caller units (pixels^2)."""
        return float(np.sum(self.obs(self.x if x is None else x)["F"])) * self.s_unit ** 2

    def iterate(self, n: int):
        """n iterations; returns F after each (pixels^2) and the metrics
        (F^a(k), Fbar^a(k), E^a(k+1), restarted) per iteration and partition,
        in pixels^2."""
        S, s2 = self.S, self.s_unit ** 2
        Ftr = np.empty(n)
        mt = np.empty((n, S, 4))
        for it in range(n):
            snext = (np.sqrt(4.0 * self.s_nes ** 2 + 1.0) + 1.0) / 2.0  # eq. nesterov_scalar
            gam = (self.s_nes - 1.0) / snext if self.accelerate else np.zeros(S)
            self.s_nes = snext
            R, t, d, l = self.x
            Rp, tp, dp, lp = self.x_prev
            gc, gl = gam[self.cpart], gam[self.lpart]
            xbar = (projrot3d(R + gc[:, None, None] * (R - Rp)),  # eq. nesterov_R
                    t + gc[:, None] * (t - tp), d + gc[:, None] * (d - dp), l + gl[:, None] * (l - lp))
            lin_prev = self.linearize(self.x_prev)
            Fk = self.E + self.gap(self.x, self.x_prev, lin_prev)  # eq. Fak
            self.Fbar = (1.0 - self.eta) * self.Fbar + self.eta * Fk  # eq. lFak
            lin_k = self.linearize(self.x)
            x_mm = self.minimize(self.x, lin_k)
            x_acc = self.minimize(xbar, self.linearize(xbar)) if self.accelerate else None
            Ecur = self.surrogate(self.x, self.x, lin_k)
            Emm = self.surrogate(x_mm, self.x, lin_k)
            restart = np.ones(S, dtype=bool)
            Enew = Emm + Fk - Ecur  # eq. Eak
            if self.accelerate:
                Eacc = self.surrogate(x_acc, self.x, lin_k)
                Ehat = Eacc + Fk - Ecur
                restart = Ehat > self.Fbar
                if self.flags & NEVER_RESTART:
                    restart[:] = False
                if self.flags & ALWAYS_RESTART:
                    restart[:] = True
                Enew = np.where(restart, Enew, Ehat)
            self.E = Enew
            self.x_prev = self.x
            take_acc_c = ~restart[self.cpart] if self.accelerate else np.zeros(self.M, bool)
            take_acc_l = ~restart[self.lpart] if self.accelerate else np.zeros(self.N, bool)
            src_c = x_acc if self.accelerate else x_mm
            self.x = (np.where(take_acc_c[:, None, None], src_c[0], x_mm[0]),
                      np.where(take_acc_c[:, None], src_c[1], x_mm[1]),
                      np.where(take_acc_c[:, None], src_c[2], x_mm[2]),
                      np.where(take_acc_l[:, None], (x_acc if self.accelerate else x_mm)[3], x_mm[3]))
            mt[it, :, 0] = s2 * Fk
            mt[it, :, 1] = s2 * self.Fbar
            mt[it, :, 2] = s2 * self.E
            mt[it, :, 3] = restart
            self.Fprev = Fk
            self.k += 1
            Ftr[it] = self.objective()
        return Ftr, mt

    def get_state(self):
        """cams [M,15] and lms [N,3] of x^k, caller units."""
        return self._cams_out(*self.x[:3]), self.x[3].copy()
