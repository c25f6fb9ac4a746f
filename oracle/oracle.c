/*
 * Plain CPU FP64 oracle of the DABA iteration.  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the GPU library.  See oracle.h for the map from functions to the
 * paper's equations.
 *
 * Readings taken where the paper is silent or ambiguous:
 *  R1  Every observation is majorized by P_ij + Q_ij (Prop. 1), so the
 *      surrogate splits per camera and per landmark ("entity level").  The S
 *      camera partitions play the paper's devices for the adaptive-restart
 *      bookkeeping of Sec. V: each has its own F^a, Fbar^a, E^a, s^a and
 *      restart decision.
 *  R2  Partition a owns cameras C_a and landmarks L_a.  E^a(x | y) = prox of
 *      a's variables + sum over i in C_a of P_ij + sum over j in L_a of Q_ij.
 *      The gap of eq. DEalpha gives each observation weight
 *      c^a_ij = 1/2 [i in C_a] + 1/2 [j in L_a], the paper's 1/2 per side for
 *      pairs split between devices and the full gap for pairs inside one.
 *  R3  Defaults: camera i is in partition floor(i / ceil(M/S)); landmark j is
 *      in the partition of the lowest camera id observing it.
 *  R4  A camera's subproblem is solved by Levenberg-Marquardt in tangent
 *      coordinates (dtheta, dt, dd), R <- R Exp(dtheta): model Hessian
 *      2 sum w J^T J + xi I9, damping mu diag(H) with mu0 = 1e-4, accept iff
 *      the exact surrogate strictly decreases (then mu /= 10), else mu *= 10
 *      and retry, giving up after 10 rejects in a row; stop after
 *      inner_steps accepted steps (the paper uses one successful inner step,
 *      Sec. VII-B); inner_steps <= 0 iterates to convergence.
 *  R5  A landmark's subproblem has the closed form
 *      l = (2 sum w lambda g + xi l^y) / (2 sum w lambda^2 + xi)
 *      (set the gradient of sum Q_ij + xi/2 |l - l^y|^2 to zero).
 *  R6  The proximal norm is Frobenius on R and Euclidean on t, d, l.
 *  R7  Internal units are pixels / s: u -> u/s, d -> (d1/s, d2 s, d3 s^3),
 *      loss width -> delta/s; F in pixels^2 is s^2 times F internal.
 *  R8  Restart test is strict (E^a(k+1) > Fbar^a(k)); s^a is never reset.
 *  R9  Loss widths: Huber rho(s) = s for s <= delta^2 else 2 delta sqrt(s) -
 *      delta^2; Welsch rho(s) = delta^2 (1 - exp(-s/delta^2)).
 *  R10 The intrinsics row of eq. DFij is transposed in the paper: the
 *      gradient of F_ij w.r.t. d is rho' e_z (1, |u|^2, |u|^4).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS2 1e-24

typedef struct { double R[9], t[3], d[3]; } ocam;
/* quantities frozen at a linearization point y (eq. w, a, gamma, g) */
typedef struct { double w, lam, g[3], a; } olin;
typedef struct { double p[3], lam, e[3], s, rho, w, a, g[3], F; } oobs;

struct orc_state {
    int64_t M, N, K;
    int S;
    int32_t *cam, *lmk;
    double *u; /* internal units */
    int32_t *cpart, *lpart;
    int64_t *coff, *cobs, *loff, *lobs;
    int loss;
    double delta, xi, eta;
    int accelerate, inner_steps;
    uint64_t flags;
    int frozen;
    double scale;
    ocam *c, *cm1;
    double *l, *lm1;
    double *s, *Fbar, *E, *Fprev;
    int64_t k;
};

/* ---------------------------------------------------------------- helpers */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void matvec(const double *R, const double *v, double *o) {
    for (int r = 0; r < 3; ++r) o[r] = R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
}
static void matTvec(const double *R, const double *v, double *o) {
    for (int r = 0; r < 3; ++r) o[r] = R[r] * v[0] + R[3 + r] * v[1] + R[6 + r] * v[2];
}
static void matmul(const double *A, const double *B, double *C) {
    double T[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) T[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
    memcpy(C, T, sizeof T);
}

static void cam_from_caller(const double *in, double s, ocam *c) {
    memcpy(c->R, in, 9 * sizeof(double));
    memcpy(c->t, in + 9, 3 * sizeof(double));
    c->d[0] = in[12] / s;
    c->d[1] = in[13] * s;
    c->d[2] = in[14] * s * s * s;
}
static void cam_to_caller(const ocam *c, double s, double *out) {
    memcpy(out, c->R, 9 * sizeof(double));
    memcpy(out + 9, c->t, 3 * sizeof(double));
    out[12] = c->d[0] * s;
    out[13] = c->d[1] / s;
    out[14] = c->d[2] / (s * s * s);
}
static void cam_from_internal15(const double *in, ocam *c) {
    memcpy(c->R, in, 9 * sizeof(double));
    memcpy(c->t, in + 9, 3 * sizeof(double));
    memcpy(c->d, in + 12, 3 * sizeof(double));
}
static void cam_to_internal15(const ocam *c, double *out) {
    memcpy(out, c->R, 9 * sizeof(double));
    memcpy(out + 9, c->t, 3 * sizeof(double));
    memcpy(out + 12, c->d, 3 * sizeof(double));
}

/* robust loss rho(s) and its derivative (Assumption 1; reading R9) */
static double loss_rho(const orc_state *st, double s, double *w) {
    double dl = st->delta / st->scale;
    switch (st->loss) {
    case ORC_LOSS_HUBER:
        if (s <= dl * dl) { *w = 1.0; return s; }
        *w = dl / sqrt(s);
        return 2.0 * dl * sqrt(s) - dl * dl;
    case ORC_LOSS_WELSCH: {
        double ex = exp(-s / (dl * dl));
        *w = ex;
        return dl * dl * (1.0 - ex);
    }
    default:
        *w = 1.0;
        return s;
    }
}

/* the ray p of eq. ray for intrinsics d and pixel u (internal units) */
static void ray(const double *d, const double *u, double *p) {
    double r2 = u[0] * u[0] + u[1] * u[1];
    p[0] = u[0];
    p[1] = u[1];
    p[2] = d[0] + d[1] * r2 + d[2] * r2 * r2;
}

/* Sec. III and Prop. 1: every per-observation quantity at (c, l). */
static int obs_eval(const orc_state *st, const ocam *c, const double *l, const double *u, oobs *o) {
    double m[3] = {l[0] - c->t[0], l[1] - c->t[1], l[2] - c->t[2]};
    double r2 = dot3(m, m);
    if (!(r2 > ORC_EPS2)) return -5; /* Assumption 2 violated */
    ray(c->d, u, o->p);
    double Rp[3], n[3];
    matvec(c->R, o->p, Rp);
    matTvec(c->R, m, n); /* R^T (l - t) */
    o->lam = dot3(m, Rp) / r2;               /* eq. lambdaij */
    double nTp = dot3(n, o->p);
    for (int a = 0; a < 3; ++a) o->e[a] = o->p[a] - n[a] * nTp / r2; /* eq. error */
    o->s = dot3(o->e, o->e);
    o->rho = loss_rho(st, o->s, &o->w);                            /* eq. w */
    o->a = 0.5 * o->rho - 0.5 * o->w * o->s;                        /* eq. a */
    for (int a = 0; a < 3; ++a) o->g[a] = 0.5 * Rp[a] + 0.5 * o->lam * c->t[a] + 0.5 * o->lam * l[a]; /* eq. g */
    o->F = 0.5 * o->rho;                                            /* eq. Fij */
    return 0;
}

/* eq. P: P_ij(c | y) with w, lambda, g, a frozen at y and p from c's d */
static double P_val(const olin *y, const ocam *c, const double *u) {
    double p[3], Rp[3], v[3];
    ray(c->d, u, p);
    matvec(c->R, p, Rp);
    for (int a = 0; a < 3; ++a) v[a] = Rp[a] + y->lam * c->t[a] - y->g[a];
    return y->w * dot3(v, v) + 0.5 * y->a;
}
/* eq. Q */
static double Q_val(const olin *y, const double *l) {
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = y->lam * l[a] - y->g[a];
    return y->w * dot3(v, v) + 0.5 * y->a;
}

static double cam_prox2(const ocam *c, const ocam *y) {
    double s = 0;
    for (int a = 0; a < 9; ++a) s += (c->R[a] - y->R[a]) * (c->R[a] - y->R[a]);
    for (int a = 0; a < 3; ++a) s += (c->t[a] - y->t[a]) * (c->t[a] - y->t[a]);
    for (int a = 0; a < 3; ++a) s += (c->d[a] - y->d[a]) * (c->d[a] - y->d[a]);
    return s;
}
static double lm_prox2(const double *l, const double *y) {
    double s = 0;
    for (int a = 0; a < 3; ++a) s += (l[a] - y[a]) * (l[a] - y[a]);
    return s;
}

/* frozen quantities of every observation at y = (cams, lms) */
static int linearize(const orc_state *st, const ocam *cams, const double *lms, olin *lin) {
    int err = 0;
#pragma omp parallel for schedule(static) reduction(min : err)
    for (int64_t o = 0; o < st->K; ++o) {
        oobs q;
        int r = obs_eval(st, &cams[st->cam[o]], &lms[3 * (int64_t)st->lmk[o]], &st->u[2 * o], &q);
        if (r) { err = r; continue; }
        lin[o].w = q.w;
        lin[o].lam = q.lam;
        memcpy(lin[o].g, q.g, sizeof q.g);
        lin[o].a = q.a;
    }
    return err;
}

/* ------------------------------------------------- rotations (eq. proj_rot3d) */

/* Exp of the skew matrix of w (Rodrigues), Taylor for tiny angles */
static void so3_exp(const double *w, double *E) {
    double th2 = dot3(w, w), th = sqrt(th2), A, B;
    if (th < 1e-8) {
        A = 1.0;
        B = 0.5;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0}, K2[9];
    matmul(K, K, K2);
    for (int a = 0; a < 9; ++a) E[a] = (a % 4 == 0 ? 1.0 : 0.0) + A * K[a] + B * K2[a];
}

/* cyclic Jacobi eigen-decomposition of a symmetric 3x3: A = V diag(ev) V^T */
static void jacobi3(const double *Ain, double *ev, double *V) {
    double A[9];
    memcpy(A, Ain, sizeof A);
    for (int a = 0; a < 9; ++a) V[a] = (a % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-30 * diag || off == 0.0) break; /* off-diagonal at rounding level */
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) { /* A <- J^T A J */
                    double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = c * akp - s * akq;
                    A[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = c * apk - s * aqk;
                    A[3 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = c * vkp - s * vkq;
                    V[3 * k + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int a = 0; a < 3; ++a) ev[a] = A[4 * a];
}

int orc_projrot3d(const double *M, double *R) {
    /* SVD M = U S V^T from the eigenvectors of M^T M; the closed form of the
     * nearest rotation is U diag(1, 1, det(U V^T)) V^T (Umeyama). */
    double MtM[9], ev[3], V[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) MtM[3 * r + c] = M[r] * M[c] + M[3 + r] * M[3 + c] + M[6 + r] * M[6 + c];
    jacobi3(MtM, ev, V);
    int ord[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a) /* descending singular values */
        for (int b = a + 1; b < 3; ++b)
            if (ev[ord[b]] > ev[ord[a]]) { int tmp = ord[a]; ord[a] = ord[b]; ord[b] = tmp; }
    double v[3][3], u[3][3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) v[a][k] = V[3 * k + ord[a]];
    /* u1 = M v1 / |M v1|, u2 = M v2 orthogonalised against u1, u3 = u1 x u2 */
    for (int a = 0; a < 2; ++a) {
        matvec(M, v[a], u[a]);
        if (a == 1) {
            double pr = dot3(u[1], u[0]);
            for (int k = 0; k < 3; ++k) u[1][k] -= pr * u[0][k];
        }
        double nn = sqrt(dot3(u[a], u[a]));
        if (!(nn > 0)) return -1; /* rank < 2: the projection is not unique */
        for (int k = 0; k < 3; ++k) u[a][k] /= nn;
    }
    u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
    u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
    u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    /* det(V) with V's columns v1, v2, v3 */
    double detV = v[0][0] * (v[1][1] * v[2][2] - v[1][2] * v[2][1]) - v[0][1] * (v[1][0] * v[2][2] - v[1][2] * v[2][0]) +
                  v[0][2] * (v[1][0] * v[2][1] - v[1][1] * v[2][0]);
    double sg[3] = {1.0, 1.0, detV >= 0 ? 1.0 : -1.0};
    /* U is proper by construction, so det(U V^T) = det(V) */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R[3 * r + c] = u[0][r] * v[0][c] * sg[0] + u[1][r] * v[1][c] * sg[1] + u[2][r] * v[2][c] * sg[2];
    return 0;
}

/* ------------------------------------------------ entity minimizers (R4, R5) */

static double cam_phi_lin(const orc_state *st, int64_t i, const olin *lin, const ocam *cy, const ocam *c) {
    double s = 0;
    for (int64_t q = st->coff[i]; q < st->coff[i + 1]; ++q) {
        int64_t o = st->cobs[q];
        s += P_val(&lin[o], c, &st->u[2 * o]);
    }
    return s + 0.5 * st->xi * cam_prox2(c, cy);
}

static double lm_phi_lin(const orc_state *st, int64_t j, const olin *lin, const double *ly, const double *l) {
    double s = 0;
    for (int64_t q = st->loff[j]; q < st->loff[j + 1]; ++q) s += Q_val(&lin[st->lobs[q]], l);
    return s + 0.5 * st->xi * lm_prox2(l, ly);
}

static void lm_min_lin(const orc_state *st, int64_t j, const olin *lin, const double *ly, double *out) {
    double num[3] = {st->xi * ly[0], st->xi * ly[1], st->xi * ly[2]}, den = st->xi;
    for (int64_t q = st->loff[j]; q < st->loff[j + 1]; ++q) {
        const olin *y = &lin[st->lobs[q]];
        for (int a = 0; a < 3; ++a) num[a] += 2.0 * y->w * y->lam * y->g[a];
        den += 2.0 * y->w * y->lam * y->lam;
    }
    for (int a = 0; a < 3; ++a) out[a] = num[a] / den;
}

static int chol_solve9(const double *Ain, const double *b, double *x) {
    double L[81];
    memset(L, 0, sizeof L);
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c <= r; ++c) {
            double s = Ain[9 * r + c];
            for (int k = 0; k < c; ++k) s -= L[9 * r + k] * L[9 * c + k];
            if (r == c) {
                if (!(s > 0)) return -1;
                L[9 * r + r] = sqrt(s);
            } else {
                L[9 * r + c] = s / L[9 * c + c];
            }
        }
    double y[9];
    for (int r = 0; r < 9; ++r) {
        double s = b[r];
        for (int k = 0; k < r; ++k) s -= L[9 * r + k] * y[k];
        y[r] = s / L[9 * r + r];
    }
    for (int r = 8; r >= 0; --r) {
        double s = y[r];
        for (int k = r + 1; k < 9; ++k) s -= L[9 * k + r] * x[k];
        x[r] = s / L[9 * r + r];
    }
    return 0;
}

/* Levenberg-Marquardt on one camera's share of E(. | y), reading R4. */
static void cam_min_lin(const orc_state *st, int64_t i, const olin *lin, const ocam *cy, int inner_steps, ocam *out,
                        int *nsucc) {
    ocam c = *cy;
    double phi = cam_phi_lin(st, i, lin, cy, &c);
    double mu = 1e-4;
    int succ = 0, rej = 0;
    for (;;) {
        if (inner_steps > 0 && succ >= inner_steps) break;
        if (inner_steps <= 0 && succ >= 100) break;
        double H[81], gr[9];
        memset(H, 0, sizeof H);
        memset(gr, 0, sizeof gr);
        for (int64_t q = st->coff[i]; q < st->coff[i + 1]; ++q) {
            int64_t o = st->cobs[q];
            const olin *y = &lin[o];
            const double *u = &st->u[2 * o];
            double p[3], Rp[3], r[3];
            ray(c.d, u, p);
            matvec(c.R, p, Rp);
            for (int a = 0; a < 3; ++a) r[a] = Rp[a] + y->lam * c.t[a] - y->g[a];
            double b[3] = {1.0, u[0] * u[0] + u[1] * u[1], 0};
            b[2] = b[1] * b[1];
            /* J = [ -R [p]x | lam I | (R e3) b^T ]  (3 x 9) */
            double px[9] = {0, -p[2], p[1], p[2], 0, -p[0], -p[1], p[0], 0}, Rpx[9];
            matmul(c.R, px, Rpx);
            double J[27];
            for (int rr = 0; rr < 3; ++rr) {
                for (int cc = 0; cc < 3; ++cc) J[9 * rr + cc] = -Rpx[3 * rr + cc];
                for (int cc = 0; cc < 3; ++cc) J[9 * rr + 3 + cc] = (rr == cc) ? y->lam : 0.0;
                for (int cc = 0; cc < 3; ++cc) J[9 * rr + 6 + cc] = c.R[3 * rr + 2] * b[cc];
            }
            for (int a = 0; a < 9; ++a) {
                for (int bb = 0; bb < 9; ++bb)
                    H[9 * a + bb] += 2.0 * y->w * (J[a] * J[bb] + J[9 + a] * J[9 + bb] + J[18 + a] * J[18 + bb]);
                gr[a] += 2.0 * y->w * (J[a] * r[0] + J[9 + a] * r[1] + J[18 + a] * r[2]);
            }
        }
        for (int a = 0; a < 9; ++a) H[10 * a] += st->xi;
        /* gradient of xi/2 |R - Ry|^2 + xi/2 |t - ty|^2 + xi/2 |d - dy|^2 */
        double Qm[9];
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc)
                Qm[3 * r + cc] = c.R[r] * cy->R[cc] + c.R[3 + r] * cy->R[3 + cc] + c.R[6 + r] * cy->R[6 + cc];
        gr[0] += -st->xi * (Qm[7] - Qm[5]);
        gr[1] += -st->xi * (Qm[2] - Qm[6]);
        gr[2] += -st->xi * (Qm[3] - Qm[1]);
        for (int a = 0; a < 3; ++a) gr[3 + a] += st->xi * (c.t[a] - cy->t[a]);
        for (int a = 0; a < 3; ++a) gr[6 + a] += st->xi * (c.d[a] - cy->d[a]);
        double A[81], rhs[9], dl[9];
        memcpy(A, H, sizeof A);
        for (int a = 0; a < 9; ++a) A[10 * a] += mu * H[10 * a];
        for (int a = 0; a < 9; ++a) rhs[a] = -gr[a];
        int ok = chol_solve9(A, rhs, dl) == 0;
        double phic = 0;
        ocam cand = c;
        if (ok) {
            double Ex[9];
            so3_exp(dl, Ex);
            matmul(c.R, Ex, cand.R);
            for (int a = 0; a < 3; ++a) cand.t[a] = c.t[a] + dl[3 + a];
            for (int a = 0; a < 3; ++a) cand.d[a] = c.d[a] + dl[6 + a];
            phic = cam_phi_lin(st, i, lin, cy, &cand);
        }
        if (ok && phic < phi) {
            double nd = 0, nx = 0;
            for (int a = 0; a < 9; ++a) nd += dl[a] * dl[a];
            for (int a = 0; a < 3; ++a) nx += c.t[a] * c.t[a] + c.d[a] * c.d[a];
            c = cand;
            phi = phic;
            mu /= 10.0;
            ++succ;
            rej = 0;
            if (inner_steps <= 0 && sqrt(nd) <= 1e-14 * (1.0 + sqrt(nx))) break;
        } else {
            mu *= 10.0;
            if (++rej >= 10) break;
        }
    }
    *out = c;
    if (nsucc) *nsucc = succ;
}

/* ------------------------------------------------------- surrogate (R1, R2) */

/* E^a(x | y) for every partition, by direct sums */
static void E_alpha(const orc_state *st, const olin *lin_y, const ocam *cy, const double *ly, const ocam *cx,
                    const double *lx, double *Eout, double *Pv, double *Qv) {
    int64_t K = st->K;
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < K; ++o) {
        Pv[o] = P_val(&lin_y[o], &cx[st->cam[o]], &st->u[2 * o]);
        Qv[o] = Q_val(&lin_y[o], &lx[3 * (int64_t)st->lmk[o]]);
    }
    for (int a = 0; a < st->S; ++a) Eout[a] = 0;
    for (int64_t i = 0; i < st->M; ++i) Eout[st->cpart[i]] += 0.5 * st->xi * cam_prox2(&cx[i], &cy[i]);
    for (int64_t j = 0; j < st->N; ++j) Eout[st->lpart[j]] += 0.5 * st->xi * lm_prox2(&lx[3 * j], &ly[3 * j]);
    for (int64_t o = 0; o < K; ++o) {
        Eout[st->cpart[st->cam[o]]] += Pv[o];
        Eout[st->lpart[st->lmk[o]]] += Qv[o];
    }
}

/* eq. DEalpha generalised by R2: DeltaE^a(x | y) */
static int dE_alpha(const orc_state *st, const olin *lin_y, const ocam *cy, const double *ly, const ocam *cx,
                    const double *lx, double *dEout, double *Pv, double *Qv, double *Fv) {
    int64_t K = st->K;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(min : err)
    for (int64_t o = 0; o < K; ++o) {
        oobs q;
        int r = obs_eval(st, &cx[st->cam[o]], &lx[3 * (int64_t)st->lmk[o]], &st->u[2 * o], &q);
        if (r) { err = r; continue; }
        Fv[o] = q.F;
        Pv[o] = P_val(&lin_y[o], &cx[st->cam[o]], &st->u[2 * o]);
        Qv[o] = Q_val(&lin_y[o], &lx[3 * (int64_t)st->lmk[o]]);
    }
    if (err) return err;
    for (int a = 0; a < st->S; ++a) dEout[a] = 0;
    for (int64_t i = 0; i < st->M; ++i) dEout[st->cpart[i]] -= 0.5 * st->xi * cam_prox2(&cx[i], &cy[i]);
    for (int64_t j = 0; j < st->N; ++j) dEout[st->lpart[j]] -= 0.5 * st->xi * lm_prox2(&lx[3 * j], &ly[3 * j]);
    for (int64_t o = 0; o < K; ++o) {
        double gap = Fv[o] - Pv[o] - Qv[o];
        dEout[st->cpart[st->cam[o]]] += 0.5 * gap;
        dEout[st->lpart[st->lmk[o]]] += 0.5 * gap;
    }
    return 0;
}

static int objective_int(const orc_state *st, const ocam *cx, const double *lx, const double *u, double *F) {
    int64_t K = st->K;
    double *Fv = malloc(sizeof(double) * (K > 0 ? K : 1));
    int err = 0;
#pragma omp parallel for schedule(static) reduction(min : err)
    for (int64_t o = 0; o < K; ++o) {
        oobs q;
        int r = obs_eval(st, &cx[st->cam[o]], &lx[3 * (int64_t)st->lmk[o]], &u[2 * o], &q);
        if (r) { err = r; continue; }
        Fv[o] = q.F;
    }
    double s = 0;
    for (int64_t o = 0; o < K; ++o) s += Fv[o];
    free(Fv);
    *F = s;
    return err;
}

/* ------------------------------------------------------------ public API */

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

void orc_destroy(orc_state *st) {
    if (!st) return;
    free(st->cam); free(st->lmk); free(st->u); free(st->cpart); free(st->lpart);
    free(st->coff); free(st->cobs); free(st->loff); free(st->lobs);
    free(st->c); free(st->cm1); free(st->l); free(st->lm1);
    free(st->s); free(st->Fbar); free(st->E); free(st->Fprev);
    free(st);
}

int orc_create(int64_t M, int64_t N, int64_t K, const int32_t *obs_cam, const int32_t *obs_lm, const double *uv,
               const double *cameras, const double *landmarks, int S, const int32_t *cam_part,
               const int32_t *lm_part, double unit_scale, int loss, double delta, double xi, double eta,
               int accelerate, int inner_steps, uint64_t flags, int frozen_partition, orc_state **out) {
    if (M <= 0 || N <= 0 || K < 0 || S <= 0 || !(unit_scale > 0) || !(xi > 0) || !(eta > 0) || eta > 1) return -1;
    orc_state *st = calloc(1, sizeof *st);
    st->M = M; st->N = N; st->K = K; st->S = S;
    st->loss = loss; st->delta = delta; st->xi = xi; st->eta = eta;
    st->accelerate = accelerate; st->inner_steps = inner_steps; st->flags = flags;
    st->frozen = frozen_partition; st->scale = unit_scale;
    size_t Kp = K > 0 ? (size_t)K : 1;
    st->cam = malloc(sizeof(int32_t) * Kp);
    st->lmk = malloc(sizeof(int32_t) * Kp);
    st->u = malloc(sizeof(double) * 2 * Kp);
    for (int64_t o = 0; o < K; ++o) {
        if (obs_cam[o] < 0 || obs_cam[o] >= M || obs_lm[o] < 0 || obs_lm[o] >= N) { orc_destroy(st); return -1; }
        st->cam[o] = obs_cam[o];
        st->lmk[o] = obs_lm[o];
        st->u[2 * o] = uv[2 * o] / unit_scale;
        st->u[2 * o + 1] = uv[2 * o + 1] / unit_scale;
    }
    /* observation lists per camera and per landmark, in input order */
    st->coff = calloc(M + 1, sizeof(int64_t));
    st->loff = calloc(N + 1, sizeof(int64_t));
    st->cobs = malloc(sizeof(int64_t) * Kp);
    st->lobs = malloc(sizeof(int64_t) * Kp);
    for (int64_t o = 0; o < K; ++o) { st->coff[st->cam[o] + 1]++; st->loff[st->lmk[o] + 1]++; }
    for (int64_t i = 0; i < M; ++i) st->coff[i + 1] += st->coff[i];
    for (int64_t j = 0; j < N; ++j) st->loff[j + 1] += st->loff[j];
    {
        int64_t *fc = malloc(sizeof(int64_t) * M), *fl = malloc(sizeof(int64_t) * N);
        memcpy(fc, st->coff, sizeof(int64_t) * M);
        memcpy(fl, st->loff, sizeof(int64_t) * N);
        for (int64_t o = 0; o < K; ++o) { st->cobs[fc[st->cam[o]]++] = o; st->lobs[fl[st->lmk[o]]++] = o; }
        free(fc); free(fl);
    }
    /* partitions (R3) */
    st->cpart = malloc(sizeof(int32_t) * M);
    st->lpart = malloc(sizeof(int32_t) * N);
    int64_t blk = (M + S - 1) / S;
    for (int64_t i = 0; i < M; ++i) {
        st->cpart[i] = cam_part ? cam_part[i] : (int32_t)(i / blk);
        if (st->cpart[i] < 0 || st->cpart[i] >= S) { orc_destroy(st); return -1; }
    }
    for (int64_t j = 0; j < N; ++j) {
        if (lm_part) {
            st->lpart[j] = lm_part[j];
        } else {
            int64_t best = -1;
            for (int64_t q = st->loff[j]; q < st->loff[j + 1]; ++q) {
                int64_t i = st->cam[st->lobs[q]];
                if (best < 0 || i < best) best = i;
            }
            st->lpart[j] = best < 0 ? 0 : st->cpart[best];
        }
        if (st->lpart[j] < 0 || st->lpart[j] >= S) { orc_destroy(st); return -1; }
    }
    st->c = malloc(sizeof(ocam) * M);
    st->cm1 = malloc(sizeof(ocam) * M);
    st->l = malloc(sizeof(double) * 3 * N);
    st->lm1 = malloc(sizeof(double) * 3 * N);
    for (int64_t i = 0; i < M; ++i) cam_from_caller(&cameras[15 * i], unit_scale, &st->c[i]);
    memcpy(st->l, landmarks, sizeof(double) * 3 * N);
    memcpy(st->cm1, st->c, sizeof(ocam) * M);
    memcpy(st->lm1, st->l, sizeof(double) * 3 * N);
    st->s = malloc(sizeof(double) * S);
    st->Fbar = malloc(sizeof(double) * S);
    st->E = malloc(sizeof(double) * S);
    st->Fprev = malloc(sizeof(double) * S);
    /* eq. Fainit: F^a(-1) = E^a(x^0 | x^0), Fbar^a(-1) = F^a(-1), E^a(0) = F^a(-1) */
    olin *lin = malloc(sizeof(olin) * Kp);
    double *Pv = malloc(sizeof(double) * Kp), *Qv = malloc(sizeof(double) * Kp);
    int err = linearize(st, st->c, st->l, lin);
    if (!err) E_alpha(st, lin, st->c, st->l, st->c, st->l, st->E, Pv, Qv);
    free(lin); free(Pv); free(Qv);
    if (err) { orc_destroy(st); return err; }
    for (int a = 0; a < S; ++a) {
        st->s[a] = 1.0;
        st->Fprev[a] = st->E[a];
        st->Fbar[a] = st->E[a];
    }
    st->k = 0;
    *out = st;
    return 0;
}

/* Steps 1-2 of an iteration (Sec. V): the Nesterov scalars of
 * eq. nesterov_scalar, s^(k+1) = (sqrt(4 s^(k)^2 + 1) + 1) / 2 and
 * gamma^(k) = (s^(k) - 1) / s^(k+1) (0 without acceleration), per partition;
 * then the extrapolated point of eq. nesterov_x, with the rotation
 * projected by eq. proj_rot3d.  s[] is advanced in place. */
static int nesterov_extrapolate(const orc_state *st, double *s, double *gam, ocam *cbar, double *lbar) {
    int err = 0;
    for (int a = 0; a < st->S; ++a) {
        double snext = (sqrt(4.0 * s[a] * s[a] + 1.0) + 1.0) / 2.0;
        gam[a] = st->accelerate ? (s[a] - 1.0) / snext : 0.0;
        s[a] = snext;
    }
#pragma omp parallel for schedule(static) reduction(min : err)
    for (int64_t i = 0; i < st->M; ++i) {
        double g = gam[st->cpart[i]], Mx[9];
        for (int a = 0; a < 9; ++a) Mx[a] = st->c[i].R[a] + g * (st->c[i].R[a] - st->cm1[i].R[a]);
        if (orc_projrot3d(Mx, cbar[i].R)) err = -5;
        for (int a = 0; a < 3; ++a) cbar[i].t[a] = st->c[i].t[a] + g * (st->c[i].t[a] - st->cm1[i].t[a]);
        for (int a = 0; a < 3; ++a) cbar[i].d[a] = st->c[i].d[a] + g * (st->c[i].d[a] - st->cm1[i].d[a]);
    }
    for (int64_t j = 0; j < st->N; ++j) {
        double g = gam[st->lpart[j]];
        for (int a = 0; a < 3; ++a) lbar[3 * j + a] = st->l[3 * j + a] + g * (st->l[3 * j + a] - st->lm1[3 * j + a]);
    }
    return err;
}

int orc_iterate(orc_state *st, int n, double *F_trace, double *metrics_trace) {
    int64_t M = st->M, N = st->N, K = st->K;
    int S = st->S;
    size_t Kp = K > 0 ? (size_t)K : 1;
    olin *lin_prev = malloc(sizeof(olin) * Kp), *lin_k = malloc(sizeof(olin) * Kp), *lin_bar = malloc(sizeof(olin) * Kp);
    double *Pv = malloc(sizeof(double) * Kp), *Qv = malloc(sizeof(double) * Kp), *Fv = malloc(sizeof(double) * Kp);
    ocam *cbar = malloc(sizeof(ocam) * M), *cacc = malloc(sizeof(ocam) * M), *cmm = malloc(sizeof(ocam) * M);
    double *lbar = malloc(sizeof(double) * 3 * N), *lacc = malloc(sizeof(double) * 3 * N), *lmm = malloc(sizeof(double) * 3 * N);
    double *gam = malloc(sizeof(double) * S), *Fk = malloc(sizeof(double) * S), *dE = malloc(sizeof(double) * S);
    double *Eacc = malloc(sizeof(double) * S), *Ecur = malloc(sizeof(double) * S), *Emm = malloc(sizeof(double) * S);
    int *restart = malloc(sizeof(int) * S);
    int err = 0;
    for (int it = 0; it < n && !err; ++it) {
        /* steps 1-2: Nesterov scalars and the extrapolated point */
        if ((err = nesterov_extrapolate(st, st->s, gam, cbar, lbar))) break;
        /* eq. Fak: F^a(k) = E^a(k) + DeltaE^a(x^k | x^(k-1)) */
        if ((err = linearize(st, st->cm1, st->lm1, lin_prev))) break;
        if ((err = dE_alpha(st, lin_prev, st->cm1, st->lm1, st->c, st->l, dE, Pv, Qv, Fv))) break;
        for (int a = 0; a < S; ++a) Fk[a] = st->E[a] + dE[a];
        /* eq. lFak */
        for (int a = 0; a < S; ++a) st->Fbar[a] = (1.0 - st->eta) * st->Fbar[a] + st->eta * Fk[a];
        /* candidates: eq. update_mm and eq. update_amm, per entity */
        if ((err = linearize(st, st->c, st->l, lin_k))) break;
        if (st->accelerate && (err = linearize(st, cbar, lbar, lin_bar))) break;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t i = 0; i < M; ++i) {
            cam_min_lin(st, i, lin_k, &st->c[i], st->inner_steps, &cmm[i], NULL);
            if (st->accelerate) cam_min_lin(st, i, lin_bar, &cbar[i], st->inner_steps, &cacc[i], NULL);
        }
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            lm_min_lin(st, j, lin_k, &st->l[3 * j], &lmm[3 * j]);
            if (st->accelerate) lm_min_lin(st, j, lin_bar, &lbar[3 * j], &lacc[3 * j]);
        }
        /* adaptive restart, eq. Eak and Algorithm 1 */
        E_alpha(st, lin_k, st->c, st->l, st->c, st->l, Ecur, Pv, Qv);
        E_alpha(st, lin_k, st->c, st->l, cmm, lmm, Emm, Pv, Qv);
        if (st->accelerate) E_alpha(st, lin_k, st->c, st->l, cacc, lacc, Eacc, Pv, Qv);
        for (int a = 0; a < S; ++a) {
            if (a == st->frozen) {
                restart[a] = 0;
                st->E[a] = Ecur[a] + Fk[a] - Ecur[a];
                continue;
            }
            if (!st->accelerate) {
                restart[a] = 1;
                st->E[a] = Emm[a] + Fk[a] - Ecur[a];
                continue;
            }
            double Ehat = Eacc[a] + Fk[a] - Ecur[a];
            int rs = Ehat > st->Fbar[a];
            if (st->flags & ORC_NEVER_RESTART) rs = 0;
            if (st->flags & ORC_ALWAYS_RESTART) rs = 1;
            restart[a] = rs;
            st->E[a] = rs ? Emm[a] + Fk[a] - Ecur[a] : Ehat;
        }
        /* roll x^(k-1) <- x^k, x^k <- x^(k+1) */
        memcpy(st->cm1, st->c, sizeof(ocam) * M);
        memcpy(st->lm1, st->l, sizeof(double) * 3 * N);
        for (int64_t i = 0; i < M; ++i) {
            int a = st->cpart[i];
            if (a == st->frozen) continue;
            st->c[i] = (st->accelerate && !restart[a]) ? cacc[i] : cmm[i];
        }
        for (int64_t j = 0; j < N; ++j) {
            int a = st->lpart[j];
            if (a == st->frozen) continue;
            memcpy(&st->l[3 * j], (st->accelerate && !restart[a]) ? &lacc[3 * j] : &lmm[3 * j], 3 * sizeof(double));
        }
        double s2 = st->scale * st->scale;
        if (metrics_trace)
            for (int a = 0; a < S; ++a) {
                double *mt = &metrics_trace[((int64_t)it * S + a) * 4];
                mt[0] = s2 * Fk[a];
                mt[1] = s2 * st->Fbar[a];
                mt[2] = s2 * st->E[a];
                mt[3] = restart[a];
            }
        for (int a = 0; a < S; ++a) st->Fprev[a] = Fk[a];
        st->k++;
        if (F_trace) {
            double F;
            if ((err = objective_int(st, st->c, st->l, st->u, &F))) break;
            F_trace[it] = s2 * F;
        }
    }
    free(lin_prev); free(lin_k); free(lin_bar); free(Pv); free(Qv); free(Fv);
    free(cbar); free(cacc); free(cmm); free(lbar); free(lacc); free(lmm);
    free(gam); free(Fk); free(dE); free(Eacc); free(Ecur); free(Emm); free(restart);
    return err;
}

static void load_x(const orc_state *st, const double *cams, const double *lms, ocam *c, double *l) {
    if (cams) for (int64_t i = 0; i < st->M; ++i) cam_from_caller(&cams[15 * i], st->scale, &c[i]);
    else memcpy(c, st->c, sizeof(ocam) * st->M);
    if (lms) memcpy(l, lms, sizeof(double) * 3 * st->N);
    else memcpy(l, st->l, sizeof(double) * 3 * st->N);
}

int orc_objective(orc_state *st, const double *cameras, const double *landmarks, const double *uv, double *F_out) {
    ocam *c = malloc(sizeof(ocam) * st->M);
    double *l = malloc(sizeof(double) * 3 * st->N);
    double *u = st->u;
    load_x(st, cameras, landmarks, c, l);
    if (uv) {
        u = malloc(sizeof(double) * 2 * (st->K > 0 ? st->K : 1));
        for (int64_t o = 0; o < 2 * st->K; ++o) u[o] = uv[o] / st->scale;
    }
    double F;
    int err = objective_int(st, c, l, u, &F);
    if (uv) free(u);
    free(c); free(l);
    if (!err) *F_out = st->scale * st->scale * F;
    return err;
}

/* App. D, eq. DFij (intrinsics row corrected, reading R10), and the pixel
 * gradient that follows from eq. ray and eq. error by the chain rule. */
int orc_grad(orc_state *st, const double *cameras, const double *landmarks, const double *uv, double *g_cams,
             double *g_lms, double *g_uv) {
    int64_t M = st->M, N = st->N, K = st->K;
    double sc = st->scale, s2 = sc * sc;
    ocam *c = malloc(sizeof(ocam) * M);
    double *l = malloc(sizeof(double) * 3 * N);
    double *u = st->u;
    load_x(st, cameras, landmarks, c, l);
    if (uv) {
        u = malloc(sizeof(double) * 2 * (K > 0 ? K : 1));
        for (int64_t o = 0; o < 2 * K; ++o) u[o] = uv[o] / sc;
    }
    double *gobs = malloc(sizeof(double) * 20 * (K > 0 ? K : 1)); /* R 9 | t 3 | d 3 | l 3 | u 2 */
    int err = 0;
#pragma omp parallel for schedule(static) reduction(min : err)
    for (int64_t o = 0; o < K; ++o) {
        const ocam *ci = &c[st->cam[o]];
        const double *lj = &l[3 * (int64_t)st->lmk[o]];
        const double *uo = &u[2 * o];
        oobs q;
        int r = obs_eval(st, ci, lj, uo, &q);
        if (r) { err = r; continue; }
        double m[3] = {lj[0] - ci->t[0], lj[1] - ci->t[1], lj[2] - ci->t[2]}, r2 = dot3(m, m);
        double *g = &gobs[20 * o];
        /* grad_R F = -rho' (m m^T / |m|^2) R (e p^T + p e^T) */
        double Sm[9], mmR[9], mm[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                Sm[3 * a + b] = q.e[a] * q.p[b] + q.p[a] * q.e[b];
                mm[3 * a + b] = m[a] * m[b] / r2;
            }
        matmul(mm, ci->R, mmR);
        matmul(mmR, Sm, g);
        for (int a = 0; a < 9; ++a) g[a] *= -q.w;
        /* grad_t F = rho' lambda R e,  grad_l F = -rho' lambda R e */
        double Re[3];
        matvec(ci->R, q.e, Re);
        for (int a = 0; a < 3; ++a) { g[9 + a] = q.w * q.lam * Re[a]; g[15 + a] = -q.w * q.lam * Re[a]; }
        /* grad_d F = rho' e_z b */
        double r2u = uo[0] * uo[0] + uo[1] * uo[1];
        g[12] = q.w * q.e[2];
        g[13] = q.w * q.e[2] * r2u;
        g[14] = q.w * q.e[2] * r2u * r2u;
        /* grad_u F = rho' (e_xy + e_z (2 d2 + 4 d3 |u|^2) u) */
        double dz = 2.0 * ci->d[1] + 4.0 * ci->d[2] * r2u;
        g[18] = q.w * (q.e[0] + q.e[2] * dz * uo[0]);
        g[19] = q.w * (q.e[1] + q.e[2] * dz * uo[1]);
    }
    if (!err) {
        if (g_cams) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < M; ++i) {
                double acc[15] = {0};
                for (int64_t q = st->coff[i]; q < st->coff[i + 1]; ++q)
                    for (int a = 0; a < 15; ++a) acc[a] += gobs[20 * st->cobs[q] + a];
                for (int a = 0; a < 12; ++a) g_cams[15 * i + a] = s2 * acc[a];
                g_cams[15 * i + 12] = s2 * acc[12] / sc;
                g_cams[15 * i + 13] = s2 * acc[13] * sc;
                g_cams[15 * i + 14] = s2 * acc[14] * sc * sc * sc;
            }
        }
        if (g_lms) {
#pragma omp parallel for schedule(static)
            for (int64_t j = 0; j < N; ++j) {
                double acc[3] = {0};
                for (int64_t q = st->loff[j]; q < st->loff[j + 1]; ++q)
                    for (int a = 0; a < 3; ++a) acc[a] += gobs[20 * st->lobs[q] + 15 + a];
                for (int a = 0; a < 3; ++a) g_lms[3 * j + a] = s2 * acc[a];
            }
        }
        if (g_uv)
            for (int64_t o = 0; o < K; ++o) {
                g_uv[2 * o] = s2 * gobs[20 * o + 18] / sc;
                g_uv[2 * o + 1] = s2 * gobs[20 * o + 19] / sc;
            }
    }
    free(gobs);
    if (uv) free(u);
    free(c); free(l);
    return err;
}

int orc_extrapolation(const orc_state *st, double *gamma_out, double *cams_bar, double *lms_bar) {
    double *s = malloc(sizeof(double) * st->S), *gam = malloc(sizeof(double) * st->S);
    ocam *cbar = malloc(sizeof(ocam) * (st->M > 0 ? st->M : 1));
    double *lbar = malloc(sizeof(double) * 3 * (st->N > 0 ? st->N : 1));
    memcpy(s, st->s, sizeof(double) * st->S);
    int err = nesterov_extrapolate(st, s, gam, cbar, lbar);
    if (!err) {
        if (gamma_out) memcpy(gamma_out, gam, sizeof(double) * st->S);
        if (cams_bar) for (int64_t i = 0; i < st->M; ++i) cam_to_caller(&cbar[i], st->scale, &cams_bar[15 * i]);
        if (lms_bar) memcpy(lms_bar, lbar, sizeof(double) * 3 * st->N);
    }
    free(s); free(gam); free(cbar); free(lbar);
    return err;
}

int orc_get_state(const orc_state *st, double *cams, double *lms, double *cams_prev, double *lms_prev, double *part4,
                  double *scalars2) {
    double s2 = st->scale * st->scale;
    if (cams) for (int64_t i = 0; i < st->M; ++i) cam_to_caller(&st->c[i], st->scale, &cams[15 * i]);
    if (lms) memcpy(lms, st->l, sizeof(double) * 3 * st->N);
    if (cams_prev) for (int64_t i = 0; i < st->M; ++i) cam_to_caller(&st->cm1[i], st->scale, &cams_prev[15 * i]);
    if (lms_prev) memcpy(lms_prev, st->lm1, sizeof(double) * 3 * st->N);
    if (part4) {
        /* E^a(x^k | x^(k-1)) by direct sums */
        size_t Kp = st->K > 0 ? (size_t)st->K : 1;
        olin *lin = malloc(sizeof(olin) * Kp);
        double *Pv = malloc(sizeof(double) * Kp), *Qv = malloc(sizeof(double) * Kp), *EE = malloc(sizeof(double) * st->S);
        int err = linearize(st, st->cm1, st->lm1, lin);
        if (!err) E_alpha(st, lin, st->cm1, st->lm1, st->c, st->l, EE, Pv, Qv);
        for (int a = 0; a < st->S; ++a) {
            part4[4 * a] = s2 * st->Fbar[a];
            part4[4 * a + 1] = s2 * st->E[a];
            part4[4 * a + 2] = err ? NAN : s2 * EE[a];
            part4[4 * a + 3] = s2 * st->Fprev[a];
        }
        free(lin); free(Pv); free(Qv); free(EE);
        if (err) return err;
    }
    if (scalars2) { scalars2[0] = st->s[0]; scalars2[1] = (double)st->k; }
    return 0;
}

int orc_set_state(orc_state *st, const double *cams, const double *lms, const double *cams_prev, const double *lms_prev,
                  const double *part4, const double *scalars2) {
    double s2 = st->scale * st->scale;
    if (cams) for (int64_t i = 0; i < st->M; ++i) cam_from_caller(&cams[15 * i], st->scale, &st->c[i]);
    if (lms) memcpy(st->l, lms, sizeof(double) * 3 * st->N);
    if (cams_prev) for (int64_t i = 0; i < st->M; ++i) cam_from_caller(&cams_prev[15 * i], st->scale, &st->cm1[i]);
    if (lms_prev) memcpy(st->lm1, lms_prev, sizeof(double) * 3 * st->N);
    if (part4)
        for (int a = 0; a < st->S; ++a) {
            st->Fbar[a] = part4[4 * a] / s2;
            st->E[a] = part4[4 * a + 1] / s2;
            st->Fprev[a] = part4[4 * a + 3] / s2;
        }
    if (scalars2) {
        for (int a = 0; a < st->S; ++a) st->s[a] = scalars2[0];
        st->k = (int64_t)scalars2[1];
    }
    return 0;
}

int orc_surrogate(orc_state *st, const double *cams_x, const double *lms_x, const double *cams_y, const double *lms_y,
                  double *E_out, double *dE_out) {
    int64_t M = st->M, N = st->N;
    size_t Kp = st->K > 0 ? (size_t)st->K : 1;
    ocam *cx = malloc(sizeof(ocam) * M), *cy = malloc(sizeof(ocam) * M);
    double *lx = malloc(sizeof(double) * 3 * N), *ly = malloc(sizeof(double) * 3 * N);
    load_x(st, cams_x, lms_x, cx, lx);
    load_x(st, cams_y, lms_y, cy, ly);
    olin *lin = malloc(sizeof(olin) * Kp);
    double *Pv = malloc(sizeof(double) * Kp), *Qv = malloc(sizeof(double) * Kp), *Fv = malloc(sizeof(double) * Kp);
    int err = linearize(st, cy, ly, lin);
    if (!err && E_out) E_alpha(st, lin, cy, ly, cx, lx, E_out, Pv, Qv);
    if (!err && dE_out) err = dE_alpha(st, lin, cy, ly, cx, lx, dE_out, Pv, Qv, Fv);
    double s2 = st->scale * st->scale;
    for (int a = 0; a < st->S && !err; ++a) {
        if (E_out) E_out[a] *= s2;
        if (dE_out) dE_out[a] *= s2;
    }
    free(cx); free(cy); free(lx); free(ly); free(lin); free(Pv); free(Qv); free(Fv);
    return err;
}

int orc_obs_eval(const orc_state *st, const double *c, const double *l, const double *u, double *out16) {
    ocam cc;
    cam_from_internal15(c, &cc);
    oobs q;
    int err = obs_eval(st, &cc, l, u, &q);
    if (err) return err;
    memcpy(out16, q.p, 3 * sizeof(double));
    out16[3] = q.lam;
    memcpy(out16 + 4, q.e, 3 * sizeof(double));
    out16[7] = q.s;
    out16[8] = q.rho;
    out16[9] = q.w;
    out16[10] = q.a;
    memcpy(out16 + 11, q.g, 3 * sizeof(double));
    out16[14] = q.F;
    out16[15] = 0;
    return 0;
}

int orc_PQ(const orc_state *st, const double *u, const double *cy, const double *ly, const double *c, const double *l,
           double *P, double *Q) {
    ocam ccy, cc;
    cam_from_internal15(cy, &ccy);
    cam_from_internal15(c, &cc);
    oobs q;
    int err = obs_eval(st, &ccy, ly, u, &q);
    if (err) return err;
    olin y = {q.w, q.lam, {q.g[0], q.g[1], q.g[2]}, q.a};
    *P = P_val(&y, &cc, u);
    *Q = Q_val(&y, l);
    return 0;
}

static olin *lin_from_internal(const orc_state *st, const double *cams_y, const double *lms_y, ocam **cy_out) {
    ocam *cy = malloc(sizeof(ocam) * st->M);
    for (int64_t i = 0; i < st->M; ++i) cam_from_internal15(&cams_y[15 * i], &cy[i]);
    olin *lin = malloc(sizeof(olin) * (st->K > 0 ? st->K : 1));
    if (linearize(st, cy, lms_y, lin)) { free(lin); free(cy); return NULL; }
    *cy_out = cy;
    return lin;
}

int orc_landmark_min(const orc_state *st, int64_t j, const double *cams_y, const double *lms_y, double *l_out) {
    ocam *cy;
    olin *lin = lin_from_internal(st, cams_y, lms_y, &cy);
    if (!lin) return -5;
    lm_min_lin(st, j, lin, &lms_y[3 * j], l_out);
    free(lin); free(cy);
    return 0;
}

int orc_camera_min(const orc_state *st, int64_t i, const double *cams_y, const double *lms_y, int inner_steps,
                   double *c_out, int *n_success) {
    ocam *cy;
    olin *lin = lin_from_internal(st, cams_y, lms_y, &cy);
    if (!lin) return -5;
    ocam out;
    cam_min_lin(st, i, lin, &cy[i], inner_steps, &out, n_success);
    cam_to_internal15(&out, c_out);
    free(lin); free(cy);
    return 0;
}

int orc_camera_phi(const orc_state *st, int64_t i, const double *cams_y, const double *lms_y, const double *c,
                   double *phi) {
    ocam *cy;
    olin *lin = lin_from_internal(st, cams_y, lms_y, &cy);
    if (!lin) return -5;
    ocam cc;
    cam_from_internal15(c, &cc);
    *phi = cam_phi_lin(st, i, lin, &cy[i], &cc);
    free(lin); free(cy);
    return 0;
}

int orc_landmark_phi(const orc_state *st, int64_t j, const double *cams_y, const double *lms_y, const double *l,
                     double *phi) {
    ocam *cy;
    olin *lin = lin_from_internal(st, cams_y, lms_y, &cy);
    if (!lin) return -5;
    *phi = lm_phi_lin(st, j, lin, &lms_y[3 * j], l);
    free(lin); free(cy);
    return 0;
}

int orc_cams_to_internal(const orc_state *st, const double *in, double *out, int64_t M) {
    for (int64_t i = 0; i < M; ++i) {
        ocam c;
        cam_from_caller(&in[15 * i], st->scale, &c);
        cam_to_internal15(&c, &out[15 * i]);
    }
    return 0;
}
