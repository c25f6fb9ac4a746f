// Per-observation evaluation of Problem 1's residual (Sec. III) on gfx950,
// shared by the iteration's kernels and the objective entry point that
// allocates nothing.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace daba {

template <typename R>
struct CamT {
    R r[9], t[3], d[3];
};

template <typename R>
__device__ __forceinline__ CamT<R> load_cam(const double* __restrict__ c) {
    CamT<R> o;
#pragma unroll
    for (int a = 0; a < 9; ++a) o.r[a] = (R)c[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.t[a] = (R)c[9 + a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.d[a] = (R)c[12 + a];
    return o;
}

// Robust loss of Assumption 1 (Huber / Welsch widths in internal units).
template <int LOSS, typename R>
__device__ __forceinline__ R loss_rho(R s, R delta, R& w) {
    if constexpr (LOSS == 1) {
        if (s <= delta * delta) {
            w = (R)1;
            return s;
        }
        R rs = sqrt(s);
        w = delta / rs;
        return (R)2 * delta * rs - delta * delta;
    } else if constexpr (LOSS == 2) {
        R d2 = delta * delta;
        R ex = exp(-s / d2);
        w = ex;
        return d2 * ((R)1 - ex);
    } else {
        w = (R)1;
        return s;
    }
}

// One observation at camera c and landmark l (Sec. III): the rotated ray Rp,
// m = l - t, the depth scalar lambda (eq. lambdaij), the world-frame residual
// e_w = R p - lambda m (= R e of eq. error), |e|^2, the weight w = rho' and rho.
template <int LOSS, typename R>
struct ObsEval {
    R Rp[3], m[3], lam, e[3], s, w, rho, r2;
};

template <int LOSS, typename R>
__device__ __forceinline__ void eval_obs(const CamT<R>& c, R l0, R l1, R l2, R ux, R uy, R r2u, R r4u, R delta,
                                         ObsEval<LOSS, R>& o) {
    R pz = c.d[0] + c.d[1] * r2u + c.d[2] * r4u;
#pragma unroll
    for (int a = 0; a < 3; ++a) o.Rp[a] = c.r[3 * a] * ux + c.r[3 * a + 1] * uy + c.r[3 * a + 2] * pz;
    o.m[0] = l0 - c.t[0];
    o.m[1] = l1 - c.t[1];
    o.m[2] = l2 - c.t[2];
    o.r2 = o.m[0] * o.m[0] + o.m[1] * o.m[1] + o.m[2] * o.m[2];
    R inv = (R)1 / o.r2;
    o.lam = (o.m[0] * o.Rp[0] + o.m[1] * o.Rp[1] + o.m[2] * o.Rp[2]) * inv;
#pragma unroll
    for (int a = 0; a < 3; ++a) o.e[a] = o.Rp[a] - o.lam * o.m[a];
    o.s = o.e[0] * o.e[0] + o.e[1] * o.e[1] + o.e[2] * o.e[2];
    o.rho = loss_rho<LOSS, R>(o.s, delta, o.w);
}

// eq. error written out in the camera frame for any 3x3 R (the form the
// objective and its gradient are defined on): n = R^T (l - t),
// lambda = n . p / |l - t|^2, e = p - lambda n.  On SO(3) it equals R^T e_w.
template <int LOSS, typename R>
struct ObsEvalCF {
    R p[3], m[3], n[3], lam, e[3], s, w, rho, r2;
};

template <int LOSS, typename R>
__device__ __forceinline__ void eval_obs_cf(const CamT<R>& c, R l0, R l1, R l2, R ux, R uy, R r2u, R r4u,
                                            R delta, ObsEvalCF<LOSS, R>& o) {
    o.p[0] = ux;
    o.p[1] = uy;
    o.p[2] = c.d[0] + c.d[1] * r2u + c.d[2] * r4u;
    o.m[0] = l0 - c.t[0];
    o.m[1] = l1 - c.t[1];
    o.m[2] = l2 - c.t[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.n[a] = c.r[a] * o.m[0] + c.r[3 + a] * o.m[1] + c.r[6 + a] * o.m[2];
    o.r2 = o.m[0] * o.m[0] + o.m[1] * o.m[1] + o.m[2] * o.m[2];
    o.lam = (o.n[0] * o.p[0] + o.n[1] * o.p[1] + o.n[2] * o.p[2]) / o.r2;
#pragma unroll
    for (int a = 0; a < 3; ++a) o.e[a] = o.p[a] - o.lam * o.n[a];
    o.s = o.e[0] * o.e[0] + o.e[1] * o.e[1] + o.e[2] * o.e[2];
    o.rho = loss_rho<LOSS, R>(o.s, delta, o.w);
}

}  // namespace daba
