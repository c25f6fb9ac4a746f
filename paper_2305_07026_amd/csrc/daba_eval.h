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

// 1/x for a positive normal x, without the IEEE division sequence (its
// range scaling and fix-up are not needed for the squared distances of an
// observation): in FP32 the hardware reciprocal (about 1 ulp); in FP64 the
// hardware estimate refined by two Newton steps y <- y + y (1 - x y), each
// of which squares the relative error, to a few ulp.
template <typename R>
__device__ __forceinline__ R recip(R x);
template <>
__device__ __forceinline__ float recip<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double recip<double>(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// sqrt(s) and 1/sqrt(s) together for a positive normal s.  FP32: the
// hardware reciprocal square root (about 1 ulp).  FP64: from the hardware
// estimate y, g = s y -> sqrt(s) and h = y / 2 -> 1 / (2 sqrt(s)) refined
// together by two coupled Newton steps on the residual 1/2 - g h.
template <typename R>
__device__ __forceinline__ void sqrt_rsqrt(R s, R& rs, R& irs);
template <>
__device__ __forceinline__ void sqrt_rsqrt<float>(float s, float& rs, float& irs) {
    irs = __builtin_amdgcn_rsqf(s);
    rs = s * irs;
}
template <>
__device__ __forceinline__ void sqrt_rsqrt<double>(double s, double& rs, double& irs) {
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    rs = fma(g, e, g);
    irs = 2.0 * fma(h, e, h);
}

// The loss of loss_rho for the iteration's per-observation passes, with the
// Huber branch's square root and division taken by sqrt_rsqrt.
template <int LOSS, typename R>
__device__ __forceinline__ R loss_rho_iter(R s, R delta, R& w) {
    if constexpr (LOSS == 1) {
        if (s <= delta * delta) {
            w = (R)1;
            return s;
        }
        R rs, irs;
        sqrt_rsqrt<R>(s, rs, irs);
        w = delta * irs;
        return (R)2 * delta * rs - delta * delta;
    } else {
        return loss_rho<LOSS, R>(s, delta, w);
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
    const R inv = recip<R>(o.r2);
    o.lam = (o.m[0] * o.Rp[0] + o.m[1] * o.Rp[1] + o.m[2] * o.Rp[2]) * inv;
#pragma unroll
    for (int a = 0; a < 3; ++a) o.e[a] = o.Rp[a] - o.lam * o.m[a];
    o.s = o.e[0] * o.e[0] + o.e[1] * o.e[1] + o.e[2] * o.e[2];
    o.rho = loss_rho_iter<LOSS, R>(o.s, delta, o.w);
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
