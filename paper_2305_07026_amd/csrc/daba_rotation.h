// Rotation helpers shared by the device code of the DABA library: Exp on
// SO(3) and the nearest rotation of eq. proj_rot3d.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace daba {

// Rodrigues formula for Exp of the skew matrix of w (Taylor below 1e-8 rad)
__device__ __forceinline__ void exp_so3(const double* w, double* E) {
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double A, B;
    if (th < 1e-8) {
        A = 1.0;
        B = 0.5;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double k2 = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
            E[3 * r + c] = (r == c ? 1.0 : 0.0) + A * K[3 * r + c] + B * k2;
        }
}


// ------------------------------------------- nearest rotation (eq. proj_rot3d)
// For det(M) > 0 the nearest rotation is the orthogonal polar factor of M,
// reached by Newton's iteration X <- (X + X^-T) / 2 (quadratic convergence;
// extrapolated rotations are close to orthogonal, so a few steps suffice).
__device__ inline bool polar_rotation(const double* M, double* R) {
    double X[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) X[a] = M[a];
    for (int it = 0; it < 16; ++it) {
        // cofactors of X: X^-T = cof(X) / det(X)
        double C[9];
        C[0] = X[4] * X[8] - X[5] * X[7];
        C[1] = X[5] * X[6] - X[3] * X[8];
        C[2] = X[3] * X[7] - X[4] * X[6];
        C[3] = X[2] * X[7] - X[1] * X[8];
        C[4] = X[0] * X[8] - X[2] * X[6];
        C[5] = X[1] * X[6] - X[0] * X[7];
        C[6] = X[1] * X[5] - X[2] * X[4];
        C[7] = X[2] * X[3] - X[0] * X[5];
        C[8] = X[0] * X[4] - X[1] * X[3];
        const double det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
        if (!(det > 0.0)) return false;
        const double id = 1.0 / det;
        double ch = 0.0;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double y = 0.5 * (X[a] + C[a] * id);
            ch += (y - X[a]) * (y - X[a]);
            X[a] = y;
        }
        if (ch <= 1e-30) {
#pragma unroll
            for (int a = 0; a < 9; ++a) R[a] = X[a];
            return true;
        }
    }
    return false;
}

// General case (any det): argmax over unit quaternions q of q^T K q with K the 4x4 symmetric matrix
// for which tr(R(q)^T M) = q^T K q (Bar-Itzhack's quaternion form of the
// nearest-rotation problem); the top eigenvector comes from cyclic Jacobi.
__device__ inline void nearest_rotation(const double* M, double* R) {
    double K[4][4];
    K[0][0] = M[0] + M[4] + M[8];
    K[1][1] = M[0] - M[4] - M[8];
    K[2][2] = -M[0] + M[4] - M[8];
    K[3][3] = -M[0] - M[4] + M[8];
    K[0][1] = K[1][0] = M[7] - M[5];
    K[0][2] = K[2][0] = M[2] - M[6];
    K[0][3] = K[3][0] = M[3] - M[1];
    K[1][2] = K[2][1] = M[1] + M[3];
    K[1][3] = K[3][1] = M[2] + M[6];
    K[2][3] = K[3][2] = M[5] + M[7];
    double V[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = 0.0, dg = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            dg += K[i][i] * K[i][i];
#pragma unroll
            for (int j = i + 1; j < 4; ++j) off += K[i][j] * K[i][j];
        }
        // off-diagonal at the rounding level of the diagonal
        if (off <= 1e-30 * dg) break;
#pragma unroll
        for (int pp = 0; pp < 3; ++pp)
#pragma unroll
            for (int qq = pp + 1; qq < 4; ++qq) {
                const double apq = K[pp][qq];
                // symmetric Schur decomposition of the (pp, qq) 2x2 block
                double cs = 1.0, sn = 0.0;
                if (apq != 0.0) {
                    double tau = (K[qq][qq] - K[pp][pp]) / (2.0 * apq);
                    double tt = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                             : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                    cs = 1.0 / sqrt(1.0 + tt * tt);
                    sn = tt * cs;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double kp = K[r][pp], kq = K[r][qq];
                    K[r][pp] = cs * kp - sn * kq;
                    K[r][qq] = sn * kp + cs * kq;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double kp = K[pp][r], kq = K[qq][r];
                    K[pp][r] = cs * kp - sn * kq;
                    K[qq][r] = sn * kp + cs * kq;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double vp = V[r][pp], vq = V[r][qq];
                    V[r][pp] = cs * vp - sn * vq;
                    V[r][qq] = sn * vp + cs * vq;
                }
            }
    }
    double bl = K[0][0], w = V[0][0], x = V[1][0], yq = V[2][0], z = V[3][0];
#pragma unroll
    for (int i = 1; i < 4; ++i)
        if (K[i][i] > bl) {
            bl = K[i][i];
            w = V[0][i];
            x = V[1][i];
            yq = V[2][i];
            z = V[3][i];
        }
    double nq = 1.0 / sqrt(w * w + x * x + yq * yq + z * z);
    w *= nq; x *= nq; yq *= nq; z *= nq;
    R[0] = w * w + x * x - yq * yq - z * z;
    R[1] = 2.0 * (x * yq - w * z);
    R[2] = 2.0 * (x * z + w * yq);
    R[3] = 2.0 * (x * yq + w * z);
    R[4] = w * w - x * x + yq * yq - z * z;
    R[5] = 2.0 * (yq * z - w * x);
    R[6] = 2.0 * (x * z - w * yq);
    R[7] = 2.0 * (yq * z + w * x);
    R[8] = w * w - x * x - yq * yq + z * z;
}

}  // namespace daba
