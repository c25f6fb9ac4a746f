// DABA with the device-level surrogate of eq. Ealpha on gfx950: pairs whose
// camera and landmark share a device are kept exact, pairs split between
// devices are majorized by P_ij + Q_ij (Prop. 1), and each device's
// subproblem is solved by Levenberg-Marquardt over all of its cameras and
// landmarks together (Sec. VII-B).  Devices are camera partitions of one GPU.
//
// One LM attempt, for every still-active partition at once:
//   kp_cam_build   one block per camera: Gauss-Newton blocks H_cc (9x9), g_c,
//                  and H_cl (9x3) of every exact pair, from the camera's
//                  observations (camera-major order);
//   kp_lm_build    one lane per landmark: H_ll (3x3), g_l, the damped inverse
//                  W = (H_ll + mu diag H_ll)^-1 and W g_l;
//   kp_rhs         one wave per camera: b_c = -g_c + sum H_cl W g_l;
//   kp_schur       one wave per lower 9x9 block of a partition's reduced
//                  camera system S = H_cc + mu diag - sum (H_cl W) H_cl^T,
//                  summed in a fixed order over a pair list built at create;
//   kp_chol_*      blocked right-looking Cholesky of every S (64x64 tiles):
//                  per step a panel solve and a trailing update, whose block
//                  for the next diagonal tile factors it in the same launch;
//   kp_trsv        L L^T dc = b per partition;
//   kp_step        dl = -W (g_l + sum H_cl^T dc) per landmark; retraction
//                  R Exp(dtheta), t + dt, d + dd, l + dl;
//   kp_eval + kp_reduce1/2   E^a at the trial point (fixed-order sums over
//                  chunks of each partition's observations);
//   kp_accept + kp_copy      strict-decrease test, damping update, and the
//                  accepted trial becomes the LM point.
// The host loops over attempts until every partition has its successful
// steps or gives up (one stream synchronization per attempt).
//
// One iteration (Algorithm 1): kp_nesterov and kp_extrap (x-bar), the gap of
// eq. DEalpha at (x^k | x^(k-1)) and eq. Fak / lFak (kp_fk), the LM solve of
// the accelerated surrogate for every partition, the restart test
// (kp_restart_test), the LM solve of the plain surrogate only for the
// partitions that fail it, eq. Eak for them (kp_restart_finish), kp_roll,
// and F at the new iterate (kp_trace).
// All FP64.  No atomics: results are bitwise reproducible.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "daba_part.h"
#include "daba_rotation.h"

namespace dpart {

constexpr int kW = 64;
constexpr int kNB = 64;          // Cholesky tile
constexpr int kMaxS = DABA_MAX_PARTITIONS;
constexpr int kCS = 16;          // doubles per camera record: R 9 | t 3 | d 3 | pad
constexpr int kLS = 4;           // doubles per landmark record
constexpr int kTraceCap = 4096;  // iterations per device F trace chunk

// per-partition scalars, kPS doubles each
enum {
    P_S = 0, P_GAM, P_FBAR, P_E, P_FK, P_ECUR, P_EMM, P_EACC, P_MU, P_PHI, P_ETRY, P_SUCC, P_REJ,
    P_ACTIVE, P_ACC, P_OK, P_RESTART, P_RED, kPS = 20
};
enum { EV_E = 0, EV_GAP = 1, EV_F = 2 };

struct PP {
    int M, N, S;
    int64_t K;
    int loss;
    double delta, xi, eta;
    int accelerate, inner_steps;
    uint64_t flags;
    int pc[kMaxS + 1], pl[kMaxS + 1];  // internal camera / landmark ranges of the partitions
    int nt[kMaxS];                     // Cholesky tiles of each partition's reduced system
    int npad[kMaxS];                   // its padded order (64 * nt)
    int64_t soff[kMaxS];               // offset of its matrix (doubles)
    int voff[kMaxS];                   // offset of its vector (doubles)
    int blkbase[kMaxS + 1];            // lower 9x9 blocks before each partition
    const int *ocam, *olm, *ointra;
    const double* ouv;
    const int *cam_off, *lm_off, *lm_obs;
    const int *seg_off, *ent;
    const int4* chunk;                 // reduction chunks: (kind, partition, begin, end)
    int chunk_base[kMaxS + 1];         // chunks of each partition
    double* partial;                   // one sum per chunk
    double *vc, *vl, *Hcl;
    double *Hcc, *gc, *W, *Wg;
    double *Smat, *vec;
    double* dinv;                      // 1 / L_rr of each factor, laid out like vec
    double* ps;
    double* trace;
    int* flag;
};
static_assert(sizeof(PP) <= 4096, "kernel arguments");

// ------------------------------------------------------------ device helpers

__device__ __forceinline__ int part_of(const int* starts, int S, int idx) {
    int a = 0;
    while (a + 1 < S && starts[a + 1] <= idx) ++a;
    return a;
}

__device__ __forceinline__ double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kW);
    return v;
}

template <int LOSS>
__device__ __forceinline__ double rho_w(double s, double dl, double& w) {
    if constexpr (LOSS == DABA_LOSS_HUBER) {
        if (s <= dl * dl) {
            w = 1.0;
            return s;
        }
        const double rs = sqrt(s);
        w = dl / rs;
        return 2.0 * dl * rs - dl * dl;
    } else if constexpr (LOSS == DABA_LOSS_WELSCH) {
        const double ex = exp(-s / (dl * dl));
        w = ex;
        return dl * dl * (1.0 - ex);
    } else {
        w = 1.0;
        return s;
    }
}

struct Cam {
    double R[9], t[3], d[3];
};

__device__ __forceinline__ Cam ld_cam(const double* c) {
    Cam o;
#pragma unroll
    for (int a = 0; a < 9; ++a) o.R[a] = c[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.t[a] = c[9 + a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.d[a] = c[12 + a];
    return o;
}

// Sec. III at camera c and landmark l: ray p (eq. ray), m = l - t,
// n = R^T m, lambda (eq. lambdaij), camera-frame residual e (eq. error),
// |e|^2, rho and rho'.  ok = false if |m|^2 <= 1e-24 (Assumption 2).
template <int LOSS>
struct Obs {
    double p[3], Rp[3], m[3], n[3], r2, lam, np, e[3], s, rho, w;
    bool ok;
};

template <int LOSS>
__device__ __forceinline__ void eval_obs(const Cam& c, const double* l, double ux, double uy, double dl, Obs<LOSS>& o) {
    const double r2u = ux * ux + uy * uy;
    o.p[0] = ux;
    o.p[1] = uy;
    o.p[2] = c.d[0] + c.d[1] * r2u + c.d[2] * r2u * r2u;
#pragma unroll
    for (int a = 0; a < 3; ++a) o.Rp[a] = c.R[3 * a] * o.p[0] + c.R[3 * a + 1] * o.p[1] + c.R[3 * a + 2] * o.p[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.m[a] = l[a] - c.t[a];
    o.r2 = o.m[0] * o.m[0] + o.m[1] * o.m[1] + o.m[2] * o.m[2];
    o.ok = o.r2 > 1e-24;
#pragma unroll
    for (int a = 0; a < 3; ++a) o.n[a] = c.R[a] * o.m[0] + c.R[3 + a] * o.m[1] + c.R[6 + a] * o.m[2];
    const double inv = 1.0 / o.r2;
    o.lam = (o.m[0] * o.Rp[0] + o.m[1] * o.Rp[1] + o.m[2] * o.Rp[2]) * inv;
    o.np = o.n[0] * o.p[0] + o.n[1] * o.p[1] + o.n[2] * o.p[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.e[a] = o.p[a] - o.n[a] * (o.np * inv);
    o.s = o.e[0] * o.e[0] + o.e[1] * o.e[1] + o.e[2] * o.e[2];
    o.rho = rho_w<LOSS>(o.s, dl, o.w);
}

// Quantities of Prop. 1 frozen at y: w, lambda, g (eq. g), a (eq. a).
struct Lin {
    double w, lam, g[3], a;
};

template <int LOSS>
__device__ __forceinline__ Lin lin_at(const Cam& cy, const double* ly, double ux, double uy, double dl, bool& ok) {
    Obs<LOSS> o;
    eval_obs<LOSS>(cy, ly, ux, uy, dl, o);
    Lin L;
    L.w = o.w;
    L.lam = o.lam;
#pragma unroll
    for (int a = 0; a < 3; ++a) L.g[a] = 0.5 * o.Rp[a] + 0.5 * o.lam * cy.t[a] + 0.5 * o.lam * ly[a];
    L.a = 0.5 * o.rho - 0.5 * o.w * o.s;
    ok = o.ok;
    return L;
}

// eq. P with camera c, eq. Q with landmark l
__device__ __forceinline__ double P_val(const Lin& y, const Cam& c, double ux, double uy) {
    const double r2u = ux * ux + uy * uy;
    const double pz = c.d[0] + c.d[1] * r2u + c.d[2] * r2u * r2u;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = c.R[3 * a] * ux + c.R[3 * a + 1] * uy + c.R[3 * a + 2] * pz + y.lam * c.t[a] - y.g[a];
        s += v * v;
    }
    return y.w * s + 0.5 * y.a;
}

__device__ __forceinline__ double Q_val(const Lin& y, const double* l) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = y.lam * l[a] - y.g[a];
        s += v * v;
    }
    return y.w * s + 0.5 * y.a;
}

// Row r of de/dn for e = (I - n n^T / |n|^2) p:
// -(n.p I + n p^T) / |n|^2 + 2 (n.p) n n^T / |n|^4.
template <int LOSS>
__device__ __forceinline__ void de_dn_row(const Obs<LOSS>& o, int r, double* D) {
    const double inv = 1.0 / o.r2;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        D[k] = -((r == k ? o.np : 0.0) + o.n[r] * o.p[k]) * inv + 2.0 * o.np * o.n[r] * o.n[k] * inv * inv;
}

// Row r of the residual's Jacobian for R <- R Exp(dtheta), t + dt, d + dd,
// l + dl: de/ddtheta = D [n]x (row: D x n), de/dt = -D R^T, de/dd =
// (I - n n^T / |n|^2) e3 b^T with b = (1, |u|^2, |u|^4), de/dl = D R^T.
// Jc gets the 9 camera entries, G the 3 landmark entries.
template <int LOSS>
__device__ __forceinline__ void jac_row(const Obs<LOSS>& o, const Cam& c, double r2u, int r, double* Jc, double* G) {
    double D[3];
    de_dn_row<LOSS>(o, r, D);
    Jc[0] = D[1] * o.n[2] - D[2] * o.n[1];
    Jc[1] = D[2] * o.n[0] - D[0] * o.n[2];
    Jc[2] = D[0] * o.n[1] - D[1] * o.n[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) G[k] = D[0] * c.R[3 * k] + D[1] * c.R[3 * k + 1] + D[2] * c.R[3 * k + 2];
#pragma unroll
    for (int k = 0; k < 3; ++k) Jc[3 + k] = -G[k];
    const double pz = (r == 2 ? 1.0 : 0.0) - o.n[r] * o.n[2] / o.r2;
    Jc[6] = pz;
    Jc[7] = pz * r2u;
    Jc[8] = pz * r2u * r2u;
}

__device__ __forceinline__ int tri_idx(int a, int b) {  // a <= b < 9, packed upper triangle
    return a * 9 - (a * (a - 1)) / 2 + (b - a);
}

// ------------------------------------------------------------------- kernels

__global__ __launch_bounds__(64) void kp_nesterov(PP p) {
    const int a = threadIdx.x;
    if (a >= p.S) return;
    double* q = p.ps + (size_t)a * kPS;
    const double s = q[P_S];
    const double sn = (sqrt(4.0 * s * s + 1.0) + 1.0) / 2.0;  // eq. nesterov_scalar
    q[P_GAM] = p.accelerate ? (s - 1.0) / sn : 0.0;
    q[P_S] = sn;
}

// eq. nesterov_x: x-bar = Proj(x + gamma (x - x_prev)), rotations by eq. proj_rot3d
__global__ __launch_bounds__(64) void kp_extrap(PP p, const double* xc, const double* pcam, const double* xl,
                                                const double* plm, double* bc, double* bl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < p.M) {
        const double g = p.ps[(size_t)part_of(p.pc, p.S, t) * kPS + P_GAM];
        const double* c = xc + (size_t)t * kCS;
        const double* o = pcam + (size_t)t * kCS;
        double Mx[9], Rb[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) Mx[a] = c[a] + g * (c[a] - o[a]);
        if (!daba::polar_rotation(Mx, Rb)) daba::nearest_rotation(Mx, Rb);
        double* out = bc + (size_t)t * kCS;
#pragma unroll
        for (int a = 0; a < 9; ++a) out[a] = Rb[a];
#pragma unroll
        for (int a = 9; a < 15; ++a) out[a] = c[a] + g * (c[a] - o[a]);
    } else if (t < p.M + p.N) {
        const int j = t - p.M;
        const double g = p.ps[(size_t)part_of(p.pl, p.S, j) * kPS + P_GAM];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = xl[(size_t)j * kLS + a];
            bl[(size_t)j * kLS + a] = v + g * (v - plm[(size_t)j * kLS + a]);
        }
    }
}

// Per-observation shares of E^a(x | y) (EV_E), of DeltaE^a(x | y) (EV_GAP) or
// of F(x) (EV_F): vc charged to the camera's partition, vl to the landmark's.
// A point that violates Assumption 2 gives NaN, which fails every test.
template <int LOSS>
__global__ __launch_bounds__(256) void kp_eval(PP p, const double* xc, const double* xl, const double* yc,
                                               const double* yl, int mode) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= p.K) return;
    const int i = p.ocam[o], j = p.olm[o];
    const bool intra = p.ointra[o] != 0;
    const double ux = p.ouv[2 * o], uy = p.ouv[2 * o + 1];
    const Cam c = ld_cam(xc + (size_t)i * kCS);
    const double* l = xl + (size_t)j * kLS;
    double vc = 0.0, vl = 0.0;
    const double nan = __builtin_nan("");
    if (mode == EV_F || (intra && mode == EV_E)) {
        Obs<LOSS> q;
        eval_obs<LOSS>(c, l, ux, uy, p.delta, q);
        vc = q.ok ? 0.5 * q.rho : nan;
    } else if (!intra) {
        bool ok;
        const Lin y = lin_at<LOSS>(ld_cam(yc + (size_t)i * kCS), yl + (size_t)j * kLS, ux, uy, p.delta, ok);
        const double P = P_val(y, c, ux, uy), Q = Q_val(y, l);
        if (mode == EV_E) {
            vc = ok ? P : nan;
            vl = ok ? Q : nan;
        } else {
            Obs<LOSS> q;
            eval_obs<LOSS>(c, l, ux, uy, p.delta, q);
            const double h = 0.5 * (0.5 * q.rho - P - Q);
            vc = vl = (ok && q.ok) ? h : nan;
        }
    }
    p.vc[o] = vc;
    p.vl[o] = vl;
}

// Partition sums of the shares, in two fixed-order levels.  A chunk is one
// of: camera-side shares of a run of the partition's observations (its
// cameras' observations are contiguous), landmark-side shares of a run of its
// landmarks' observations, or the proximal term of a run of its cameras or
// landmarks (+xi/2 |x - y|^2 for EV_E, -xi/2 for EV_GAP, none for EV_F).
enum { CH_CAM_OBS = 0, CH_LM_OBS = 1, CH_CAM_PROX = 2, CH_LM_PROX = 3 };
constexpr int kChunk = 2048;     // observations or landmarks per chunk
constexpr int kChunkCam = 256;   // cameras per proximal chunk

__global__ __launch_bounds__(256) void kp_reduce1(PP p, const double* xc, const double* xl, const double* yc,
                                                  const double* yl, int mode) {
    __shared__ double red[4];
    const int4 ch = p.chunk[blockIdx.x];
    const int tid = threadIdx.x;
    double s = 0.0;
    if (ch.x == CH_CAM_OBS) {
#pragma unroll 8
        for (int o = ch.z + tid; o < ch.w; o += 256) s += p.vc[o];
    } else if (ch.x == CH_LM_OBS) {
#pragma unroll 8
        for (int q = ch.z + tid; q < ch.w; q += 256) s += p.vl[p.lm_obs[q]];
    } else if (mode != EV_F) {
        double pr = 0.0;
        if (ch.x == CH_CAM_PROX) {
            for (int i = ch.z + tid; i < ch.w; i += 256)
                for (int k = 0; k < 15; ++k) {
                    const double d = xc[(size_t)i * kCS + k] - yc[(size_t)i * kCS + k];
                    pr += d * d;
                }
        } else {
            for (int j = ch.z + tid; j < ch.w; j += 256)
                for (int k = 0; k < 3; ++k) {
                    const double d = xl[(size_t)j * kLS + k] - yl[(size_t)j * kLS + k];
                    pr += d * d;
                }
        }
        s = (mode == EV_E ? 0.5 : -0.5) * p.xi * pr;
    }
    s = wsum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) p.partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One wave per partition: the sum of its chunks into ps[a][slot].
__global__ __launch_bounds__(64) void kp_reduce2(PP p, int slot) {
    const int a = blockIdx.x, lane = threadIdx.x;
    double s = 0.0;
    for (int c = p.chunk_base[a] + lane; c < p.chunk_base[a + 1]; c += kW) s += p.partial[c];
    s = wsum(s);
    if (lane == 0) p.ps[(size_t)a * kPS + slot] = s;
}

// eq. Fak and eq. lFak from the gap in P_RED
__global__ __launch_bounds__(64) void kp_fk(PP p) {
    const int a = threadIdx.x;
    if (a >= p.S) return;
    double* q = p.ps + (size_t)a * kPS;
    q[P_FK] = q[P_E] + q[P_RED];
    q[P_FBAR] = (1.0 - p.eta) * q[P_FBAR] + p.eta * q[P_FK];
}

// eq. Fainit from E^a(x^0 | x^0) in P_RED
__global__ __launch_bounds__(64) void kp_init_metrics(PP p) {
    const int a = threadIdx.x;
    if (a >= p.S) return;
    double* q = p.ps + (size_t)a * kPS;
    q[P_S] = 1.0;
    q[P_E] = q[P_FBAR] = q[P_FK] = q[P_RED];
    q[P_RESTART] = 0.0;
}

// Start of an LM solve: every partition with unknowns, or (only_restarted)
// only those whose restart test failed.  flag[0] = any partition active.
__global__ __launch_bounds__(64) void kp_lm_init(PP p, int only_restarted) {
    const int a = threadIdx.x;
    int act = 0;
    if (a < p.S) {
        double* q = p.ps + (size_t)a * kPS;
        q[P_MU] = 1e-4;
        q[P_SUCC] = q[P_REJ] = 0.0;
        act = (p.pc[a + 1] > p.pc[a] || p.pl[a + 1] > p.pl[a]) &&
              (!only_restarted || q[P_RESTART] != 0.0);
        q[P_ACTIVE] = act ? 1.0 : 0.0;
        q[P_ACC] = 0.0;
        q[P_OK] = 1.0;
    }
    const unsigned long long any = __ballot(act);
    if (a == 0) p.flag[0] = any != 0ull ? 1 : 0;
}

// dst <- src for every camera and landmark (mask 0), or only for those whose
// partition accepted its trial (mask 1).
__global__ __launch_bounds__(64) void kp_copy(PP p, const double* sc, const double* sl, double* dc, double* dl,
                                              int mask) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < p.M) {
        if (mask && p.ps[(size_t)part_of(p.pc, p.S, t) * kPS + P_ACC] == 0.0) return;
#pragma unroll
        for (int a = 0; a < 15; ++a) dc[(size_t)t * kCS + a] = sc[(size_t)t * kCS + a];
    } else if (t < p.M + p.N) {
        const int j = t - p.M;
        if (mask && p.ps[(size_t)part_of(p.pl, p.S, j) * kPS + P_ACC] == 0.0) return;
#pragma unroll
        for (int a = 0; a < 3; ++a) dl[(size_t)j * kLS + a] = sl[(size_t)j * kLS + a];
    }
}

// Gauss-Newton blocks of one camera of an active partition at x (current LM
// point) for the surrogate at y: exact pairs give rho' J^T J, rho' J^T e and
// H_cl = rho' J_c^T J_l; split pairs give 2 w J_P^T J_P and 2 w J_P^T r of
// eq. P; plus xi I and the proximal gradient.
template <int LOSS>
__global__ __launch_bounds__(256) void kp_cam_build(PP p, const double* xc, const double* xl, const double* yc,
                                                    const double* yl) {
    __shared__ double red[4][54];
    __shared__ double fin[54];
    const int i = blockIdx.x;
    const int a = part_of(p.pc, p.S, i);
    if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0) return;  // uniform over the block
    const int tid = threadIdx.x;
    const Cam c = ld_cam(xc + (size_t)i * kCS);
    double acc[54];
#pragma unroll
    for (int k = 0; k < 54; ++k) acc[k] = 0.0;
    for (int o = p.cam_off[i] + tid; o < p.cam_off[i + 1]; o += 256) {
        const int j = p.olm[o];
        const double ux = p.ouv[2 * (size_t)o], uy = p.ouv[2 * (size_t)o + 1];
        const double r2u = ux * ux + uy * uy;
        if (p.ointra[o]) {
            Obs<LOSS> q;
            eval_obs<LOSS>(c, xl + (size_t)j * kLS, ux, uy, p.delta, q);
            double hcl[27];
#pragma unroll
            for (int k = 0; k < 27; ++k) hcl[k] = 0.0;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                double J[9], G[3];
                jac_row<LOSS>(q, c, r2u, r, J, G);
#pragma unroll
                for (int u = 0; u < 9; ++u) {
#pragma unroll
                    for (int v = u; v < 9; ++v) acc[tri_idx(u, v)] += q.w * J[u] * J[v];
                    acc[45 + u] += q.w * J[u] * q.e[r];
#pragma unroll
                    for (int k = 0; k < 3; ++k) hcl[3 * u + k] += q.w * J[u] * G[k];
                }
            }
            double* dst = p.Hcl + (size_t)o * 27;
#pragma unroll
            for (int k = 0; k < 27; ++k) dst[k] = hcl[k];
        } else {
            bool ok;
            const Lin y = lin_at<LOSS>(ld_cam(yc + (size_t)i * kCS), yl + (size_t)j * kLS, ux, uy, p.delta, ok);
            const double pz = c.d[0] + c.d[1] * r2u + c.d[2] * r2u * r2u;
            const double pv[3] = {ux, uy, pz};
            const double b[3] = {1.0, r2u, r2u * r2u};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double* Rr = &c.R[3 * r];
                const double rr = Rr[0] * ux + Rr[1] * uy + Rr[2] * pz + y.lam * c.t[r] - y.g[r];
                double J[9];
                // -R [p]x row r = -(R_r x p)
                J[0] = -(Rr[1] * pv[2] - Rr[2] * pv[1]);
                J[1] = -(Rr[2] * pv[0] - Rr[0] * pv[2]);
                J[2] = -(Rr[0] * pv[1] - Rr[1] * pv[0]);
#pragma unroll
                for (int k = 0; k < 3; ++k) J[3 + k] = (r == k) ? y.lam : 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) J[6 + k] = Rr[2] * b[k];
                const double w2 = 2.0 * y.w;
#pragma unroll
                for (int u = 0; u < 9; ++u) {
#pragma unroll
                    for (int v = u; v < 9; ++v) acc[tri_idx(u, v)] += w2 * J[u] * J[v];
                    acc[45 + u] += w2 * J[u] * rr;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 54; ++k) {
        const double v = wsum(acc[k]);
        if ((tid & 63) == 0) red[tid >> 6][k] = v;
    }
    __syncthreads();
    if (tid < 54) fin[tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    __syncthreads();
    if (tid < 81) {
        const int u = tid / 9, v = tid % 9;
        double h = fin[tri_idx(u < v ? u : v, u < v ? v : u)];
        if (u == v) h += p.xi;
        p.Hcc[(size_t)i * 81 + tid] = h;
    } else if (tid < 90) {
        const int r = tid - 81;
        const double* cy = yc + (size_t)i * kCS;
        double g = fin[45 + r];
        if (r < 3) {
            // gradient of xi/2 |R Exp(w) - R^y|^2 at w = 0: -xi (A12 - A21, A20 - A02, A01 - A10), A = Y^T R
            const int u = (r + 1) % 3, v = (r + 2) % 3;
            double Auv = 0.0, Avu = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Auv += cy[3 * k + u] * c.R[3 * k + v];
                Avu += cy[3 * k + v] * c.R[3 * k + u];
            }
            g += -p.xi * (Auv - Avu);
        } else if (r < 6) {
            g += p.xi * (c.t[r - 3] - cy[9 + r - 3]);
        } else {
            g += p.xi * (c.d[r - 6] - cy[12 + r - 6]);
        }
        p.gc[(size_t)i * 16 + r] = g;
    }
}

// One lane per landmark of an active partition: H_ll, g_l from its
// observations (exact pairs: rho' J_l^T J_l, rho' J_l^T e; split pairs: eq. Q's
// 2 w lambda^2 I and 2 w lambda (lambda l - g)), xi I and the prox gradient;
// then W = (H_ll + mu diag H_ll)^-1 and W g_l.
template <int LOSS>
__global__ __launch_bounds__(64) void kp_lm_build(PP p, const double* xc, const double* xl, const double* yc,
                                                  const double* yl) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.N) return;
    const int a = part_of(p.pl, p.S, j);
    double* q = p.ps + (size_t)a * kPS;
    if (q[P_ACTIVE] == 0.0) return;
    const double* l = xl + (size_t)j * kLS;
    double H[6] = {0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0};  // H: xx xy xz yy yz zz
    for (int k = p.lm_off[j]; k < p.lm_off[j + 1]; ++k) {
        const int o = p.lm_obs[k];
        const int i = p.ocam[o];
        const double ux = p.ouv[2 * (size_t)o], uy = p.ouv[2 * (size_t)o + 1];
        if (p.ointra[o]) {
            const Cam c = ld_cam(xc + (size_t)i * kCS);
            Obs<LOSS> ob;
            eval_obs<LOSS>(c, l, ux, uy, p.delta, ob);
            double G[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                double D[3];
                de_dn_row<LOSS>(ob, r, D);
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) G[r][kk] = D[0] * c.R[3 * kk] + D[1] * c.R[3 * kk + 1] + D[2] * c.R[3 * kk + 2];
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                H[0] += ob.w * G[r][0] * G[r][0];
                H[1] += ob.w * G[r][0] * G[r][1];
                H[2] += ob.w * G[r][0] * G[r][2];
                H[3] += ob.w * G[r][1] * G[r][1];
                H[4] += ob.w * G[r][1] * G[r][2];
                H[5] += ob.w * G[r][2] * G[r][2];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) g[kk] += ob.w * G[r][kk] * ob.e[r];
            }
        } else {
            bool ok;
            const Lin y = lin_at<LOSS>(ld_cam(yc + (size_t)i * kCS), yl + (size_t)j * kLS, ux, uy, p.delta, ok);
            const double h = 2.0 * y.w * y.lam * y.lam;
            H[0] += h;
            H[3] += h;
            H[5] += h;
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) g[kk] += 2.0 * y.w * y.lam * (y.lam * l[kk] - y.g[kk]);
        }
    }
    const double* ly = yl + (size_t)j * kLS;
    H[0] += p.xi;
    H[3] += p.xi;
    H[5] += p.xi;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) g[kk] += p.xi * (l[kk] - ly[kk]);
    const double mu = q[P_MU];
    // Cholesky of the damped 3x3 block, then its inverse
    const double A00 = H[0] * (1.0 + mu), A11 = H[3] * (1.0 + mu), A22 = H[5] * (1.0 + mu);
    double L00 = A00, L10, L20, L11, L21, L22;
    bool ok = L00 > 0.0;
    L00 = ok ? sqrt(L00) : 1.0;
    L10 = H[1] / L00;
    L20 = H[2] / L00;
    L11 = A11 - L10 * L10;
    ok = ok && L11 > 0.0;
    L11 = L11 > 0.0 ? sqrt(L11) : 1.0;
    L21 = (H[4] - L20 * L10) / L11;
    L22 = A22 - L20 * L20 - L21 * L21;
    ok = ok && L22 > 0.0;
    L22 = L22 > 0.0 ? sqrt(L22) : 1.0;
    if (!ok) q[P_OK] = 0.0;
    // W = L^-T L^-1 from the inverse lower factor
    const double i00 = 1.0 / L00, i11 = 1.0 / L11, i22 = 1.0 / L22;
    const double i10 = -L10 * i00 * i11;
    const double i21 = -L21 * i11 * i22;
    const double i20 = -(L20 * i00 + L21 * i10) * i22;
    double Wm[9];
    Wm[0] = i00 * i00 + i10 * i10 + i20 * i20;
    Wm[1] = i10 * i11 + i20 * i21;
    Wm[2] = i20 * i22;
    Wm[4] = i11 * i11 + i21 * i21;
    Wm[5] = i21 * i22;
    Wm[8] = i22 * i22;
    Wm[3] = Wm[1];
    Wm[6] = Wm[2];
    Wm[7] = Wm[5];
#pragma unroll
    for (int kk = 0; kk < 9; ++kk) p.W[(size_t)j * 9 + kk] = Wm[kk];
#pragma unroll
    for (int r = 0; r < 3; ++r) p.Wg[(size_t)j * kLS + r] = Wm[3 * r] * g[0] + Wm[3 * r + 1] * g[1] + Wm[3 * r + 2] * g[2];
}

// One wave per camera: b_c = -g_c + sum over its exact pairs of H_cl W g_l.
__global__ __launch_bounds__(64) void kp_rhs(PP p) {
    const int i = blockIdx.x;
    const int a = part_of(p.pc, p.S, i);
    if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0) return;
    const int lane = threadIdx.x;
    double b[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) b[r] = 0.0;
    for (int o = p.cam_off[i] + lane; o < p.cam_off[i + 1]; o += kW) {
        if (!p.ointra[o]) continue;
        const double* h = p.Hcl + (size_t)o * 27;
        const double* wg = p.Wg + (size_t)p.olm[o] * kLS;
        const double w0 = wg[0], w1 = wg[1], w2 = wg[2];
#pragma unroll
        for (int r = 0; r < 9; ++r) b[r] += h[3 * r] * w0 + h[3 * r + 1] * w1 + h[3 * r + 2] * w2;
    }
    const int q = i - p.pc[a];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const double v = wsum(b[r]);
        if (lane == 0) p.vec[p.voff[a] + 9 * q + r] = -p.gc[(size_t)i * 16 + r] + v;
    }
}

// One wave per lower 9x9 block (q1 >= q2) of a partition's reduced camera
// system: S = [q1 == q2] (H_cc + mu diag H_cc) - sum over the block's pairs of
// T(o1) H_cl(o2)^T with T(o1) = H_cl(o1) W formed here, the pairs (two exact
// observations of one landmark by cameras q1 and q2) taken from the pair
// list.  Lane = (pair slot, row third
// g = lane & 3, slot 3 idle): 16 pairs at a time, each lane a 3x9 piece; a
// butterfly over the slots then sums the pieces in a fixed order.
__global__ __launch_bounds__(256) void kp_schur(PP p) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gb = blockIdx.x * 4 + wv;
    if (gb >= p.blkbase[p.S]) return;
    const int a = part_of(p.blkbase, p.S, gb);
    const double* q = p.ps + (size_t)a * kPS;
    if (q[P_ACTIVE] == 0.0) return;
    const int kk = gb - p.blkbase[a];
    int q1 = (int)((sqrt(8.0 * kk + 1.0) - 1.0) * 0.5);
    while ((q1 + 1) * (q1 + 2) / 2 <= kk) ++q1;
    while (q1 * (q1 + 1) / 2 > kk) --q1;
    const int q2 = kk - q1 * (q1 + 1) / 2;
    const int i1 = p.pc[a] + q1;
    const double mu = q[P_MU];
    const int e0 = p.seg_off[gb], e1 = p.seg_off[gb + 1];
    const int g = lane & 3, slot = lane >> 2;
    double acc[3][9];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int v = 0; v < 9; ++v) acc[u][v] = 0.0;
    if (g < 3) {
        for (int e = e0 + slot; e < e1; e += 16) {
            const int o1 = p.ent[2 * e];
            const double* h1 = p.Hcl + (size_t)o1 * 27 + 9 * g;          // rows 3g .. 3g+2 of H_cl(o1)
            const double* W = p.W + (size_t)p.olm[o1] * 9;               // the pair's landmark
            const double* h = p.Hcl + (size_t)p.ent[2 * e + 1] * 27;    // H_cl(o2), 9 x 3
            double tv[9], hv[27], hr[9], wv[9];
#pragma unroll
            for (int x = 0; x < 9; ++x) hr[x] = h1[x];
#pragma unroll
            for (int x = 0; x < 9; ++x) wv[x] = W[x];
#pragma unroll
            for (int u = 0; u < 3; ++u)  // rows 3g .. 3g+2 of T(o1) = H_cl(o1) W
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    tv[3 * u + c] = hr[3 * u] * wv[c] + hr[3 * u + 1] * wv[3 + c] + hr[3 * u + 2] * wv[6 + c];
#pragma unroll
            for (int x = 0; x < 27; ++x) hv[x] = h[x];
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
                for (int v = 0; v < 9; ++v)
                    acc[u][v] += tv[3 * u] * hv[3 * v] + tv[3 * u + 1] * hv[3 * v + 1] + tv[3 * u + 2] * hv[3 * v + 2];
        }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int v = 0; v < 9; ++v) {
            double x = acc[u][v];
            for (int off = 4; off < kW; off <<= 1) x += __shfl_xor(x, off, kW);
            acc[u][v] = x;
        }
    if (lane < 3) {  // lane g now holds rows 3g .. 3g+2 summed over every pair
        const int np = p.npad[a];
        double* Sa = p.Smat + p.soff[a];
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 9; ++v) {
                const int r = 3 * g + u;
                double val = -acc[u][v];
                if (q1 == q2) {
                    const double hc = p.Hcc[(size_t)i1 * 81 + 9 * r + v];
                    val += (r == v) ? hc * (1.0 + mu) : hc;
                }
                Sa[(size_t)(9 * q1 + r) * np + 9 * q2 + v] = val;
            }
    }
}

// Lane j's value of x (j uniform): two v_readlane, no LDS round trip.
__device__ __forceinline__ double lane_value(double x, int j) {
    const int2 v = __builtin_bit_cast(int2, x);
    int2 o;
    o.x = __builtin_amdgcn_readlane(v.x, j);
    o.y = __builtin_amdgcn_readlane(v.y, j);
    return __builtin_bit_cast(double, o);
}

// 1/sqrt(d) for a normal d > 0: the hardware reciprocal square root refined
// by two coupled Newton steps on g ~ sqrt(d), h ~ 1/(2 sqrt(d)), each of
// which squares the relative error.  A few ulp, with no division or
// square-root sequence on the factorisation's serial chain.
__device__ __forceinline__ double rsqrt_refined(double d) {
    const double y = __builtin_amdgcn_rsq(d);
    double g = d * y, h = 0.5 * y;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    h = fma(h, e, h);
    return 2.0 * h;
}

constexpr int kPW = 16;          // tile columns per wave in the four-wave tile kernels
constexpr int kNW = kNB / kPW;   // waves of those kernels
constexpr int kLD = kNB + 2;     // LDS row stride of a staged tile: 16-byte aligned rows, read in pairs

// n consecutive doubles at a 16-byte aligned LDS address, read as pairs.
template <int N>
__device__ __forceinline__ void lds_pairs(const double* src, double* v) {
    static_assert(N % 2 == 0, "pairs");
#pragma unroll
    for (int c = 0; c < N; c += 2) {
        const double2 t = *reinterpret_cast<const double2*>(src + c);
        v[c] = t.x;
        v[c + 1] = t.y;
    }
}

// A copy of v that the compiler takes as varying across lanes, so that
// address arithmetic scaled by it stays in vector registers instead of
// being hoisted into dozens of scalar registers (one ds_bpermute).
__device__ __forceinline__ int varying(int v) { return __shfl(v, threadIdx.x & 63, kW); }

// Panel P of a diagonal tile's factorisation, run by wave P, whose lane r
// holds x[i] = entry (r, 16P + i) of the tile after the earlier panels'
// updates.  Column C = 16P + i: the pivot from lane C by readlane; every
// lane scales its entry by 1/sqrt(pivot) (L_rC below the diagonal,
// A_CC / sqrt(A_CC) = L_CC on it); the panel's later columns j take
// L_rC L_jC, with L_(C+1)C (on the pivot chain) read from lane C + 1 and the
// others broadcast from col (LDS).  The right-hand side rides along as one
// more column: y_C = b_C / L_CC, then b_r -= L_rC y_C.  Lane C keeps y_C
// and 1/L_CC.  The updates need no per-lane select: lanes above the
// diagonal carry values of the upper triangle, which are never stored or
// read.  The previous panel's rank-16 update (in T, row stride kLD) reaches
// each column just before its pivot, so that its products fill the pivot
// chain's idle issue slots.
template <int P>
__device__ __forceinline__ void factor_panel(double (&x)[kPW], const double (*T)[kLD], double* col, double& yb,
                                             double& yfin, double& invfin, int r, bool& bad) {
    double a[kPW];  // this row's entries in the previous panel
    if constexpr (P > 0) lds_pairs<kPW>(T[r] + kPW * (P - 1), a);
#pragma unroll
    for (int i = 0; i < kPW; ++i) {
        const int C = kPW * P + i;
        if constexpr (P > 0) {
            double l[kPW];
            lds_pairs<kPW>(T[C] + kPW * (P - 1), l);
            double s0 = x[i], s1 = 0.0;
#pragma unroll
            for (int c = 0; c < kPW; c += 2) {
                s0 = fma(-a[c], l[c], s0);
                s1 = fma(-a[c + 1], l[c + 1], s1);
            }
            x[i] = s0 + s1;
        }
        const double d = lane_value(x[i], C);
        bad = bad || !(d > 0.0);
        const double inv = rsqrt_refined(d > 0.0 ? d : 1.0);
        x[i] *= inv;
        const double yc = lane_value(yb, C) * inv;
        if (r == C) {
            yfin = yc;
            invfin = inv;
        }
        yb = fma(-x[i], yc, yb);
        if (i + 1 < kPW) {
            x[i + 1] = fma(-x[i], lane_value(x[i], C + 1), x[i + 1]);
            if (i + 2 < kPW) {
                col[r] = x[i];
                const int j0 = (i + 2) & ~1;  // pairs from an even column; column i + 1 is masked out
                double v[kPW];
#pragma unroll
                for (int j = j0; j < kPW; j += 2) {
                    const double2 t = *reinterpret_cast<const double2*>(col + kPW * P + j);
                    v[j] = t.x;
                    v[j + 1] = t.y;
                }
#pragma unroll
                for (int j = i + 2; j < kPW; ++j) x[j] = fma(-x[i], v[j], x[j]);
            }
        }
    }
}

// Rank-16 update of wave w's columns by panel P (w > P):
// x[i] -= sum_c M_(r, 16P+c) M_(16w+i, 16P+c), M a tile in LDS (row stride
// kLD): the lane's own row, and the rows of the wave's columns by broadcast,
// in pairs.
template <int P>
__device__ __forceinline__ void panel_update(double (&x)[kPW], const double (*M)[kLD], int r, int w) {
    double a[kPW];
    lds_pairs<kPW>(M[r] + kPW * P, a);
#pragma unroll
    for (int i = 0; i < kPW; ++i) {
        double l[kPW];
        lds_pairs<kPW>(M[kPW * w + i] + kPW * P, l);
        double s0 = x[i], s1 = 0.0;
#pragma unroll
        for (int c = 0; c < kPW; c += 2) {
            s0 = fma(-a[c], l[c], s0);
            s1 = fma(-a[c + 1], l[c + 1], s1);
        }
        x[i] = s0 + s1;
    }
}

template <int P>
__device__ __forceinline__ void factor_panels(double (&x)[kPW], double (*T)[kLD], double* ybuf, double& yb,
                                              double& yfin, double& invfin, int r, int w, bool& bad) {
    if (w == P) {
        if constexpr (P > 0) yb = ybuf[r];
        factor_panel<P>(x, T, ybuf + kNB, yb, yfin, invfin, r, bad);
#pragma unroll
        for (int c = 0; c < kPW; ++c) T[r][kPW * P + c] = x[c];
        ybuf[r] = yb;
    }
    __syncthreads();
    if constexpr (P + 1 < kNW) {
        if (w > P + 1) panel_update<P>(x, T, r, w);  // wave P + 1 takes it column by column
        factor_panels<P + 1>(x, T, ybuf, yb, yfin, invfin, r, w, bad);
    }
}

// Blocked right-looking Cholesky: factor diagonal tile k of partition a,
// which T (LDS, row-major, stride kLD) holds after every earlier step's
// update, with the block's four waves, wave w holding columns 16w .. 16w+15
// of every row (lane r: row r).  Panel P is factored by wave P and published
// in T; after a barrier the waves to its right take its rank-16 update.
// Stores L_kk (lower triangle, coalesced from T), 1/L_rr, and the forward
// substitution folded into the factorisation: y_k = L_kk^-1 b_k, b_k already
// reduced by the earlier panels, which then take L_ik y_k out of b_i for the
// tiles below.  Every thread of the 256-thread block calls it, with bv =
// entry (threadIdx.x mod 64) of b_k, loaded early by the caller, and ybuf
// 128 doubles of LDS (16-byte aligned).
__device__ __forceinline__ void factor_tile(const PP& p, int a, int k, double (*T)[kLD], double* ybuf,
                                            double bv) {
    const int r = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double x[kPW];
#pragma unroll
    for (int i = 0; i < kPW; ++i) {
        const double v = T[r][kPW * w + i];
        x[i] = kPW * w + i <= r ? v : 0.0;
    }
    double* bk = p.vec + p.voff[a] + kNB * k;
    double yb = w == 0 ? bv : 0.0, yfin = 0.0, invfin = 1.0;
    bool bad = false;
    factor_panels<0>(x, T, ybuf, yb, yfin, invfin, r, w, bad);
    if (r == 0 && bad) p.ps[(size_t)a * kPS + P_OK] = 0.0;
    if ((r >> 4) == w) {  // rows of the wave's own panel: their y and 1/L_rr
        p.dinv[p.voff[a] + kNB * k + r] = invfin;
        bk[r] = yfin;
    }
    const int np = p.npad[a];
    double* S = p.Smat + p.soff[a] + (size_t)(kNB * k) * np + kNB * k;
#pragma unroll
    for (int i = 0; i < kPW; ++i) {  // wave w stores rows 16w .. 16w+15, lane r column r
        const int rr = kPW * w + i;
        if (r <= rr) S[(size_t)rr * np + r] = T[rr][r];
    }
}

// The first diagonal tile of every partition (each later one is factored by
// the update launch that completes it).
__global__ __launch_bounds__(256) void kp_chol_diag(PP p, int k) {
    __shared__ __align__(16) double T[kNB][kLD];
    __shared__ __align__(16) double ybuf[2 * kNB];
    const int a = blockIdx.x;
    if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0 || k >= p.nt[a]) return;
    const int np = p.npad[a];
    const double* S = p.Smat + p.soff[a] + (size_t)(kNB * k) * np + kNB * k;
    const int tid = threadIdx.x;
    const double bv = p.vec[p.voff[a] + kNB * k + (tid & 63)];
    double v[kNB * kNB / 256];
#pragma unroll
    for (int u = 0; u < kNB * kNB / 256; ++u) {
        const int e = tid + 256 * u;
        v[u] = S[(size_t)(e / kNB) * np + e % kNB];
    }
#pragma unroll
    for (int u = 0; u < kNB * kNB / 256; ++u) {
        const int e = tid + 256 * u;
        T[e / kNB][e % kNB] = v[u];
    }
    __syncthreads();
    factor_tile(p, a, k, T, ybuf, bv);
}

// Panel P of a panel tile's triangular solve x L_kk^T = a (wave P; lane r:
// row r): x_C = a_C / L_CC, then x_C L_jC leaves a_j for the panel's later
// columns j; the panel is published in X, and after a barrier the waves to
// its right take its rank-16 update (the next wave column by column, just
// before each division, the others at once).
template <int P>
__device__ __forceinline__ void trsm_panels(double (&x)[kPW], const double (*Lk)[kLD], double (*X)[kLD],
                                            const double* iv, int r, int w) {
    if (w == P) {
        double s[kPW];  // this row's solved entries in the previous panel
        if constexpr (P > 0) lds_pairs<kPW>(X[r] + kPW * (P - 1), s);
#pragma unroll
        for (int i = 0; i < kPW; ++i) {
            const int C = kPW * P + i;
            if constexpr (P > 0) {  // the previous panel's update, column by column
                double l[kPW];
                lds_pairs<kPW>(Lk[C] + kPW * (P - 1), l);
                double t0 = x[i], t1 = 0.0;
#pragma unroll
                for (int c = 0; c < kPW; c += 2) {
                    t0 = fma(-s[c], l[c], t0);
                    t1 = fma(-s[c + 1], l[c + 1], t1);
                }
                x[i] = t0 + t1;
            }
            x[i] *= iv[C];
#pragma unroll
            for (int j = i + 1; j < kPW; ++j) x[j] = fma(-x[i], Lk[kPW * P + j][C], x[j]);
        }
#pragma unroll
        for (int c = 0; c < kPW; ++c) X[r][kPW * P + c] = x[c];
    }
    __syncthreads();
    if constexpr (P + 1 < kNW) {
        if (w > P + 1) {  // x[i] -= sum_c X_(r, 16P+c) L_(16w+i, 16P+c); wave P + 1 takes it column by column
            double s[kPW];
            lds_pairs<kPW>(X[r] + kPW * P, s);
#pragma unroll
            for (int i = 0; i < kPW; ++i) {
                double l[kPW];
                lds_pairs<kPW>(Lk[kPW * w + i] + kPW * P, l);
                double t0 = x[i], t1 = 0.0;
#pragma unroll
                for (int c = 0; c < kPW; c += 2) {
                    t0 = fma(-s[c], l[c], t0);
                    t1 = fma(-s[c + 1], l[c + 1], t1);
                }
                x[i] = t0 + t1;
            }
        }
        trsm_panels<P + 1>(x, Lk, X, iv, r, w);
    }
}

// Step k: L_ik = A_ik L_kk^-T for every tile row i > k, one block of four
// waves per tile (wave w: columns 16w .. 16w+15, lane r: row r), blocked
// over panels like the factorisation, with the stored reciprocals of
// L_kk's diagonal; then b_i -= L_ik y_k.
__global__ __launch_bounds__(256) void kp_chol_trsm(PP p, int k) {
    __shared__ __align__(16) double Lk[kNB][kLD];
    __shared__ __align__(16) double X[kNB][kLD];
    __shared__ double yk[kNB], iv[kNB];
    const int a = blockIdx.y;
    const int i = k + 1 + blockIdx.x;
    if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0 || i >= p.nt[a]) return;
    const int np = p.npad[a];
    const int tid = threadIdx.x, r = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double* Lkk = p.Smat + p.soff[a] + (size_t)(kNB * k) * np + kNB * k;
    double2* Ar = reinterpret_cast<double2*>(p.Smat + p.soff[a] + (size_t)(kNB * i + r) * np + kNB * k + kPW * w);
    double* b = p.vec + p.voff[a];
    // every global load in flight before the first wait
    double x[kPW];
#pragma unroll
    for (int m = 0; m < kPW / 2; ++m) {
        const double2 v = Ar[m];
        x[2 * m] = v.x;
        x[2 * m + 1] = v.y;
    }
    double v[kNB * kNB / 256];
#pragma unroll
    for (int u = 0; u < kNB * kNB / 256; ++u) {
        const int e = tid + 256 * u;
        v[u] = Lkk[(size_t)(e / kNB) * np + e % kNB];
    }
    const double ykr = b[kNB * k + r];  // y_k, solved by the diagonal step
    const double ivr = p.dinv[p.voff[a] + kNB * k + r];
    const double bir = b[kNB * i + r];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kNB * kNB / 256; ++u) {
        const int e = tid + 256 * u;
        Lk[e / kNB][e % kNB] = v[u];
    }
    if (w == 0) {
        yk[r] = ykr;
        iv[r] = ivr;
    }
    __syncthreads();
    trsm_panels<0>(x, Lk, X, iv, r, w);
#pragma unroll
    for (int m = 0; m < kPW / 2; ++m) Ar[m] = make_double2(x[2 * m], x[2 * m + 1]);
    if (w == 0) {  // forward substitution of the right-hand side: b_i -= L_ik y_k
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int c = 0; c < kNB; c += 2) {
            s0 += X[r][c] * yk[c];
            s1 += X[r][c + 1] * yk[c + 1];
        }
        b[kNB * i + r] = bir - (s0 + s1);
    }
}

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// Step k: A_ij -= L_ik L_jk^T for tiles k < j <= i, on the matrix cores:
// v_mfma_f64_16x16x4f64, each wave a 32 x 32 quadrant of the tile as 2 x 2
// blocks of 16 x 16, the inner dimension in two halves of 32 columns staged
// in LDS (rows padded to 34 doubles: two-way bank conflicts for the operand
// reads).  Operand layout of the instruction: lane l holds A(l mod 16,
// l / 16) and B(l / 16, l mod 16); accumulator register v of lane l holds
// D(l / 16 + 4 v, l mod 16).  The block of tile (k+1, k+1), whose update is
// the last one it receives, completes it in LDS and factors it for step
// k + 1 while the other tiles update.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void kp_chol_update(PP p, int k) {
    constexpr int kH = kNB / 2, kS = kH + 2;
    __shared__ __align__(16) double sh[2 * kNB * kS];
    __shared__ __align__(16) double ybuf[2 * kNB];
    static_assert(kNB * kLD <= 2 * kNB * kS, "tile buffer");
    double (*Li)[kS] = reinterpret_cast<double (*)[kS]>(sh);
    double (*Lj)[kS] = reinterpret_cast<double (*)[kS]>(sh + kNB * kS);
    const int a = blockIdx.y;
    if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0) return;
    const int m = p.nt[a] - k - 1;  // trailing tiles
    const int t = blockIdx.x;
    if (m <= 0 || t >= m * (m + 1) / 2) return;
    int ii = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
    while (ii * (ii + 1) / 2 > t) --ii;
    const int jj = t - ii * (ii + 1) / 2;
    const int i = k + 1 + ii, j = k + 1 + jj;
    const int np = p.npad[a];
    const double* base = p.Smat + p.soff[a];
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rb = 32 * (w >> 1), cb = 32 * (w & 1);  // the wave's quadrant
    const int lr = l & 15, lk = l >> 4;
    double* Aij = p.Smat + p.soff[a] + (size_t)(kNB * i) * np + kNB * j;
    // tile (k+1, k+1) is factored after its update: its b entry now
    const double bv = t == 0 ? p.vec[p.voff[a] + kNB * (k + 1) + l] : 0.0;
    mfma_d4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    for (int h = 0; h < kNB; h += kH) {
        __syncthreads();
        double vi[kNB * kH / 256], vj[kNB * kH / 256];
#pragma unroll
        for (int u = 0; u < kNB * kH / 256; ++u) {
            const int e = tid + 256 * u, r = e / kH, c = e % kH;
            vi[u] = base[(size_t)(kNB * i + r) * np + kNB * k + h + c];
            vj[u] = base[(size_t)(kNB * j + r) * np + kNB * k + h + c];
        }
#pragma unroll
        for (int u = 0; u < kNB * kH / 256; ++u) {
            const int e = tid + 256 * u, r = e / kH, c = e % kH;
            Li[r][c] = vi[u];
            Lj[r][c] = vj[u];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kH; ks += 4) {
            const double a0 = Li[rb + lr][ks + lk], a1 = Li[rb + 16 + lr][ks + lk];
            const double b0 = Lj[cb + lr][ks + lk], b1 = Lj[cb + 16 + lr][ks + lk];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    if (t == 0) {  // tile (k+1, k+1): complete it in LDS and factor it
        double (*T)[kLD] = reinterpret_cast<double (*)[kLD]>(sh);
        __syncthreads();  // every wave is done with Li and Lj
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = rb + 16 * u + lk + 4 * q, c = cb + 16 * v + lr;
                    T[r][c] = Aij[(size_t)r * np + c] - acc[u][v][q];
                }
        __syncthreads();
        factor_tile(p, a, k + 1, T, ybuf, bv);
        return;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rb + 16 * u + lk + 4 * q, c = cb + 16 * v + lr;
                Aij[(size_t)r * np + c] -= acc[u][v][q];
            }
}

// Stages the strictly lower part of diagonal tile c0 / 64 in D (LDS, only
// wave 0's), every row's load in flight at once.
__device__ __forceinline__ void trsv_stage(const double* L, int np, int c0, double (*D)[kNB + 1]) {
    const int lane = threadIdx.x & 63;
    const int npv = varying(np);
    const double* q = L + (size_t)c0 * npv + c0 + lane;
    double v[kNB];  // loaded by every lane: a select below, not a branch around a load
#pragma unroll
    for (int rr = 0; rr < kNB; ++rr) {
        v[rr] = *q;
        q += npv;
    }
    __builtin_amdgcn_sched_barrier(0);  // every load issued before the first wait
#pragma unroll
    for (int rr = 0; rr < kNB; ++rr) D[rr][lane] = lane < rr ? v[rr] : 0.0;
}

// Dot of tile c0 / 64's rows of L, column r, with x of that tile:
// sum_c L_(c0+c, r) x_c.  Every load is issued before the first use.
__device__ __forceinline__ double trsv_dot(const double* L, int npv, int c0, int r, const double* xk) {
    const double* q = L + (size_t)c0 * npv + r;
    double v[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
        v[c] = *q;
        q += npv;
    }
    __builtin_amdgcn_sched_barrier(0);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int c = 0; c < kNB; c += 2) {
        s0 = fma(v[c], xk[c], s0);
        s1 = fma(v[c + 1], xk[c + 1], s1);
    }
    return s0 + s1;
}

// Backward sweep of a staged diagonal tile for wave 0 (lane = row c0 +
// lane, y its right-hand side entry reduced by every later tile), with L^T,
// (L^T)_(lane, c) = L_(c, lane), and the stored reciprocals of the
// diagonal: lane c's entry is final at step c.
__device__ __forceinline__ double trsv_solve(const double (*D)[kNB + 1], const double* dinv, int c0, double y) {
    const int lane = threadIdx.x & 63;
    const double iv = dinv[c0 + lane];
    double xv = y;
#pragma unroll
    for (int c = kNB - 1; c >= 0; --c) xv = fma(-D[c][lane], lane_value(xv * iv, c), xv);
    return xv * iv;
}

// L^T x = y in place on the partition's vector (the forward half, L y = b,
// is folded into the factorisation), one 64-row tile at a time from the
// last, with look-ahead: once x of tile kt is known, wave 0 takes it out of
// the rows of tile kt - 1 and solves that tile's triangle; wave 1 stages
// the diagonal tile wave 0 needs next; the other waves take x of tile kt out
// of the rows above (one thread per row, reading tile kt's rows of L,
// consecutive across lanes).
__global__ __launch_bounds__(512) void kp_trsv(PP p) {
    constexpr int kT = 512;
    __shared__ double xs[2][kNB];
    __shared__ double D[2][kNB][kNB + 1];  // diagonal tiles kt and kt - 1
    const int a = blockIdx.x;
    if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0) return;
    const int np = p.npad[a], nt = p.nt[a];
    if (nt == 0) return;
    const double* L = p.Smat + p.soff[a];
    double* b = p.vec + p.voff[a];
    const double* dinv = p.dinv + p.voff[a];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int npv = varying(np);
    if (wave == 0) {
        const int c0 = kNB * (nt - 1);
        const double y = b[c0 + lane];
        trsv_stage(L, np, c0, D[(nt - 1) & 1]);
        const double x = trsv_solve(D[(nt - 1) & 1], dinv, c0, y);
        xs[(nt - 1) & 1][lane] = x;
        b[c0 + lane] = x;
    } else if (wave == 1 && nt >= 2) {
        trsv_stage(L, np, kNB * (nt - 2), D[(nt - 2) & 1]);
    }
    for (int kt = nt - 1; kt >= 1; --kt) {
        __syncthreads();  // x of tile kt is in xs[kt & 1], diagonal tile kt - 1 in D[(kt - 1) & 1]
        const int c0 = kNB * kt;
        const double* xk = xs[kt & 1];
        if (wave == 0) {
            const int r = c0 - kNB + lane;
            const double y = b[r];
            const double x = trsv_solve(D[(kt - 1) & 1], dinv, c0 - kNB, y - trsv_dot(L, npv, c0, r, xk));
            xs[(kt - 1) & 1][lane] = x;
            b[r] = x;
        } else if (wave == 1) {
            if (kt >= 2) trsv_stage(L, np, c0 - 2 * kNB, D[kt & 1]);  // tile kt's buffer is free now
        } else {
            for (int r = tid - 2 * kW; r < c0 - kNB; r += kT - 2 * kW) b[r] -= trsv_dot(L, npv, c0, r, xk);
        }
    }
}

// Trial point of every active partition: cameras R Exp(dtheta), t + dt,
// d + dd from the solved vector; landmarks l + dl with
// dl = -W g_l - W sum over exact pairs of H_cl^T dc.
__global__ __launch_bounds__(64) void kp_step(PP p, const double* cc, const double* cl, double* tc, double* tl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < p.M) {
        const int a = part_of(p.pc, p.S, t);
        if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0) return;
        const double* dv = p.vec + p.voff[a] + 9 * (t - p.pc[a]);
        const double* c = cc + (size_t)t * kCS;
        double* o = tc + (size_t)t * kCS;
        double E[9];
        daba::exp_so3(dv, E);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                o[3 * r + k] = c[3 * r] * E[k] + c[3 * r + 1] * E[3 + k] + c[3 * r + 2] * E[6 + k];
#pragma unroll
        for (int k = 0; k < 6; ++k) o[9 + k] = c[9 + k] + dv[3 + k];
    } else if (t < p.M + p.N) {
        const int j = t - p.M;
        const int a = part_of(p.pl, p.S, j);
        if (p.ps[(size_t)a * kPS + P_ACTIVE] == 0.0) return;
        double u[3] = {0.0, 0.0, 0.0};  // sum over exact pairs of H_cl^T dc
        for (int k = p.lm_off[j]; k < p.lm_off[j + 1]; ++k) {
            const int o = p.lm_obs[k];
            if (!p.ointra[o]) continue;
            const int i = p.ocam[o];
            const double* dv = p.vec + p.voff[a] + 9 * (i - p.pc[a]);
            const double* H = p.Hcl + (size_t)o * 27;
            for (int r = 0; r < 9; ++r) {
                const double x = dv[r];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) u[kk] += H[3 * r + kk] * x;
            }
        }
        const double* W = p.W + (size_t)j * 9;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            tl[(size_t)j * kLS + k] = cl[(size_t)j * kLS + k] - p.Wg[(size_t)j * kLS + k] -
                                      (W[3 * k] * u[0] + W[3 * k + 1] * u[1] + W[3 * k + 2] * u[2]);
    }
}

// Strict-decrease test of each active partition's trial (P_ETRY vs P_PHI),
// damping update, and whether any partition is still active.
__global__ __launch_bounds__(64) void kp_accept(PP p) {
    const int a = threadIdx.x;
    int act = 0;
    if (a < p.S) {
        double* q = p.ps + (size_t)a * kPS;
        if (q[P_ACTIVE] != 0.0) {
            const bool acc = q[P_OK] != 0.0 && q[P_ETRY] < q[P_PHI];
            if (acc) {
                q[P_PHI] = q[P_ETRY];
                q[P_MU] /= 10.0;
                q[P_SUCC] += 1.0;
                q[P_REJ] = 0.0;
            } else {
                q[P_MU] *= 10.0;
                q[P_REJ] += 1.0;
            }
            q[P_ACC] = acc ? 1.0 : 0.0;
            act = (q[P_SUCC] < p.inner_steps && q[P_REJ] < 10.0) ? 1 : 0;
            q[P_ACTIVE] = act ? 1.0 : 0.0;
        } else {
            q[P_ACC] = 0.0;
        }
        q[P_OK] = 1.0;
    }
    const unsigned long long any = __ballot(act);
    if (a == 0) p.flag[0] = any != 0ull ? 1 : 0;
}

// Restart test (Algorithm 1; eq. Eak) from P_FK, P_FBAR, P_ECUR and P_EACC:
// a partition keeps its accelerated step unless E^a(k+1) would exceed
// Fbar^a(k); without acceleration every partition takes the plain step.
__global__ __launch_bounds__(64) void kp_restart_test(PP p) {
    const int a = threadIdx.x;
    if (a >= p.S) return;
    double* q = p.ps + (size_t)a * kPS;
    if (!p.accelerate) {
        q[P_RESTART] = 1.0;
        return;
    }
    const double Ehat = q[P_EACC] + q[P_FK] - q[P_ECUR];
    bool rs = Ehat > q[P_FBAR];
    if (p.flags & DABA_DEBUG_NEVER_RESTART) rs = false;
    if (p.flags & DABA_DEBUG_ALWAYS_RESTART) rs = true;
    q[P_RESTART] = rs ? 1.0 : 0.0;
    if (!rs) q[P_E] = Ehat;
}

// E^a(k+1) of the partitions that take the plain step (eq. Eak with P_EMM).
__global__ __launch_bounds__(64) void kp_restart_finish(PP p) {
    const int a = threadIdx.x;
    if (a >= p.S) return;
    double* q = p.ps + (size_t)a * kPS;
    if (q[P_RESTART] != 0.0) q[P_E] = q[P_EMM] + q[P_FK] - q[P_ECUR];
}

// x^(k-1) <- x^k; x^(k+1) <- the accelerated or the plain candidate.
__global__ __launch_bounds__(64) void kp_roll(PP p, double* xc, double* pcam, const double* mc, const double* ac,
                                              double* xl, double* plm, const double* ml, const double* al) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < p.M) {
        const bool acc = p.accelerate && p.ps[(size_t)part_of(p.pc, p.S, t) * kPS + P_RESTART] == 0.0;
        const double* src = acc ? ac : mc;
#pragma unroll
        for (int k = 0; k < 15; ++k) {
            pcam[(size_t)t * kCS + k] = xc[(size_t)t * kCS + k];
            xc[(size_t)t * kCS + k] = src[(size_t)t * kCS + k];
        }
    } else if (t < p.M + p.N) {
        const int j = t - p.M;
        const bool acc = p.accelerate && p.ps[(size_t)part_of(p.pl, p.S, j) * kPS + P_RESTART] == 0.0;
        const double* src = acc ? al : ml;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            plm[(size_t)j * kLS + k] = xl[(size_t)j * kLS + k];
            xl[(size_t)j * kLS + k] = src[(size_t)j * kLS + k];
        }
    }
}

// trace[it] = sum over partitions of P_RED (fixed order)
__global__ __launch_bounds__(64) void kp_trace(PP p, int it) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int a = 0; a < p.S; ++a) s += p.ps[(size_t)a * kPS + P_RED];
    p.trace[it] = s;
}

// Zero the reduced systems and put ones on the padding's diagonal; the
// padding stays the identity under every later factorisation.
__global__ __launch_bounds__(256) void kp_init_smat(PP p, int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int a = 0;
    while (a + 1 < p.S && p.soff[a + 1] <= e) ++a;
    const int64_t loc = e - p.soff[a];
    const int np = p.npad[a];
    const int r = (int)(loc / np), c = (int)(loc % np);
    const int n = 9 * (p.pc[a + 1] - p.pc[a]);
    p.Smat[e] = (r == c && r >= n) ? 1.0 : 0.0;
}

}  // namespace dpart

// ===================================================================== host

using namespace dpart;

namespace {

thread_local std::string g_err = "no error";

struct Fail {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Fail{code, buf};
}

void hipck(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(DABA_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Host-side layout: internal orders and the Schur pair list.
struct PLayout {
    int M = 0, N = 0, S = 1;
    int64_t K = 0;
    double scale = 1.0;
    std::vector<int> cam_ext, cam_int, lm_ext, lm_int;  // internal <-> caller
    std::vector<int> pc, pl;                            // [S+1]
    std::vector<int> ocam, olm, ointra;                 // internal obs
    std::vector<double> ouv;
    std::vector<int> cam_off, lm_off, lm_obs;
    std::vector<int> nt, npad, voff, blkbase;
    std::vector<int64_t> soff;
    std::vector<int> seg_off, ent;
    std::vector<int> chunk, chunk_base;  // 4 ints per chunk; [S+1]
    int64_t smat_total = 0;
    int vec_total = 0;
};

bool rotation_ok(const double* R) {
    double e = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = R[r] * R[c] + R[3 + r] * R[3 + c] + R[6 + r] * R[6 + c];
            e = std::max(e, std::fabs(s - (r == c ? 1.0 : 0.0)));
        }
    double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                 R[2] * (R[3] * R[7] - R[4] * R[6]);
    return e < 1e-6 && det > 0.0;
}

void validate_options(const daba_options* o) {
    if (!o) fail(DABA_E_INVAL, "options are NULL");
    if (o->loss < 0 || o->loss > 2) fail(DABA_E_INVAL, "unknown loss %d", o->loss);
    if (o->loss != DABA_LOSS_TRIVIAL && !(o->loss_delta > 0.0 && std::isfinite(o->loss_delta)))
        fail(DABA_E_INVAL, "loss_delta must be positive");
    if (!(o->xi > 0.0 && std::isfinite(o->xi))) fail(DABA_E_INVAL, "xi must be positive");
    if (!(o->eta > 0.0 && o->eta <= 1.0)) fail(DABA_E_INVAL, "eta must be in (0, 1]");
    if (o->accelerate != 0 && o->accelerate != 1) fail(DABA_E_INVAL, "accelerate must be 0 or 1");
    if (o->inner_steps < 1) fail(DABA_E_INVAL, "inner_steps must be >= 1 for the device surrogate");
    if (o->precision != DABA_FP64) fail(DABA_E_INVAL, "the device surrogate runs in FP64 only");
    if (o->debug_flags & ~(uint64_t)(DABA_DEBUG_NEVER_RESTART | DABA_DEBUG_ALWAYS_RESTART))
        fail(DABA_E_INVAL, "unknown debug flag");
}

void build_layout(const daba_problem* pr, PLayout& L) {
    if (!pr) fail(DABA_E_INVAL, "problem is NULL");
    if (pr->n_cameras < 1 || pr->n_landmarks < 1 || pr->n_obs < 0) fail(DABA_E_INVAL, "sizes must be M, N >= 1, K >= 0");
    if (pr->n_cameras > (1 << 30) || pr->n_landmarks > (1 << 30) || pr->n_obs > (int64_t)INT32_MAX / 2)
        fail(DABA_E_INVAL, "problem too large");
    if (pr->n_partitions < 1 || pr->n_partitions > DABA_MAX_PARTITIONS)
        fail(DABA_E_INVAL, "n_partitions must be in [1, %d]", DABA_MAX_PARTITIONS);
    if (!(pr->unit_scale > 0.0 && std::isfinite(pr->unit_scale))) fail(DABA_E_INVAL, "unit_scale must be positive");
    if (pr->n_obs > 0 && (!pr->obs_camera || !pr->obs_landmark || !pr->obs_uv))
        fail(DABA_E_INVAL, "observation arrays are NULL");
    const int M = (int)pr->n_cameras, N = (int)pr->n_landmarks, S = pr->n_partitions;
    const int64_t K = pr->n_obs;
    L.M = M;
    L.N = N;
    L.S = S;
    L.K = K;
    L.scale = pr->unit_scale;
    for (int64_t o = 0; o < K; ++o) {
        if (pr->obs_camera[o] < 0 || pr->obs_camera[o] >= M) fail(DABA_E_INVAL, "obs_camera[%lld] out of range", (long long)o);
        if (pr->obs_landmark[o] < 0 || pr->obs_landmark[o] >= N)
            fail(DABA_E_INVAL, "obs_landmark[%lld] out of range", (long long)o);
    }
    std::vector<int> cpart(M), lpart(N);
    const int blk = (M + S - 1) / S;
    for (int i = 0; i < M; ++i) {
        cpart[i] = pr->camera_partition ? pr->camera_partition[i] : i / blk;
        if (cpart[i] < 0 || cpart[i] >= S) fail(DABA_E_INVAL, "camera_partition[%d] out of range", i);
    }
    if (pr->landmark_partition) {
        for (int j = 0; j < N; ++j) {
            lpart[j] = pr->landmark_partition[j];
            if (lpart[j] < 0 || lpart[j] >= S) fail(DABA_E_INVAL, "landmark_partition[%d] out of range", j);
        }
    } else {
        std::vector<int> first(N, M);
        for (int64_t o = 0; o < K; ++o) first[pr->obs_landmark[o]] = std::min(first[pr->obs_landmark[o]], pr->obs_camera[o]);
        for (int j = 0; j < N; ++j) lpart[j] = first[j] < M ? cpart[first[j]] : 0;
    }
    // partition-major internal orders (stable in caller ids)
    auto order = [&](const std::vector<int>& part, int n, std::vector<int>& ext, std::vector<int>& in,
                     std::vector<int>& start) {
        start.assign(S + 1, 0);
        for (int x = 0; x < n; ++x) start[part[x] + 1]++;
        for (int a = 0; a < S; ++a) start[a + 1] += start[a];
        std::vector<int> fill(start.begin(), start.end() - 1);
        ext.resize(n);
        in.resize(n);
        for (int x = 0; x < n; ++x) {
            ext[fill[part[x]]] = x;
            in[x] = fill[part[x]]++;
        }
    };
    order(cpart, M, L.cam_ext, L.cam_int, L.pc);
    order(lpart, N, L.lm_ext, L.lm_int, L.pl);
    for (int a = 0; a < S; ++a)
        if (L.pc[a + 1] - L.pc[a] > DABA_PART_MAX_CAMERAS)
            fail(DABA_E_INVAL, "partition %d has %d cameras (at most %d)", a, L.pc[a + 1] - L.pc[a], DABA_PART_MAX_CAMERAS);
    // observations in (internal camera, internal landmark, caller index)
    // order: a stable counting sort by landmark, then one by camera
    std::vector<int64_t> ord(K);
    {
        std::vector<int64_t> tmp(K), cnt((size_t)std::max(M, N) + 1);
        std::fill(cnt.begin(), cnt.begin() + N + 1, 0);
        for (int64_t o = 0; o < K; ++o) cnt[L.lm_int[pr->obs_landmark[o]] + 1]++;
        for (int j = 0; j < N; ++j) cnt[j + 1] += cnt[j];
        for (int64_t o = 0; o < K; ++o) tmp[cnt[L.lm_int[pr->obs_landmark[o]]]++] = o;
        std::fill(cnt.begin(), cnt.begin() + M + 1, 0);
        for (int64_t o = 0; o < K; ++o) cnt[L.cam_int[pr->obs_camera[o]] + 1]++;
        for (int i = 0; i < M; ++i) cnt[i + 1] += cnt[i];
        for (int64_t q = 0; q < K; ++q) {
            const int64_t o = tmp[q];
            ord[cnt[L.cam_int[pr->obs_camera[o]]]++] = o;
        }
    }
    L.ocam.resize(K);
    L.olm.resize(K);
    L.ointra.resize(K);
    L.ouv.resize(2 * K);
    L.cam_off.assign(M + 1, 0);
    L.lm_off.assign(N + 1, 0);
    for (int64_t q = 0; q < K; ++q) {
        const int64_t o = ord[q];
        const int i = L.cam_int[pr->obs_camera[o]], j = L.lm_int[pr->obs_landmark[o]];
        L.ocam[q] = i;
        L.olm[q] = j;
        L.ointra[q] = cpart[pr->obs_camera[o]] == lpart[pr->obs_landmark[o]] ? 1 : 0;
        L.ouv[2 * q] = pr->obs_uv[2 * o] / L.scale;
        L.ouv[2 * q + 1] = pr->obs_uv[2 * o + 1] / L.scale;
        if (!std::isfinite(L.ouv[2 * q]) || !std::isfinite(L.ouv[2 * q + 1])) fail(DABA_E_INVAL, "obs_uv has a non-finite entry");
        L.cam_off[i + 1]++;
        L.lm_off[j + 1]++;
    }
    for (int i = 0; i < M; ++i) L.cam_off[i + 1] += L.cam_off[i];
    for (int j = 0; j < N; ++j) L.lm_off[j + 1] += L.lm_off[j];
    L.lm_obs.resize(K);
    {
        std::vector<int> fill(L.lm_off.begin(), L.lm_off.end() - 1);
        for (int64_t q = 0; q < K; ++q) L.lm_obs[fill[L.olm[q]]++] = (int)q;
    }
    // reduced systems: order 9 M_a padded to the tile, lower 9x9 blocks
    L.nt.assign(S, 0);
    L.npad.assign(S, 0);
    L.voff.assign(S, 0);
    L.soff.assign(S, 0);
    L.blkbase.assign(S + 1, 0);
    int64_t so = 0;
    int vo = 0;
    for (int a = 0; a < S; ++a) {
        const int ma = L.pc[a + 1] - L.pc[a];
        L.nt[a] = (9 * ma + kNB - 1) / kNB;
        L.npad[a] = kNB * L.nt[a];
        L.soff[a] = so;
        L.voff[a] = vo;
        so += (int64_t)L.npad[a] * L.npad[a];
        vo += L.npad[a];
        L.blkbase[a + 1] = L.blkbase[a] + ma * (ma + 1) / 2;
    }
    L.smat_total = so;
    L.vec_total = vo;
    // pair list: for every landmark, every ordered pair of its exact
    // observations (o1, o2) with camera(o1) >= camera(o2), keyed by block
    const int TB = L.blkbase[S];
    std::vector<int64_t> cnt(TB + 1, 0);
    auto block_of = [&](int a, int q1, int q2) { return L.blkbase[a] + q1 * (q1 + 1) / 2 + q2; };
    std::vector<int> ex;
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<int64_t> fill;
        if (pass == 1) fill.assign(cnt.begin(), cnt.end() - 1);
        int a = 0;
        for (int j = 0; j < N; ++j) {
            while (a + 1 < S && L.pl[a + 1] <= j) ++a;  // landmarks are in partition order
            ex.clear();
            for (int k = L.lm_off[j]; k < L.lm_off[j + 1]; ++k)
                if (L.ointra[L.lm_obs[k]]) ex.push_back(L.lm_obs[k]);
            if (ex.empty()) continue;
            for (int o1 : ex)
                for (int o2 : ex) {
                    const int q1 = L.ocam[o1] - L.pc[a], q2 = L.ocam[o2] - L.pc[a];
                    if (q1 < q2) continue;
                    const int b = block_of(a, q1, q2);
                    if (pass == 0) {
                        cnt[b + 1]++;
                    } else {
                        const int64_t e = fill[b]++;
                        L.ent[2 * e] = o1;
                        L.ent[2 * e + 1] = o2;
                    }
                }
        }
        if (pass == 0) {
            for (int b = 0; b < TB; ++b) cnt[b + 1] += cnt[b];
            if (cnt[TB] > INT32_MAX / 2) fail(DABA_E_INVAL, "too many landmark pairs for the Schur pair list");
            L.ent.assign(2 * (size_t)cnt[TB], 0);
        }
    }
    L.seg_off.resize(TB + 1);
    for (int b = 0; b <= TB; ++b) L.seg_off[b] = (int)cnt[b];
    // reduction chunks, partition by partition
    L.chunk.clear();
    L.chunk_base.assign(S + 1, 0);
    auto add = [&](int kind, int a, int lo, int hi, int step) {
        for (int x = lo; x < hi; x += step) {
            L.chunk.push_back(kind);
            L.chunk.push_back(a);
            L.chunk.push_back(x);
            L.chunk.push_back(std::min(hi, x + step));
        }
    };
    for (int a = 0; a < S; ++a) {
        L.chunk_base[a] = (int)(L.chunk.size() / 4);
        add(CH_CAM_OBS, a, L.cam_off[L.pc[a]], L.cam_off[L.pc[a + 1]], kChunk);
        add(CH_LM_OBS, a, L.lm_off[L.pl[a]], L.lm_off[L.pl[a + 1]], kChunk);
        add(CH_CAM_PROX, a, L.pc[a], L.pc[a + 1], kChunkCam);
        add(CH_LM_PROX, a, L.pl[a], L.pl[a + 1], kChunk);
    }
    L.chunk_base[S] = (int)(L.chunk.size() / 4);
}

struct Carve {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * std::max<size_t>(n, 1);
        return p;
    }
};

struct Bufs {
    double *x_c, *xp_c, *xb_c, *mm_c, *ac_c, *cur_c, *try_c;
    double *x_l, *xp_l, *xb_l, *mm_l, *ac_l, *cur_l, *try_l;
};

void carve(const PLayout& L, Carve& c, PP& p, Bufs& b) {
    const size_t M = L.M, N = L.N, K = (size_t)L.K;
    double** cams[] = {&b.x_c, &b.xp_c, &b.xb_c, &b.mm_c, &b.ac_c, &b.cur_c, &b.try_c};
    double** lms[] = {&b.x_l, &b.xp_l, &b.xb_l, &b.mm_l, &b.ac_l, &b.cur_l, &b.try_l};
    for (auto q : cams) *q = c.take<double>(M * kCS);
    for (auto q : lms) *q = c.take<double>(N * kLS);
    p.ocam = c.take<int>(K);
    p.olm = c.take<int>(K);
    p.ointra = c.take<int>(K);
    p.ouv = c.take<double>(2 * K);
    p.cam_off = c.take<int>(M + 1);
    p.lm_off = c.take<int>(N + 1);
    p.lm_obs = c.take<int>(K);
    p.seg_off = c.take<int>(L.seg_off.size());
    p.ent = c.take<int>(L.ent.size());
    p.chunk = c.take<int4>(L.chunk.size() / 4);
    p.partial = c.take<double>(L.chunk.size() / 4);
    p.vc = c.take<double>(K);
    p.vl = c.take<double>(K);
    p.Hcl = c.take<double>(27 * K);
    p.Hcc = c.take<double>(81 * M);
    p.gc = c.take<double>(16 * M);
    p.W = c.take<double>(9 * N);
    p.Wg = c.take<double>(kLS * N);
    p.Smat = c.take<double>((size_t)L.smat_total);
    p.vec = c.take<double>((size_t)L.vec_total);
    p.dinv = c.take<double>((size_t)L.vec_total);
    p.ps = c.take<double>((size_t)L.S * kPS);
    p.trace = c.take<double>(kTraceCap);
    p.flag = c.take<int>(64);
}

}  // namespace

struct daba_part_handle {
    PP p{};
    Bufs b{};
    PLayout L;
    daba_options opt{};
    hipStream_t stream = nullptr;
    std::string err = "no error";
    int64_t attempts = 0, chol_launches = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    double cat_ms[6] = {0, 0, 0, 0, 0, 0};
    bool timing = false;
    ~daba_part_handle() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

// Timing brackets: when h->timing is set, every launch group is bracketed by
// events and its time added to a category.
enum { C_EVAL = 0, C_BUILD, C_SCHUR, C_CHOL, C_SOLVE, C_REST };

struct Timed {
    daba_part_handle* h;
    int cat;
    Timed(daba_part_handle* hh, int c) : h(hh), cat(c) {
        if (h->timing) hipck(hipEventRecord(h->ev[0], h->stream), "event");
    }
    ~Timed() {
        if (!h->timing) return;
        float ms = 0.f;
        if (hipEventRecord(h->ev[1], h->stream) == hipSuccess && hipEventSynchronize(h->ev[1]) == hipSuccess &&
            hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess)
            h->cat_ms[cat] += ms;
    }
};

inline unsigned gdim(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int LOSS>
void eval_reduce_t(daba_part_handle* h, const double* xc, const double* xl, const double* yc, const double* yl,
                   int mode, int slot) {
    const PP& p = h->p;
    if (p.K > 0) hipLaunchKernelGGL(kp_eval<LOSS>, dim3(gdim(p.K, 256)), dim3(256), 0, h->stream, p, xc, xl, yc, yl, mode);
    const int nch = p.chunk_base[p.S];
    if (nch > 0) hipLaunchKernelGGL(kp_reduce1, dim3(nch), dim3(256), 0, h->stream, p, xc, xl, yc, yl, mode);
    hipLaunchKernelGGL(kp_reduce2, dim3(p.S), dim3(64), 0, h->stream, p, slot);
}

void eval_reduce(daba_part_handle* h, const double* xc, const double* xl, const double* yc, const double* yl,
                 int mode, int slot) {
    Timed t(h, C_EVAL);
    switch (h->p.loss) {
    case DABA_LOSS_HUBER: eval_reduce_t<DABA_LOSS_HUBER>(h, xc, xl, yc, yl, mode, slot); break;
    case DABA_LOSS_WELSCH: eval_reduce_t<DABA_LOSS_WELSCH>(h, xc, xl, yc, yl, mode, slot); break;
    default: eval_reduce_t<DABA_LOSS_TRIVIAL>(h, xc, xl, yc, yl, mode, slot); break;
    }
    hipck(hipGetLastError(), "evaluation");
}

template <int LOSS>
void build_t(daba_part_handle* h, const double* yc, const double* yl) {
    const PP& p = h->p;
    const Bufs& b = h->b;
    hipLaunchKernelGGL(kp_cam_build<LOSS>, dim3(p.M), dim3(256), 0, h->stream, p, b.cur_c, b.cur_l, yc, yl);
    hipLaunchKernelGGL(kp_lm_build<LOSS>, dim3(gdim(p.N, 64)), dim3(64), 0, h->stream, p, b.cur_c, b.cur_l, yc, yl);
    hipLaunchKernelGGL(kp_rhs, dim3(p.M), dim3(64), 0, h->stream, p);
}

// Levenberg-Marquardt of every partition from y (P2 of the partition-level
// reading), or only of the partitions whose restart test failed; the result
// goes to (oc, ol).  Returns false if no partition was solved.
bool lm_all(daba_part_handle* h, const double* yc, const double* yl, double* oc, double* ol, bool only_restarted) {
    const PP& p = h->p;
    const Bufs& b = h->b;
    const unsigned ge = gdim(p.M + p.N, 64);
    {
        Timed t(h, C_REST);
        hipLaunchKernelGGL(kp_lm_init, dim3(1), dim3(64), 0, h->stream, p, only_restarted ? 1 : 0);
        hipck(hipGetLastError(), "LM init");
        if (only_restarted) {  // nothing to solve when every partition kept its accelerated step
            int any = 0;
            hipck(hipMemcpyAsync(&any, p.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream), "flag copy");
            hipck(hipStreamSynchronize(h->stream), "stream sync");
            if (!any) return false;
        }
        hipLaunchKernelGGL(kp_copy, dim3(ge), dim3(64), 0, h->stream, p, yc, yl, b.cur_c, b.cur_l, 0);
    }
    eval_reduce(h, b.cur_c, b.cur_l, yc, yl, EV_E, P_PHI);
    int ntmax = 0;
    for (int a = 0; a < p.S; ++a) ntmax = std::max(ntmax, p.nt[a]);
    const int max_attempts = h->opt.inner_steps + 10 * (h->opt.inner_steps + 1);
    for (int att = 0; att < max_attempts; ++att) {
        {
            Timed t(h, C_BUILD);
            switch (p.loss) {
            case DABA_LOSS_HUBER: build_t<DABA_LOSS_HUBER>(h, yc, yl); break;
            case DABA_LOSS_WELSCH: build_t<DABA_LOSS_WELSCH>(h, yc, yl); break;
            default: build_t<DABA_LOSS_TRIVIAL>(h, yc, yl); break;
            }
            hipck(hipGetLastError(), "normal equations");
        }
        {
            Timed t(h, C_SCHUR);
            if (p.blkbase[p.S] > 0)
                hipLaunchKernelGGL(kp_schur, dim3(gdim(p.blkbase[p.S], 4)), dim3(256), 0, h->stream, p);
            hipck(hipGetLastError(), "Schur complement");
        }
        {
            Timed t(h, C_CHOL);
            // the first diagonal tile; each later one is factored by the
            // update launch that completes it
            hipLaunchKernelGGL(kp_chol_diag, dim3(p.S), dim3(256), 0, h->stream, p, 0);
            h->chol_launches += 1;
            for (int k = 0; k + 1 < ntmax; ++k) {
                const int m = ntmax - k - 1;
                hipLaunchKernelGGL(kp_chol_trsm, dim3(m, p.S), dim3(256), 0, h->stream, p, k);
                hipLaunchKernelGGL(kp_chol_update, dim3(m * (m + 1) / 2, p.S), dim3(256), 0, h->stream, p, k);
                h->chol_launches += 2;
            }
            hipck(hipGetLastError(), "Cholesky");
        }
        {
            Timed t(h, C_SOLVE);
            hipLaunchKernelGGL(kp_trsv, dim3(p.S), dim3(512), 0, h->stream, p);
            hipLaunchKernelGGL(kp_step, dim3(ge), dim3(64), 0, h->stream, p, b.cur_c, b.cur_l, b.try_c, b.try_l);
            hipck(hipGetLastError(), "solve");
        }
        eval_reduce(h, b.try_c, b.try_l, yc, yl, EV_E, P_ETRY);
        int any = 0;
        {
            Timed t(h, C_REST);
            hipLaunchKernelGGL(kp_accept, dim3(1), dim3(64), 0, h->stream, p);
            hipLaunchKernelGGL(kp_copy, dim3(ge), dim3(64), 0, h->stream, p, b.try_c, b.try_l, b.cur_c, b.cur_l, 1);
            hipck(hipGetLastError(), "accept");
            hipck(hipMemcpyAsync(&any, p.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream), "flag copy");
            hipck(hipStreamSynchronize(h->stream), "stream sync");
        }
        ++h->attempts;
        if (!any) break;
    }
    Timed t(h, C_REST);
    hipLaunchKernelGGL(kp_copy, dim3(ge), dim3(64), 0, h->stream, p, b.cur_c, b.cur_l, oc, ol, 0);
    return true;
}

void iterate(daba_part_handle* h, int n, double* F_trace) {
    PP& p = h->p;
    Bufs& b = h->b;
    const unsigned ge = gdim(p.M + p.N, 64);
    for (int done = 0; done < n;) {
        const int chunk = std::min(n - done, kTraceCap);
        for (int it = 0; it < chunk; ++it) {
            {
                Timed t(h, C_REST);
                hipLaunchKernelGGL(kp_nesterov, dim3(1), dim3(64), 0, h->stream, p);
                hipLaunchKernelGGL(kp_extrap, dim3(ge), dim3(64), 0, h->stream, p, b.x_c, b.xp_c, b.x_l, b.xp_l, b.xb_c,
                                   b.xb_l);
            }
            eval_reduce(h, b.x_c, b.x_l, b.xp_c, b.xp_l, EV_GAP, P_RED);  // eq. DEalpha at (x^k | x^(k-1))
            {
                Timed t(h, C_REST);
                hipLaunchKernelGGL(kp_fk, dim3(1), dim3(64), 0, h->stream, p);
            }
            // Algorithm 1: the accelerated step (eq. update_amm) first; the
            // plain MM step (eq. update_mm) only for the partitions whose
            // restart test fails (every partition without acceleration).
            eval_reduce(h, b.x_c, b.x_l, b.x_c, b.x_l, EV_E, P_ECUR);
            if (p.accelerate) {
                lm_all(h, b.xb_c, b.xb_l, b.ac_c, b.ac_l, false);
                eval_reduce(h, b.ac_c, b.ac_l, b.x_c, b.x_l, EV_E, P_EACC);
            }
            {
                Timed t(h, C_REST);
                hipLaunchKernelGGL(kp_restart_test, dim3(1), dim3(64), 0, h->stream, p);
            }
            if (lm_all(h, b.x_c, b.x_l, b.mm_c, b.mm_l, true))
                eval_reduce(h, b.mm_c, b.mm_l, b.x_c, b.x_l, EV_E, P_EMM);
            {
                Timed t(h, C_REST);
                hipLaunchKernelGGL(kp_restart_finish, dim3(1), dim3(64), 0, h->stream, p);
                hipLaunchKernelGGL(kp_roll, dim3(ge), dim3(64), 0, h->stream, p, b.x_c, b.xp_c, b.mm_c, b.ac_c, b.x_l,
                                   b.xp_l, b.mm_l, b.ac_l);
            }
            eval_reduce(h, b.x_c, b.x_l, b.x_c, b.x_l, EV_F, P_RED);
            {
                Timed t(h, C_REST);
                hipLaunchKernelGGL(kp_trace, dim3(1), dim3(64), 0, h->stream, p, it);
                hipck(hipGetLastError(), "iteration");
            }
        }
        std::vector<double> tr(chunk);
        hipck(hipMemcpyAsync(tr.data(), p.trace, sizeof(double) * chunk, hipMemcpyDeviceToHost, h->stream), "trace copy");
        hipck(hipStreamSynchronize(h->stream), "stream sync");
        const double s2 = h->L.scale * h->L.scale;
        for (int it = 0; it < chunk; ++it) {
            if (!std::isfinite(tr[it])) fail(DABA_E_NONFINITE, "non-finite objective at iteration %d", done + it);
            if (F_trace) F_trace[done + it] = s2 * tr[it];
        }
        done += chunk;
    }
}

}  // namespace

extern "C" {

size_t daba_part_workspace_bytes(const daba_problem* prob, const daba_options* opt) {
    try {
        validate_options(opt);
        PLayout L;
        build_layout(prob, L);
        Carve c{nullptr};
        PP p{};
        Bufs b{};
        carve(L, c, p, b);
        return c.off;
    } catch (...) {
        return 0;
    }
}

int daba_part_create(const daba_problem* prob, const daba_options* opt, void* dev_workspace, size_t workspace_bytes,
                     void* hip_stream, daba_part_handle** out) {
    if (!out) {
        g_err = "out is NULL";
        return DABA_E_INVAL;
    }
    *out = nullptr;
    daba_part_handle* h = nullptr;
    try {
        validate_options(opt);
        if (!prob) fail(DABA_E_INVAL, "problem is NULL");
        if (!prob->cameras || !prob->landmarks) fail(DABA_E_INVAL, "problem arrays are NULL");
        for (int64_t i = 0; i < prob->n_cameras; ++i) {
            const double* c = prob->cameras + 15 * (size_t)i;
            for (int a = 0; a < 15; ++a)
                if (!std::isfinite(c[a])) fail(DABA_E_INVAL, "camera %lld has a non-finite entry", (long long)i);
            if (!rotation_ok(c)) fail(DABA_E_INVAL, "camera %lld: R is not a rotation", (long long)i);
        }
        for (int64_t j = 0; j < 3 * prob->n_landmarks; ++j)
            if (!std::isfinite(prob->landmarks[j])) fail(DABA_E_INVAL, "landmarks have a non-finite entry");
        h = new daba_part_handle();
        h->opt = *opt;
        h->stream = (hipStream_t)hip_stream;
        build_layout(prob, h->L);
        const PLayout& L = h->L;
        for (int64_t o = 0; o < prob->n_obs; ++o) {  // Assumption 2 at x^(0)
            const double* t = prob->cameras + 15 * (size_t)prob->obs_camera[o] + 9;
            const double* l = prob->landmarks + 3 * (size_t)prob->obs_landmark[o];
            const double m0 = l[0] - t[0], m1 = l[1] - t[1], m2 = l[2] - t[2];
            if (!(m0 * m0 + m1 * m1 + m2 * m2 > 1e-24))
                fail(DABA_E_DEGENERATE, "observation %lld: landmark at the camera centre (Assumption 2)", (long long)o);
        }
        Carve cz{nullptr};
        PP tmp{};
        Bufs tb{};
        carve(L, cz, tmp, tb);
        if (!dev_workspace) fail(DABA_E_INVAL, "workspace is NULL");
        if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) fail(DABA_E_INVAL, "workspace must be 256-byte aligned");
        if (workspace_bytes < cz.off) fail(DABA_E_NOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, cz.off);
        Carve cv{static_cast<char*>(dev_workspace)};
        PP& p = h->p;
        carve(L, cv, p, h->b);
        p.M = L.M;
        p.N = L.N;
        p.S = L.S;
        p.K = L.K;
        p.loss = opt->loss;
        p.delta = opt->loss == DABA_LOSS_TRIVIAL ? 1.0 : opt->loss_delta / L.scale;
        p.xi = opt->xi;
        p.eta = opt->eta;
        p.accelerate = opt->accelerate;
        p.inner_steps = opt->inner_steps;
        p.flags = opt->debug_flags;
        for (int a = 0; a <= L.S; ++a) {
            p.pc[a] = L.pc[a];
            p.pl[a] = L.pl[a];
            p.blkbase[a] = L.blkbase[a];
        }
        for (int a = 0; a < L.S; ++a) {
            p.nt[a] = L.nt[a];
            p.npad[a] = L.npad[a];
            p.soff[a] = L.soff[a];
            p.voff[a] = L.voff[a];
        }
        hipStream_t s = h->stream;
        auto up = [&](void* dst, const void* src, size_t bytes) {
            if (bytes) hipck(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "upload");
        };
        const size_t K = (size_t)L.K;
        up((void*)p.ocam, L.ocam.data(), 4 * K);
        up((void*)p.olm, L.olm.data(), 4 * K);
        up((void*)p.ointra, L.ointra.data(), 4 * K);
        up((void*)p.ouv, L.ouv.data(), 16 * K);
        up((void*)p.cam_off, L.cam_off.data(), 4 * L.cam_off.size());
        up((void*)p.lm_off, L.lm_off.data(), 4 * L.lm_off.size());
        up((void*)p.lm_obs, L.lm_obs.data(), 4 * K);
        up((void*)p.seg_off, L.seg_off.data(), 4 * L.seg_off.size());
        up((void*)p.ent, L.ent.data(), 4 * L.ent.size());
        up((void*)p.chunk, L.chunk.data(), 4 * L.chunk.size());
        for (int a = 0; a <= L.S; ++a) p.chunk_base[a] = L.chunk_base[a];
        std::vector<double> cam((size_t)L.M * kCS, 0.0), lm((size_t)L.N * kLS, 0.0);
        const double sc = L.scale;
        for (int q = 0; q < L.M; ++q) {
            const double* c = prob->cameras + 15 * (size_t)L.cam_ext[q];
            double* d = &cam[(size_t)q * kCS];
            for (int a = 0; a < 12; ++a) d[a] = c[a];
            d[12] = c[12] / sc;
            d[13] = c[13] * sc;
            d[14] = c[14] * sc * sc * sc;
        }
        for (int q = 0; q < L.N; ++q)
            for (int a = 0; a < 3; ++a) lm[(size_t)q * kLS + a] = prob->landmarks[3 * (size_t)L.lm_ext[q] + a];
        const Bufs& b = h->b;
        for (double* d : {b.x_c, b.xp_c, b.xb_c, b.mm_c, b.ac_c, b.cur_c, b.try_c}) up(d, cam.data(), 8 * cam.size());
        for (double* d : {b.x_l, b.xp_l, b.xb_l, b.mm_l, b.ac_l, b.cur_l, b.try_l}) up(d, lm.data(), 8 * lm.size());
        if (L.smat_total > 0)
            hipLaunchKernelGGL(kp_init_smat, dim3(gdim(L.smat_total, 256)), dim3(256), 0, s, p, L.smat_total);
        // the padding entries of the right-hand sides are never written and
        // must be zero (they meet zero rows of L in the substitutions)
        if (L.vec_total > 0) hipck(hipMemsetAsync(p.vec, 0, sizeof(double) * (size_t)L.vec_total, s), "memset");
        hipck(hipGetLastError(), "init");
        for (auto& e : h->ev) hipck(hipEventCreate(&e), "event create");
        eval_reduce(h, b.x_c, b.x_l, b.x_c, b.x_l, EV_E, P_RED);  // eq. Fainit
        hipLaunchKernelGGL(kp_init_metrics, dim3(1), dim3(64), 0, s, p);
        hipck(hipGetLastError(), "init");
        hipck(hipStreamSynchronize(s), "stream sync");
        *out = h;
        return DABA_OK;
    } catch (const Fail& f) {
        g_err = f.msg;
        delete h;
        return f.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        delete h;
        return DABA_E_NOMEM;
    }
}

int daba_part_iterate(daba_part_handle* h, int n_iters, double* F_trace) {
    if (!h) return DABA_E_INVAL;
    try {
        if (n_iters < 0) fail(DABA_E_INVAL, "n_iters must be >= 0");
        iterate(h, n_iters, F_trace);
        return DABA_OK;
    } catch (const Fail& f) {
        h->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        h->err = "host allocation failed";
        return DABA_E_NOMEM;
    }
}

int daba_part_iterate_timed(daba_part_handle* h, int n_iters, double* ms_out) {
    if (!h) return DABA_E_INVAL;
    try {
        if (n_iters < 0 || !ms_out) fail(DABA_E_INVAL, "n_iters must be >= 0 and ms_out not NULL");
        for (double& v : h->cat_ms) v = 0.0;
        h->attempts = h->chol_launches = 0;
        h->timing = true;
        try {
            iterate(h, n_iters, nullptr);
        } catch (...) {
            h->timing = false;
            throw;
        }
        h->timing = false;
        for (int c = 0; c < 6; ++c) ms_out[c] = h->cat_ms[c];
        ms_out[6] = (double)h->attempts;
        ms_out[7] = (double)h->chol_launches;
        return DABA_OK;
    } catch (const Fail& f) {
        h->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        h->err = "host allocation failed";
        return DABA_E_NOMEM;
    }
}

int daba_part_get_state(daba_part_handle* h, double* cams, double* lms, double* metrics) {
    if (!h) return DABA_E_INVAL;
    try {
        const PLayout& L = h->L;
        hipck(hipStreamSynchronize(h->stream), "stream sync");
        const double sc = L.scale;
        if (cams) {
            std::vector<double> c((size_t)L.M * kCS);
            hipck(hipMemcpy(c.data(), h->b.x_c, 8 * c.size(), hipMemcpyDeviceToHost), "download");
            for (int q = 0; q < L.M; ++q) {
                const double* s = &c[(size_t)q * kCS];
                double* d = cams + 15 * (size_t)L.cam_ext[q];
                for (int a = 0; a < 12; ++a) d[a] = s[a];
                d[12] = s[12] * sc;
                d[13] = s[13] / sc;
                d[14] = s[14] / (sc * sc * sc);
            }
        }
        if (lms) {
            std::vector<double> l((size_t)L.N * kLS);
            hipck(hipMemcpy(l.data(), h->b.x_l, 8 * l.size(), hipMemcpyDeviceToHost), "download");
            for (int q = 0; q < L.N; ++q)
                for (int a = 0; a < 3; ++a) lms[3 * (size_t)L.lm_ext[q] + a] = l[(size_t)q * kLS + a];
        }
        if (metrics) {
            std::vector<double> ps((size_t)L.S * kPS);
            hipck(hipMemcpy(ps.data(), h->p.ps, 8 * ps.size(), hipMemcpyDeviceToHost), "download");
            const double s2 = sc * sc;
            for (int a = 0; a < L.S; ++a) {
                const double* q = &ps[(size_t)a * kPS];
                metrics[4 * a + 0] = s2 * q[P_FK];
                metrics[4 * a + 1] = s2 * q[P_FBAR];
                metrics[4 * a + 2] = s2 * q[P_E];
                metrics[4 * a + 3] = q[P_RESTART];
            }
        }
        return DABA_OK;
    } catch (const Fail& f) {
        h->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        h->err = "host allocation failed";
        return DABA_E_NOMEM;
    }
}

}  // extern "C"

namespace {

void download_cams(daba_part_handle* h, const double* dev, double* out) {
    const PLayout& L = h->L;
    const double sc = L.scale;
    std::vector<double> c((size_t)L.M * kCS);
    hipck(hipMemcpy(c.data(), dev, 8 * c.size(), hipMemcpyDeviceToHost), "download");
    for (int q = 0; q < L.M; ++q) {
        const double* s = &c[(size_t)q * kCS];
        double* d = out + 15 * (size_t)L.cam_ext[q];
        for (int a = 0; a < 12; ++a) d[a] = s[a];
        d[12] = s[12] * sc;
        d[13] = s[13] / sc;
        d[14] = s[14] / (sc * sc * sc);
    }
}

void download_lms(daba_part_handle* h, const double* dev, double* out) {
    const PLayout& L = h->L;
    std::vector<double> l((size_t)L.N * kLS);
    hipck(hipMemcpy(l.data(), dev, 8 * l.size(), hipMemcpyDeviceToHost), "download");
    for (int q = 0; q < L.N; ++q)
        for (int a = 0; a < 3; ++a) out[3 * (size_t)L.lm_ext[q] + a] = l[(size_t)q * kLS + a];
}

void upload_cams(daba_part_handle* h, const double* in, double* dev) {
    const PLayout& L = h->L;
    const double sc = L.scale;
    std::vector<double> c((size_t)L.M * kCS, 0.0);
    for (int q = 0; q < L.M; ++q) {
        const double* s = in + 15 * (size_t)L.cam_ext[q];
        double* d = &c[(size_t)q * kCS];
        for (int a = 0; a < 15; ++a)
            if (!std::isfinite(s[a])) fail(DABA_E_INVAL, "camera %d has a non-finite entry", L.cam_ext[q]);
        for (int a = 0; a < 12; ++a) d[a] = s[a];
        d[12] = s[12] / sc;
        d[13] = s[13] * sc;
        d[14] = s[14] * sc * sc * sc;
    }
    hipck(hipMemcpyAsync(dev, c.data(), 8 * c.size(), hipMemcpyHostToDevice, h->stream), "upload");
    hipck(hipStreamSynchronize(h->stream), "stream sync");  // the staging vector goes out of scope
}

void upload_lms(daba_part_handle* h, const double* in, double* dev) {
    const PLayout& L = h->L;
    std::vector<double> l((size_t)L.N * kLS, 0.0);
    for (int q = 0; q < L.N; ++q)
        for (int a = 0; a < 3; ++a) {
            const double v = in[3 * (size_t)L.lm_ext[q] + a];
            if (!std::isfinite(v)) fail(DABA_E_INVAL, "landmark %d has a non-finite entry", L.lm_ext[q]);
            l[(size_t)q * kLS + a] = v;
        }
    hipck(hipMemcpyAsync(dev, l.data(), 8 * l.size(), hipMemcpyHostToDevice, h->stream), "upload");
    hipck(hipStreamSynchronize(h->stream), "stream sync");
}

}  // namespace

extern "C" {

int daba_part_get_checkpoint(daba_part_handle* h, double* cams, double* lms, double* cams_prev, double* lms_prev,
                             double* part3) {
    if (!h) return DABA_E_INVAL;
    try {
        hipck(hipStreamSynchronize(h->stream), "stream sync");
        if (cams) download_cams(h, h->b.x_c, cams);
        if (lms) download_lms(h, h->b.x_l, lms);
        if (cams_prev) download_cams(h, h->b.xp_c, cams_prev);
        if (lms_prev) download_lms(h, h->b.xp_l, lms_prev);
        if (part3) {
            const int S = h->L.S;
            std::vector<double> ps((size_t)S * kPS);
            hipck(hipMemcpy(ps.data(), h->p.ps, 8 * ps.size(), hipMemcpyDeviceToHost), "download");
            const double s2 = h->L.scale * h->L.scale;
            for (int a = 0; a < S; ++a) {
                part3[3 * a + 0] = s2 * ps[(size_t)a * kPS + P_FBAR];
                part3[3 * a + 1] = s2 * ps[(size_t)a * kPS + P_E];
                part3[3 * a + 2] = ps[(size_t)a * kPS + P_S];
            }
        }
        return DABA_OK;
    } catch (const Fail& f) {
        h->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        h->err = "host allocation failed";
        return DABA_E_NOMEM;
    }
}

int daba_part_set_checkpoint(daba_part_handle* h, const double* cams, const double* lms, const double* cams_prev,
                             const double* lms_prev, const double* part3) {
    if (!h) return DABA_E_INVAL;
    try {
        hipck(hipStreamSynchronize(h->stream), "stream sync");
        // every input is checked before anything is changed, so that a call
        // that fails leaves the handle as it was
        const PLayout& L = h->L;
        for (const double* cs : {cams, cams_prev}) {
            if (!cs) continue;
            for (int64_t i = 0; i < L.M; ++i) {
                const double* c = cs + 15 * (size_t)i;
                for (int a = 0; a < 15; ++a)
                    if (!std::isfinite(c[a])) fail(DABA_E_INVAL, "camera %lld has a non-finite entry", (long long)i);
                if (!rotation_ok(c)) fail(DABA_E_INVAL, "camera %lld: R is not a rotation", (long long)i);
            }
        }
        for (const double* ls : {lms, lms_prev}) {
            if (!ls) continue;
            for (int64_t j = 0; j < 3 * (int64_t)L.N; ++j)
                if (!std::isfinite(ls[j])) fail(DABA_E_INVAL, "landmarks have a non-finite entry");
        }
        if (part3)
            for (int a = 0; a < L.S; ++a) {
                for (int c = 0; c < 3; ++c)
                    if (!std::isfinite(part3[3 * a + c])) fail(DABA_E_INVAL, "part3 has a non-finite entry");
                if (!(part3[3 * a + 2] >= 1.0)) fail(DABA_E_INVAL, "s^a must be >= 1");
            }
        if (cams) upload_cams(h, cams, h->b.x_c);
        if (lms) upload_lms(h, lms, h->b.x_l);
        if (cams_prev) upload_cams(h, cams_prev, h->b.xp_c);
        if (lms_prev) upload_lms(h, lms_prev, h->b.xp_l);
        if (part3) {
            const int S = h->L.S;
            std::vector<double> ps((size_t)S * kPS);
            hipck(hipMemcpy(ps.data(), h->p.ps, 8 * ps.size(), hipMemcpyDeviceToHost), "download");
            const double s2 = h->L.scale * h->L.scale;
            for (int a = 0; a < S; ++a) {
                ps[(size_t)a * kPS + P_FBAR] = part3[3 * a + 0] / s2;
                ps[(size_t)a * kPS + P_E] = part3[3 * a + 1] / s2;
                ps[(size_t)a * kPS + P_S] = part3[3 * a + 2];
            }
            hipck(hipMemcpy(h->p.ps, ps.data(), 8 * ps.size(), hipMemcpyHostToDevice), "upload");
        }
        return DABA_OK;
    } catch (const Fail& f) {
        h->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        h->err = "host allocation failed";
        return DABA_E_NOMEM;
    }
}

int daba_part_destroy(daba_part_handle* h) {
    delete h;
    return DABA_OK;
}

const char* daba_part_last_error(const daba_part_handle* h) {
    if (!h) return g_err.c_str();
    return h->err.c_str();
}

}  // extern "C"
