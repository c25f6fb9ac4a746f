// gfx950 kernels of one DABA iteration (Fan et al., Algorithm 1, Sec. VI)
// with every observation majorized (Prop. 1): the surrogate separates per
// camera and per landmark, and camera partitions act as the devices of the
// adaptive restart (Sec. V).
//
// Per iteration k (k mod 3 picks the camera generation, k mod 2 the parity
// of the candidate buffers), three launches:
//   k_decide   (one block per partition) the restart test of iteration
//              k - 1 (eq. Fak, lFak, Eak), which picks each partition's
//              candidate (eq. update_amm or update_mm) as x^k;
//   k_obs_dma  one wave per camera tile evaluates every observation at x^k,
//              taken from that candidate, at the extrapolated
//              x-bar^k and at x^(k-1); accumulates the camera moments of both
//              surrogates (FP64), the F share and the surrogate-gap share;
//              bins the landmark-side shares per partition; writes the
//              landmark-side record to its slot.
//   k_entity   camera subproblems (Levenberg-Marquardt on the moments, and
//              the next extrapolation of each candidate, eq. nesterov_x) and,
//              in other blocks of the same launch, the column sums of the
//              partition bins (the first also sums the objective the restart
//              test split by partition) and landmark subproblems (one lane
//              per landmark: the records k_obs_dma wrote at its slots, then
//              the closed form).
// At the end of a call a last k_decide takes the restart test, and
// k_finalize writes the chosen candidates everywhere, so that between calls
// x^k is stored plainly.
//
// Numerics.  Camera statistics are taken about the linearization point y
// (Appendix-style moment form): with z = (ux, uy, 1, |u|^2, |u|^4, lambda),
// Z = sum w z z^T and Y = sum w r^y z^T where r^y = (R p + lambda t - g)|_y =
// e_w / 2 (the touching identity behind eq. approx0), the camera surrogate is
//   Phi(c) - Phi(y) = tr(Mx Z Mx^T) + 2 tr(Mx^T Y) + prox,
// with Mx the 3x6 map z -> R p(d) - R^y p(d^y) + lambda (t - t^y).  Every term
// is small near y, so no large cancelling sums appear.  The landmark side
// uses W = sum w lambda^2 and V = sum w lambda e_w: its minimizer is
// l^y + V / (2W + xi) and its surrogate change is (W + xi/2)|dl|^2 - dl . V.
#include "daba_internal.h"
#include "daba_rotation.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

namespace daba {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

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

// Moments of one surrogate (see header comment): a[0..19] = Z, a[20..37] = Y.
// The per-observation quantities (FP32 in the mixed form) are widened once;
// products and sums are FP64.
template <typename R>
__device__ __forceinline__ void add_moments(double* a, R w_, R lam_, R ux_, R uy_, R r2_, R r4_, R r6_, R r8_,
                                            const R* e) {
    const double w = (double)w_, lam = (double)lam_, ux = (double)ux_, uy = (double)uy_;
    const double r2 = (double)r2_, r4 = (double)r4_, r6 = (double)r6_, r8 = (double)r8_;
    const double wu = w * ux, wv = w * uy, wl = w * lam;
    a[0] += wu * ux;
    a[1] += wu * uy;
    a[2] += wv * uy;
    a[3] += wu;
    a[4] += wu * r2;
    a[5] += wu * r4;
    a[6] += wv;
    a[7] += wv * r2;
    a[8] += wv * r4;
    a[9] += w;
    a[10] += w * r2;
    a[11] += w * r4;
    a[12] += w * r6;
    a[13] += w * r8;
    a[14] += wl * ux;
    a[15] += wl * uy;
    a[16] += wl;
    a[17] += wl * r2;
    a[18] += wl * r4;
    a[19] += wl * lam;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double g = 0.5 * w * (double)e[k];  // w r^y with r^y = e_w / 2
        a[20 + 6 * k + 0] += g * ux;
        a[20 + 6 * k + 1] += g * uy;
        a[20 + 6 * k + 2] += g;
        a[20 + 6 * k + 3] += g * r2;
        a[20 + 6 * k + 4] += g * r4;
        a[20 + 6 * k + 5] += g * lam;
    }
}

template <typename R>
struct LmRead {
    R lk[3], lp[3];
    int beta;
};

__device__ __forceinline__ LmRead<double> read_pair(const double* __restrict__ base, int li) {
    const double2* q = reinterpret_cast<const double2*>(base + (size_t)li * kLmPair);
    double2 a = q[0], b = q[1], c = q[2], d = q[3];
    LmRead<double> o;
    o.lk[0] = a.x; o.lk[1] = a.y; o.lk[2] = b.x;
    o.beta = (int)__double_as_longlong(b.y);
    o.lp[0] = c.x; o.lp[1] = c.y; o.lp[2] = d.x;
    return o;
}

__device__ __forceinline__ LmRead<float> read_pair(const float* __restrict__ base, int li) {
    const float4* q = reinterpret_cast<const float4*>(base + (size_t)li * kLmPair);
    float4 a = q[0], b = q[1];
    LmRead<float> o;
    o.lk[0] = a.x; o.lk[1] = a.y; o.lk[2] = a.z;
    o.beta = __float_as_int(a.w);
    o.lp[0] = b.x; o.lp[1] = b.y; o.lp[2] = b.z;
    return o;
}

// candidate pair records read by iteration k (written by iteration k - 1)
template <typename R>
__device__ __forceinline__ const R* pair_base(const Params& p, int k, int cand);
template <>
__device__ __forceinline__ const double* pair_base<double>(const Params& p, int k, int cand) {
    return p.lcp[(k + 1) & 1][cand];
}
template <>
__device__ __forceinline__ const float* pair_base<float>(const Params& p, int k, int cand) {
    return p.lcp32[(k + 1) & 1][cand];
}

template <typename R>
__device__ __forceinline__ R* rec_base(const Params& p);
template <>
__device__ __forceinline__ double* rec_base<double>(const Params& p) { return p.rec; }
template <>
__device__ __forceinline__ float* rec_base<float>(const Params& p) { return p.rec32; }

// Segmented sum over lanes whose keys are sorted (equal keys contiguous);
// the last lane of each run adds the run's sum into bins[key].
__device__ __forceinline__ void bin_add_sorted(double v0, double v1, int key, int lane, double* bins0,
                                               double* bins1) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        double o0 = __shfl_up(v0, d, kWave);
        double o1 = __shfl_up(v1, d, kWave);
        int ok = __shfl_up(key, d, kWave);
        if (lane >= d && ok == key) {
            v0 += o0;
            v1 += o1;
        }
    }
    int nk = __shfl_down(key, 1, kWave);
    bool last = (lane == kWave - 1) || (nk != key);
    if (last && key >= 0) {
        bins0[key] += v0;
        bins1[key] += v1;
    }
}

// Adds a run's per-lane sums into bins[key] (no-op for key < 0) and clears them.
__device__ __forceinline__ void flush_run(int key, double& r0, double& r1, int lane, double* bins0, double* bins1) {
    if (key >= 0) {
        const double s0 = wave_sum(r0), s1 = wave_sum(r1);
        if (lane == 0) {
            bins0[key] += s0;
            bins1[key] += s1;
        }
    }
    r0 = 0.0;
    r1 = 0.0;
}

// --------------------------------------------------- restart test (Sec. V)

// eq. nesterov_scalar: s^(k+1) from s^(k), and gamma^(k+1) = (s^(k+1) - 1) / s^(k+2)
__device__ __forceinline__ double next_gamma(const Params& p, double s, double* s1_out) {
    const double s1 = (sqrt(4.0 * s * s + 1.0) + 1.0) / 2.0;
    const double s2 = (sqrt(4.0 * s1 * s1 + 1.0) + 1.0) / 2.0;
    *s1_out = s1;
    return p.accelerate ? (s1 - 1.0) / s2 : 0.0;
}

// Restart test of iteration kp (eq. Fak, lFak, Eak), one block per
// partition a = blockIdx.x.  The block sums the values k_entity left for
// partition a (its camera blocks' and landmark blocks' sums, threads
// strided, then a fixed-order block reduction) and thread 0 takes the test.
// It stores the bookkeeping of slot (kp + 1) & 1, the metrics, the flag
// (1: the partition restarts, i.e. keeps the plain MM candidate) and the
// partition's share of F(x^kp).  Block 0 also stores the next Nesterov
// state and the iteration count.  Every input is requested before the
// first wait; with skip_if_decided the block returns, before any store,
// when the test is already stored.  kp may be -1.
__device__ void restart_test_part(const Params& p, int kp, bool skip_if_decided, double (*red)[6]) {
    const int a = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int S = p.S;
    const int cur = (kp & 1) * S;
    const int decided = skip_if_decided ? p.st[0].decided : 0;
    double E = 0.0, EE = 0.0, Fbar = 0.0, col0 = 0.0, col1 = 0.0, s_in = 0.0;
    int64_t k_in = 0;
    if (tid == 0) {
        E = p.E[cur + a];
        EE = p.EE[cur + a];
        Fbar = p.Fbar[cur + a];
        col0 = p.colsum[a];
        col1 = p.colsum[S + a];
        if (a == 0) {
            s_in = p.st[kp & 1].s;
            k_in = p.st[kp & 1].k;
        }
    }
    double c[4] = {0, 0, 0, 0}, l[2] = {0, 0};
    {
        const int c0 = p.pcb[a], nc = p.pcb[a + 1] - c0, l0 = p.plb[a], nl = p.plb[a + 1] - l0;
        const int n = nc > nl ? nc : nl;
        // unrolled so that several rounds of loads are in flight together
#pragma unroll 4
        for (int q = tid; q < n; q += 256) {
            if (q < nc) {
                const double4 v = *reinterpret_cast<const double4*>(p.camblk_vals + (size_t)(c0 + q) * 4);
                c[0] += v.x; c[1] += v.y; c[2] += v.z; c[3] += v.w;
            }
            if (q < nl) {
                const double2 v = *reinterpret_cast<const double2*>(p.lmblk_vals + (size_t)(l0 + q) * 2);
                l[0] += v.x; l[1] += v.y;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] = wave_sum(c[q]);
    l[0] = wave_sum(l[0]);
    l[1] = wave_sum(l[1]);
    if (decided) return;  // uniform over the block
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wv][q] = c[q];
        red[wv][4] = l[0];
        red[wv][5] = l[1];
    }
    __syncthreads();
    if (tid != 0) return;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double v = 0.0;
        for (int w = 0; w < 4; ++w) v += red[w][q];
        if (q < 4) c[q] = v;
        else l[q - 4] = v;
    }
    const int nxt = ((kp + 1) & 1) * S;
    // E^a(x^k | x^k): each pair's F split in halves between its sides
    const double Fsh = c[2] + col0;
    // [E^a + DeltaE^a](x^k | x^(k-1)) = Fsh + cross-partition gap shares
    const double V = Fsh + c[3] + col1;
    const double Fk = E + V - EE;                        // eq. Fak
    const double Fb = (1.0 - p.eta) * Fbar + p.eta * Fk;  // eq. lFak
    const double dmm = c[0] + l[0], dacc = c[1] + l[1];
    int rs = p.accelerate ? (Fk + dacc > Fb) : 1;        // eq. Eak test
    if (p.accelerate && (p.flags & 1)) rs = 0;
    if (p.accelerate && (p.flags & 2)) rs = 1;
    const double dch = rs ? dmm : dacc;
    p.Fprev[nxt + a] = Fk;
    p.Fbar[nxt + a] = Fb;
    p.E[nxt + a] = Fk + dch;
    p.EE[nxt + a] = Fsh + dch;
    p.metrics[4 * a + 0] = Fk;
    p.metrics[4 * a + 1] = Fb;
    p.metrics[4 * a + 2] = Fk + dch;
    p.metrics[4 * a + 3] = (double)rs;
    p.restart[a] = rs;
    p.fsh[a] = Fsh;
    if (a == 0) {
        double s1;
        const double gam = next_gamma(p, s_in, &s1);
        DevState& sn = p.st[(kp + 1) & 1];
        sn.s = s1;
        sn.gamma = gam;
        sn.k = k_in + 1;
    }
}

// Start of iteration k: the restart test of iteration k - 1, unless it is
// already stored (after daba_create, daba_set_state or a previous call).
// One block per partition.
__global__ __launch_bounds__(256) void k_decide(Params p, int k, int skip_if_decided) {
    __shared__ double red[4][6];
    restart_test_part(p, k - 1, skip_if_decided != 0, red);
}

// F(x^(k-1)) from the partition shares the restart test of iteration k - 1
// stored (summed in partition order), into the trace and the state of slot
// k & 1; a non-finite F sets the sticky error.  All threads of the block
// call it.
__device__ void store_trace(const Params& p, int k, double* sh) {
    if ((int)threadIdx.x < p.S) sh[threadIdx.x] = p.fsh[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        double F = 0.0;
        for (int a = 0; a < p.S; ++a) F += sh[a];
        if (!isfinite(F) && p.st[0].err == 0) p.st[0].err = -4;  // a degenerate point reported first wins
        DevState& sc = p.st[k & 1];
        const int64_t kk = sc.k - 1;
        if (kk >= 0) p.trace[kk & (int64_t)(p.trace_cap - 1)] = F;
        sc.F = F;
    }
}

// The restart flags of iteration k - 1 as a bit mask (stored by k_decide).
__device__ __forceinline__ uint64_t restart_mask(const Params& p) {
    const int lane = threadIdx.x & (kWave - 1);
    return __ballot(lane < p.S && p.restart[lane] != 0);
}
// candidate chosen for partition a: 0 (plain MM) on restart, else 1
__device__ __forceinline__ int chosen(uint64_t restart, int a) { return ((restart >> a) & 1) ? 0 : 1; }

// ------------------------------------- observation pass, restructured form
// The observation pass with its memory traffic restructured for gfx950
// (FP64, and FP32-mixed with 32-byte records):
//  * a step's 64 landmark pair records are fetched straight into LDS
//    (global_load_lds, no VGPRs), several lanes per record (16 bytes each) so
//    that a wave instruction touches a few cache lines instead of 64; pixels
//    and slots come the same way.  The fetch for step s + 1 is issued while
//    step s computes, into the other of two buffers, and the landmark
//    indices it needs are loaded one step earlier still;
//  * the landmark-side records of step s are staged in LDS and written at
//    the start of step s + 1, again several lanes per record.  On this
//    target a load's wait also waits for every store issued before it, so
//    stores go out right after a step's wait, a whole step ahead of the next.
// Every wave waits for all of its vector memory operations at the start of
// a step, explicitly: the compiler does not order an LDS read after an LDS
// DMA into the same object.  The two buffers are separate objects, so that
// reading one while the other is being filled needs no wait.
constexpr int kRedHalf = 7;  // rows of the reduction transpose per buffer (7 x 65 <= 512)
template <typename R>
struct ObsBuf;
template <>
struct __align__(16) ObsBuf<double> {
    double pair[kWave * kLmPair];  // pair records of a step, in observation order
    double2 uv[kWave];
    int slot[kWave];
    __device__ double* red() { return pair; }  // reused for the tile reduction
};
template <>
struct __align__(16) ObsBuf<float> {
    float pair[kWave * kLmPair];
    float ux[kWave], uy[kWave];
    int slot[kWave];
    double red_[kRedHalf * (kWave + 1)];
    __device__ double* red() { return red_; }
};
static_assert(kRedHalf * (kWave + 1) <= kWave * kLmPair, "reduction fits a pair buffer");

typedef __attribute__((address_space(3))) void* lds_ptr;
__device__ __forceinline__ void dma16(const void* g, void* l) {
    __builtin_amdgcn_global_load_lds(g, (lds_ptr)l, 16, 0, 0);
}
__device__ __forceinline__ void dma4(const void* g, void* l) {
    __builtin_amdgcn_global_load_lds(g, (lds_ptr)l, 4, 0, 0);
}
// vmcnt(0) with expcnt and lgkmcnt left alone (gfx9 encoding); the builtin
// keeps the compiler's own wait bookkeeping informed, the empty asm keeps
// memory accesses from moving across it
__device__ __forceinline__ void wait_vmem() {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// One wave per workgroup (one tile each): every LDS address is then a
// compile-time offset from the lane's own, which keeps VGPRs for the 78
// FP64 accumulators.
template <typename R, int LOSS, bool ACC>
__global__ __launch_bounds__(kWave) void k_obs_dma(Params p, int k) {
    constexpr int kRecB = 8 * (int)sizeof(R);  // bytes of a pair record and of a landmark-side record
    constexpr int kLPR = kRecB / 16;           // lanes per record
    constexpr int kRPI = kWave / kLPR;         // records per wave instruction
    constexpr int kNI = kWave / kRPI;          // instructions per step
    constexpr int kEPC = 16 / (int)sizeof(R);  // elements per 16-byte chunk
    __shared__ ObsBuf<R> A;
    __shared__ ObsBuf<R> B;
    __shared__ __align__(16) R stg[kWave * 8];  // landmark-side records of a step
    __shared__ double bins[2][kMaxPart];
    __shared__ double cprev[kCamRec];  // x^(k-1) of the tile's camera (used by the gap only)
    __shared__ double cbarl[kCamRec];  // x-bar^k of the tile's camera
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    const bool active = t < p.T;
    const int S = p.S;

    for (int b = lane; b < S; b += kWave) {
        bins[0][b] = 0.0;
        bins[1][b] = 0.0;
    }

    // the 2 x 38 moments; the tile's F and gap shares are the sums of its
    // partition bins
    constexpr int kAccR = 2 * kMom;
    double acc[kAccR];
#pragma unroll
    for (int a = 0; a < kAccR; ++a) acc[a] = 0.0;

    const uint64_t restart = restart_mask(p);
    int beg = 0, end = 0, ci = 0, alpha = 0;
    if (active) {
        ci = uniform_int(p.tile_cam[t]);
        beg = uniform_int(p.tile_begin[t]);
        end = uniform_int(p.tile_end[t]);
        alpha = uniform_int(p.cam_part[ci]);
    }
    const int cc = chosen(restart, alpha);
    const CamT<R> ck = load_cam<R>(p.ccand[(k + 1) & 1][cc] + (size_t)ci * kCamRec);
    if (lane < kCamRec) cprev[lane] = p.cams[(k + 2) % 3][(size_t)ci * kCamRec + lane];
    if (ACC && lane < kCamRec) cbarl[lane] = p.cbar[(k + 1) & 1][cc][(size_t)ci * kCamRec + lane];
    const R gam = ACC ? (R)p.st[k & 1].gamma : (R)0;
    const R delta = (R)p.delta;
    // both candidate buffers of a parity are one allocation: candidate 1
    // follows candidate 0 after N records
    const char* __restrict__ pbase = reinterpret_cast<const char*>(pair_base<R>(p, k, 0));
    const uint64_t cand_stride = (uint64_t)p.N * kRecB;
    R* __restrict__ rec = rec_base<R>(p);
    bool bad = false;
    int run_key = -1;
    double run0 = 0.0, run1 = 0.0;
    __syncthreads();

    const int last = end - 1;  // tiles are never empty
    const int ns = active ? (end - beg + kWave - 1) / kWave : 0;
    // landmark index (with its partition in the top bits) of each lane's
    // observation, one step ahead of the fetch; lane kLPR r + c fetches
    // chunk c of record kRPI i + r in instruction i
    int li_ahead = 0;
    auto load_li = [&](int st) { li_ahead = p.obs_lm[min(beg + kWave * st + lane, last)]; };
    // Lane-derived offsets are recomputed inside each step from a lane index
    // the optimizer cannot see through: hoisted out of the loop they would
    // hold VGPRs for its whole length.
    auto opaque_lane = [&]() {
        int l = lane;
        asm volatile("" : "+v"(l));
        return l;
    };
    auto fetch = [&](int st, ObsBuf<R>& D) {
        const int ln = opaque_lane(), rr = ln / kLPR, qc = ln % kLPR;
#pragma unroll
        for (int i = 0; i < kNI; ++i) {
            const unsigned lp = (unsigned)__shfl(li_ahead, kRPI * i + rr);
            const unsigned li = lp & kLmMask;
            const uint64_t off = (uint64_t)chosen(restart, (int)(lp >> kLmBits)) * cand_stride +
                                 (uint64_t)li * kRecB + 16u * qc;
            dma16(pbase + off, &D.pair[kRPI * i * 8]);
        }
        const unsigned o = (unsigned)min(beg + kWave * st + ln, last);
        if constexpr (sizeof(R) == 8) {
            dma16(reinterpret_cast<const char*>(p.uv) + 16u * o, &D.uv[0]);
        } else {
            dma4(reinterpret_cast<const char*>(p.uv32) + 8u * o, &D.ux[0]);
            dma4(reinterpret_cast<const char*>(p.uv32) + 8u * o + 4u, &D.uy[0]);
        }
        dma4(reinterpret_cast<const char*>(p.obs_slot) + 4u * o, &D.slot[0]);
    };
    // records of step st (staged) to their slots (in D, the buffer of step st)
    auto store_recs = [&](int st, const ObsBuf<R>& D) {
        const int ln = opaque_lane(), rr = ln / kLPR, qc = ln % kLPR;
        const int b0 = beg + kWave * st;
#pragma unroll
        for (int i = 0; i < kNI; ++i) {
            const int r = kRPI * i + rr;
            if (b0 + r < end) {
                const float4 v = *reinterpret_cast<const float4*>(&stg[r * 8 + kEPC * qc]);
                *reinterpret_cast<float4*>(rec + (size_t)D.slot[r] * 8 + kEPC * qc) = v;
            }
        }
    };
    // step st reads buffer C; the next step's data goes to N
    auto step = [&](int st, const ObsBuf<R>& C, ObsBuf<R>& N) {
        wait_vmem();
        if (st > 0) store_recs(st - 1, N);
        __builtin_amdgcn_sched_barrier(0);
        if (st + 1 < ns) {
            fetch(st + 1, N);
            if (st + 2 < ns) load_li(st + 2);
        }
        __builtin_amdgcn_sched_barrier(0);
        const int ln = opaque_lane();
        const int o = beg + kWave * st + ln;
        const bool on = o < end;
        double hF = 0.0, gp = 0.0;
        int key = -1;
        if (on) {
            R ux, uy, lk0, lk1, lk2, lp0, lp1, lp2;
            int beta;
            const R* pr = &C.pair[ln * 8];
            if constexpr (sizeof(R) == 8) {
                const double2 u2 = C.uv[ln];
                ux = u2.x;
                uy = u2.y;
                const double2 q0 = *reinterpret_cast<const double2*>(pr);
                const double2 q1 = *reinterpret_cast<const double2*>(pr + 2);
                const double2 q2 = *reinterpret_cast<const double2*>(pr + 4);
                lk0 = q0.x; lk1 = q0.y; lk2 = q1.x;
                beta = (int)__double_as_longlong(q1.y);
                lp0 = q2.x; lp1 = q2.y; lp2 = pr[6];
            } else {
                ux = C.ux[ln];
                uy = C.uy[ln];
                const float4 f0 = *reinterpret_cast<const float4*>(pr);
                const float4 f1 = *reinterpret_cast<const float4*>(pr + 4);
                lk0 = f0.x; lk1 = f0.y; lk2 = f0.z;
                beta = __float_as_int(f0.w);
                lp0 = f1.x; lp1 = f1.y; lp2 = f1.z;
            }
            const R r2u = ux * ux + uy * uy, r4u = r2u * r2u;
            const R r6u = r4u * r2u, r8u = r4u * r4u;
            R* sg = &stg[ln * 8];
            ObsEval<LOSS, R> ek;
            eval_obs<LOSS, R>(ck, lk0, lk1, lk2, ux, uy, r2u, r4u, delta, ek);
            bad |= !(ek.r2 > (R)1e-24);
            add_moments<R>(acc, ek.w, ek.lam, ux, uy, r2u, r4u, r6u, r8u, ek.e);
            // landmark-side record: W = w lambda^2 and V = w lambda e_w per surrogate
            const R wl = ek.w * ek.lam;
            sg[0] = wl * ek.lam;
            sg[1] = wl * ek.e[0];
            sg[2] = wl * ek.e[1];
            sg[3] = wl * ek.e[2];
            // F share: each side of the pair gets half of F_ij = rho / 2
            hF = (double)((R)0.25 * ek.rho);
            key = beta;
            if (beta != alpha) {
                // surrogate gap of the previous linearization y = x^(k-1) at x^k:
                // P - Q = w (|Dc|^2 - |Dl|^2 + e^y . (Dc + Dl)) with
                // Dc = R^k p^k - R^y p^y + lambda^y (t^k - t^y), Dl = lambda^y (l^k - l^y)
                const R lp[3] = {lp0, lp1, lp2};
                const R lk[3] = {lk0, lk1, lk2};
                // x^(k-1) from LDS, through an address the optimizer cannot
                // hoist: kept in SGPRs with the other two cameras it would
                // spill them
                int co = 0;
                asm volatile("" : "+v"(co));
                const CamT<R> cp = load_cam<R>(cprev + co);
                ObsEval<LOSS, R> ep;
                eval_obs<LOSS, R>(cp, lp0, lp1, lp2, ux, uy, r2u, r4u, delta, ep);
                // R^k p^k again (cheaper than keeping it live), and the camera
                // terms as separate products so that no difference of two
                // loop-invariant values is kept in registers
                const R pz = ck.d[0] + ck.d[1] * r2u + ck.d[2] * r4u;
                R q = (R)0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R rpk = ck.r[3 * a] * ux + ck.r[3 * a + 1] * uy + ck.r[3 * a + 2] * pz;
                    const R dc = rpk - ep.Rp[a] + ep.lam * ck.t[a] - ep.lam * cp.t[a];
                    const R dl = ep.lam * (lk[a] - lp[a]);
                    q += dc * dc - dl * dl + ep.e[a] * (dc + dl);
                }
                gp = (double)((R)0.5 * ep.w * q);
            }
            if constexpr (ACC) {
                const R lb0 = lk0 + gam * (lk0 - lp0);
                const R lb1 = lk1 + gam * (lk1 - lp1);
                const R lb2 = lk2 + gam * (lk2 - lp2);
                int co = 0;
                asm volatile("" : "+v"(co));
                const CamT<R> cb = load_cam<R>(cbarl + co);
                ObsEval<LOSS, R> eb;
                eval_obs<LOSS, R>(cb, lb0, lb1, lb2, ux, uy, r2u, r4u, delta, eb);
                bad |= !(eb.r2 > (R)1e-24);
                add_moments<R>(acc + kMom, eb.w, eb.lam, ux, uy, r2u, r4u, r6u, r8u, eb.e);
                const R wb = eb.w * eb.lam;
                sg[4] = wb * eb.lam;
                sg[5] = wb * eb.e[0];
                sg[6] = wb * eb.e[1];
                sg[7] = wb * eb.e[2];
            } else {
                sg[4] = sg[5] = sg[6] = sg[7] = (R)0;
            }
        }
        {
            // landmark-side shares by landmark partition.  Within a camera the
            // observations are sorted by landmark partition, so most steps
            // hold one partition: accumulate those per lane and reduce once
            // per run; a step that straddles partitions uses a segmented sum.
            const int k0 = uniform_int(key);
            const bool uni = __all(!on || key == k0);
            if (uni) {
                if (k0 != run_key) {
                    flush_run(run_key, run0, run1, lane, bins[0], bins[1]);
                    run_key = k0;
                }
                run0 += hF;
                run1 -= gp;
            } else {
                flush_run(run_key, run0, run1, lane, bins[0], bins[1]);
                run_key = -1;
                bin_add_sorted(hF, -gp, key, lane, bins[0], bins[1]);
            }
        }
    };

    if (ns > 0) {
        load_li(0);
        fetch(0, A);
        if (ns > 1) load_li(1);
    }
    for (int st = 0; st < ns; st += 2) {
        step(st, A, B);
        if (st + 1 < ns) step(st + 1, B, A);
    }
    wait_vmem();
    if (ns > 0) store_recs(ns - 1, (ns - 1) & 1 ? B : A);
    flush_run(run_key, run0, run1, lane, bins[0], bins[1]);
    if (bad) p.st[0].err = -5;

    // tile totals: LDS transpose in the two buffers (rows 0..6 in A, 7..13
    // in B), lane v sums value v over the 64 lanes
    wait_vmem();
    constexpr int kCh = 2 * kRedHalf;
    double* redA = A.red();
    double* redB = B.red();
#pragma unroll
    for (int c0 = 0; c0 < kAccR; c0 += kCh) {
#pragma unroll
        for (int v = 0; v < kCh; ++v) {
            if (c0 + v < kAccR) {
                double* row = v < kRedHalf ? &redA[v * (kWave + 1)] : &redB[(v - kRedHalf) * (kWave + 1)];
                row[lane] = acc[c0 + v];
            }
        }
        __syncthreads();
        if (active && lane < kCh && c0 + lane < kAccR) {
            const double* row = lane < kRedHalf ? &redA[lane * (kWave + 1)]
                                                : &redB[(lane - kRedHalf) * (kWave + 1)];
            double sum = 0.0;
            for (int q = 0; q < kWave; ++q) sum += row[q];
            p.tile_vals[(size_t)t * kTileVals + c0 + lane] = sum;
        }
        __syncthreads();
    }
    if (active) {
        for (int b = lane; b < S; b += kWave) {
            p.tile_bins[(size_t)b * p.T + t] = bins[0][b];
            p.tile_bins[(size_t)(S + b) * p.T + t] = bins[1][b];
        }
        if (lane == 0) {
            double f = 0.0, g = 0.0;
            for (int b = 0; b < S; ++b) {
                f += bins[0][b];
                g += bins[1][b];
            }
            p.tile_vals[(size_t)t * kTileVals + 2 * kMom] = f;
            p.tile_vals[(size_t)t * kTileVals + 2 * kMom + 1] = -g;
        }
    }
}

// ---------------------------------------------------- camera subproblem

struct CamD {
    double R[9], t[3], d[3];
};

__device__ __forceinline__ CamD load_camd(const double* __restrict__ c) {
    CamD o;
#pragma unroll
    for (int a = 0; a < 9; ++a) o.R[a] = c[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.t[a] = c[9 + a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.d[a] = c[12 + a];
    return o;
}
__device__ __forceinline__ void store_camd(double* __restrict__ c, const CamD& o) {
#pragma unroll
    for (int a = 0; a < 9; ++a) c[a] = o.R[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[9 + a] = o.t[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[12 + a] = o.d[a];
    c[15] = 0.0;
}

// 6x6 symmetric Z from its 20 distinct moments (z = ux, uy, 1, r2, r4, lambda)
__device__ __forceinline__ void unpack_Z(const double* a, double Z[6][6]) {
    Z[0][0] = a[0]; Z[0][1] = a[1]; Z[1][1] = a[2];
    Z[0][2] = a[3]; Z[0][3] = a[4]; Z[0][4] = a[5];
    Z[1][2] = a[6]; Z[1][3] = a[7]; Z[1][4] = a[8];
    Z[2][2] = a[9]; Z[2][3] = a[10]; Z[2][4] = a[11];
    Z[3][3] = a[11]; Z[3][4] = a[12]; Z[4][4] = a[13];
    Z[0][5] = a[14]; Z[1][5] = a[15];
    Z[2][5] = a[16]; Z[3][5] = a[17]; Z[4][5] = a[18];
    Z[5][5] = a[19];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) Z[i][j] = Z[j][i];
}

// Mx: the 3x6 map z -> R p(d) - Ry p(dy) + lambda (t - ty)
__device__ __forceinline__ void build_Mx(const CamD& y, const CamD& c, double Mx[3][6]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Mx[r][0] = c.R[3 * r] - y.R[3 * r];
        Mx[r][1] = c.R[3 * r + 1] - y.R[3 * r + 1];
        double dR2 = c.R[3 * r + 2] - y.R[3 * r + 2];
#pragma unroll
        for (int k = 0; k < 3; ++k) Mx[r][2 + k] = c.d[k] * dR2 + (c.d[k] - y.d[k]) * y.R[3 * r + 2];
        Mx[r][5] = c.t[r] - y.t[r];
    }
}

__device__ __forceinline__ double prox2(const CamD& y, const CamD& c) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) s += (c.R[a] - y.R[a]) * (c.R[a] - y.R[a]);
#pragma unroll
    for (int a = 0; a < 3; ++a) s += (c.t[a] - y.t[a]) * (c.t[a] - y.t[a]) + (c.d[a] - y.d[a]) * (c.d[a] - y.d[a]);
    return s;
}

// Phi(c) - Phi(y) of one camera's surrogate (moments about y)
__device__ double phi_delta(const double* mom, const CamD& y, const CamD& c, double xi) {
    double Z[6][6], Mx[3][6];
    unpack_Z(mom, Z);
    build_Mx(y, c, Mx);
    double q = 0.0, lin = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double za = 0.0;
#pragma unroll
            for (int b = 0; b < 6; ++b) za += Z[a][b] * Mx[r][b];
            q += Mx[r][a] * za;
            lin += Mx[r][a] * mom[20 + 6 * r + a];
        }
    return q + 2.0 * lin + 0.5 * xi * prox2(y, c);
}

// Gauss-Newton model at c: H = 2 sum w J^T J + xi I (lower triangle, packed)
// and gradient of the exact surrogate, in tangent coordinates (dtheta, dt, dd)
// with R <- R Exp(dtheta).
__device__ void grad_hess(const double* mom, const CamD& y, const CamD& c, double xi, double* Hp, double* g) {
    double Z[6][6], Mx[3][6];
    unpack_Z(mom, Z);
    build_Mx(y, c, Mx);
    const double* d = c.d;
    double G00 = Z[0][0], G01 = Z[0][1], G11 = Z[1][1];
    double G02 = d[0] * Z[0][2] + d[1] * Z[0][3] + d[2] * Z[0][4];
    double G12 = d[0] * Z[1][2] + d[1] * Z[1][3] + d[2] * Z[1][4];
    double G22 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) G22 += d[a] * d[b] * Z[2 + a][2 + b];
    double G[3][3] = {{G00, G01, G02}, {G01, G11, G12}, {G02, G12, G22}};
    double tr = G00 + G11 + G22;
    double pl[3] = {Z[0][5], Z[1][5], d[0] * Z[2][5] + d[1] * Z[3][5] + d[2] * Z[4][5]};
    double px[3][3] = {{0, -pl[2], pl[1]}, {pl[2], 0, -pl[0]}, {-pl[1], pl[0], 0}};
    double H[9][9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            H[a][b] = 2.0 * ((a == b ? tr : 0.0) - G[a][b]);
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) s += px[a][q] * c.R[3 * b + q];
            H[a][3 + b] = 2.0 * s;
            H[3 + a][3 + b] = (a == b) ? 2.0 * Z[5][5] : 0.0;
            H[3 + a][6 + b] = 2.0 * c.R[3 * a + 2] * Z[2 + b][5];
            H[6 + a][6 + b] = 2.0 * Z[2 + a][2 + b];
        }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        H[0][6 + b] = 2.0 * Z[1][2 + b];
        H[1][6 + b] = -2.0 * Z[0][2 + b];
        H[2][6 + b] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) H[a][a] += xi;
    int idx = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            // lower triangle from the blocks filled above (upper-right stored)
            Hp[idx++] = (i / 3 == j / 3) ? H[i][j] : H[j][i];
        }
    // residual moments at c: Yc = Y + Mx Z
    double Yc[3][6];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            double s = mom[20 + 6 * r + a];
#pragma unroll
            for (int b = 0; b < 6; ++b) s += Mx[r][b] * Z[b][a];
            Yc[r][a] = s;
        }
    double Yp[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Yp[r][0] = Yc[r][0];
        Yp[r][1] = Yc[r][1];
        Yp[r][2] = d[0] * Yc[r][2] + d[1] * Yc[r][3] + d[2] * Yc[r][4];
    }
    double W[3][3], Q[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double s = 0.0, s2 = 0.0;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                s += c.R[3 * r + a] * Yp[r][b];
                s2 += c.R[3 * r + a] * y.R[3 * r + b];
            }
            W[a][b] = s;
            Q[a][b] = s2;
        }
    g[0] = 2.0 * (W[2][1] - W[1][2]) - xi * (Q[2][1] - Q[1][2]);
    g[1] = 2.0 * (W[0][2] - W[2][0]) - xi * (Q[0][2] - Q[2][0]);
    g[2] = 2.0 * (W[1][0] - W[0][1]) - xi * (Q[1][0] - Q[0][1]);
#pragma unroll
    for (int a = 0; a < 3; ++a) g[3 + a] = 2.0 * Yc[a][5] + xi * (c.t[a] - y.t[a]);
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2)
        g[6 + k2] = 2.0 * (c.R[2] * Yc[0][2 + k2] + c.R[5] * Yc[1][2 + k2] + c.R[8] * Yc[2][2 + k2]) +
                    xi * (c.d[k2] - y.d[k2]);
}

// (A) x = b for SPD A given as packed lower triangle; false if not SPD.
// One division per pivot (its reciprocal); every other quotient is a
// product, which keeps FP64 divisions off the solve's serial chain.
__device__ bool chol9(double* L, const double* b, double* x) {
    double inv[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = L[i * (i + 1) / 2 + j];
#pragma unroll
            for (int q = 0; q < j; ++q) s -= L[i * (i + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
            if (i == j) {
                if (!(s > 0.0)) return false;
                const double dj = sqrt(s);
                L[i * (i + 1) / 2 + i] = dj;
                inv[i] = 1.0 / dj;
            } else {
                L[i * (i + 1) / 2 + j] = s * inv[j];
            }
        }
    }
    double z[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        double s = b[i];
#pragma unroll
        for (int q = 0; q < i; ++q) s -= L[i * (i + 1) / 2 + q] * z[q];
        z[i] = s * inv[i];
    }
#pragma unroll
    for (int i = 8; i >= 0; --i) {
        double s = z[i];
#pragma unroll
        for (int q = i + 1; q < 9; ++q) s -= L[q * (q + 1) / 2 + i] * x[q];
        x[i] = s * inv[i];
    }
    return true;
}

// Levenberg-Marquardt on one camera's surrogate: start at y, mu = 1e-4,
// accept iff the surrogate strictly decreases (mu /= 10), else mu *= 10,
// give up after 10 rejects in a row; inner_steps accepted steps (<= 0:
// until the step is negligible or 100 accepted steps).  *phi_out receives
// Phi(result) - Phi(y), exactly as phi_delta computes it (0 if no step was
// accepted).
__device__ CamD lm_camera(const double* mom, const CamD& y, double xi, int inner_steps, double* phi_out) {
    CamD c = y;
    double phi = 0.0;
    double mu = 1e-4;
    int succ = 0, rej = 0;
    for (;;) {
        if (inner_steps > 0 && succ >= inner_steps) break;
        if (inner_steps <= 0 && succ >= 100) break;
        // the model is rebuilt on every pass, so the damped matrix is formed
        // in place from it
        double A[45], g[9], rhs[9], dl[9];
        grad_hess(mom, y, c, xi, A, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            A[i * (i + 1) / 2 + i] += mu * A[i * (i + 1) / 2 + i];
            rhs[i] = -g[i];
        }
        bool ok = chol9(A, rhs, dl);
        CamD cand = c;
        double phic = 0.0;
        if (ok) {
            double E[9];
            exp_so3(dl, E);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    cand.R[3 * r + q] = c.R[3 * r] * E[q] + c.R[3 * r + 1] * E[3 + q] + c.R[3 * r + 2] * E[6 + q];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cand.t[a] = c.t[a] + dl[3 + a];
                cand.d[a] = c.d[a] + dl[6 + a];
            }
            phic = phi_delta(mom, y, cand, xi);
        }
        if (ok && phic < phi) {
            double nd = 0.0, nx = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) nd += dl[a] * dl[a];
#pragma unroll
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
    *phi_out = phi;
    return c;
}

// ------------------------------------------------------------ entity pass

// x-bar for the next iteration from a camera's next and current values (eq.
// nesterov_x with the rotation projected by eq. proj_rot3d)
__device__ void extrapolate_cam(const double* cn, const double* co, double gam, double* out) {
    double Mx[9], Rb[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) Mx[a] = cn[a] + gam * (cn[a] - co[a]);
    if (!polar_rotation(Mx, Rb)) nearest_rotation(Mx, Rb);
#pragma unroll
    for (int a = 0; a < 9; ++a) out[a] = Rb[a];
#pragma unroll
    for (int a = 9; a < 15; ++a) out[a] = cn[a] + gam * (cn[a] - co[a]);
    out[15] = 0.0;
}


// Partition of block b from by-value block ranges (starts[a] = first block
// of partition a, non-decreasing, starts[0] = 0): no memory load.
__device__ __forceinline__ int block_partition(const int* starts, int S, int b) {
    int a = 0;
    for (int q = 1; q < S; ++q) a += (starts[q] <= b);
    return a;
}

// LDS of a camera block: the accelerated candidates handed to the lanes of
// the plain surrogate.
struct CamLds {
    double c[kCamBlock][16];
};

// Sum of one surrogate's moments over a camera's tiles (two tiles' loads in
// flight at a time; the sums keep the tile order).  f receives the camera's
// F and gap shares.
__device__ __forceinline__ void camera_moments(const Params& p, int t0, int t1, int off, double* mom, double* f) {
    int t = t0;
    for (; t + 1 < t1; t += 2) {
        const double* u = p.tile_vals + (size_t)t * kTileVals;
        const double* v = u + kTileVals;
        double x[kMom + 2], y[kMom + 2];
#pragma unroll
        for (int a = 0; a < kMom; ++a) {
            x[a] = u[off + a];
            y[a] = v[off + a];
        }
        x[kMom] = u[2 * kMom];
        x[kMom + 1] = u[2 * kMom + 1];
        y[kMom] = v[2 * kMom];
        y[kMom + 1] = v[2 * kMom + 1];
#pragma unroll
        for (int a = 0; a < kMom; ++a) mom[a] = (mom[a] + x[a]) + y[a];
        f[0] = (f[0] + x[kMom]) + y[kMom];
        f[1] = (f[1] + x[kMom + 1]) + y[kMom + 1];
    }
    if (t < t1) {
        const double* u = p.tile_vals + (size_t)t * kTileVals;
#pragma unroll
        for (int a = 0; a < kMom; ++a) mom[a] += u[off + a];
        f[0] += u[2 * kMom];
        f[1] += u[2 * kMom + 1];
    }
}

// Camera subproblems of one block of <= 128 cameras in one partition:
// threads [0,128) solve the plain surrogate, [128,256) the accelerated one.
// The block's partition (and so the restart flag that picks x^k among the
// candidates of iteration k - 1) comes from the kernel arguments, so the
// moments and x^k are each one load away.  The plain surrogate's lane also
// evaluates the plain surrogate at the accelerated candidate, which the
// accelerated lane hands over through LDS.
template <bool ACC>
__device__ __forceinline__ void camera_role(const Params& p, int k, int b, CamLds& sh, double (*red)[4]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const double xi = p.xi;
    const int surr = threadIdx.x / kCamBlock;
    const int cl = threadIdx.x % kCamBlock;
    const int a = block_partition(p.pcb, p.S, b);
    const int ci = p.pcam[a] + (b - p.pcb[a]) * kCamBlock + cl;
    const bool cam = ci < p.pcam[a + 1];
    const int cc = p.restart[a] ? 0 : 1;  // x^k: the candidate chosen by the last restart test
    double dv = 0.0, dacc = 0.0, f[2] = {0.0, 0.0};
    double mom[kMom];
    CamD ck;
    if (cam && (surr == 0 || ACC)) {
        const size_t o = (size_t)ci * kCamRec;
#pragma unroll
        for (int q = 0; q < kMom; ++q) mom[q] = 0.0;
        camera_moments(p, p.cam_tile_off[ci], p.cam_tile_off[ci + 1], surr == 0 ? 0 : kMom, mom, f);
        ck = load_camd(p.ccand[(k + 1) & 1][cc] + o);
        if (surr == 0) store_camd(p.cams[k % 3] + o, ck);
        const CamD y = surr == 0 ? ck : load_camd(p.cbar[(k + 1) & 1][cc] + o);
        double phi;
        const CamD c = lm_camera(mom, y, xi, p.inner_steps, &phi);
        store_camd(p.ccand[k & 1][surr] + o, c);
        if constexpr (ACC) {
            // the extrapolation the next iteration uses if this candidate is
            // chosen; gamma^(k+1) depends only on s^(k), so it is known now
            double s1;
            const double gnext = next_gamma(p, p.st[k & 1].s, &s1);
            double cn[16], cko[16], cbar[16];
            store_camd(cn, c);
            store_camd(cko, ck);
            extrapolate_cam(cn, cko, gnext, cbar);
            double* dst = p.cbar[k & 1][surr] + o;
#pragma unroll
            for (int q = 0; q < 16; ++q) dst[q] = cbar[q];
            if (surr == 1) store_camd(sh.c[cl], c);
        }
        // about y = x^k, the accepted change is the plain surrogate's change
        if (surr == 0) dv = phi;
        else f[0] = f[1] = 0.0;
    }
    if constexpr (ACC) {
        __syncthreads();  // the accelerated candidates are in LDS
        if (cam && surr == 0) dacc = phi_delta(mom, ck, load_camd(sh.c[cl]), xi);
    }
    // block sums in a fixed order: (dmm, dacc, F share, gap share)
    double v0 = wave_sum(dv), v1 = wave_sum(dacc);
    f[0] = wave_sum(f[0]);
    f[1] = wave_sum(f[1]);
    if (lane == 0) {
        red[wv][0] = v0;
        red[wv][1] = v1;
        red[wv][2] = f[0];
        red[wv][3] = f[1];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += red[w][threadIdx.x];
        p.camblk_vals[(size_t)b * 4 + threadIdx.x] = s;
    }
}

// Sums a landmark's records (slots base + q n + lane, q < D), eight in flight
// per lane; FP32 records are accumulated in FP64.
template <typename RT, bool ACC>
__device__ __forceinline__ void sum_records(const RT* __restrict__ rec, int64_t base, int n, int lane, int D,
                                            double& W0, double* V0, double& W1, double* V1) {
    using V4 = typename std::conditional<std::is_same<RT, double>::value, double4, float4>::type;
    constexpr int U = 8;  // the camera role already sets this kernel's VGPR budget
    for (int q0 = 0; q0 < D; q0 += U) {
        V4 ra[U], rb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (q0 + u < D) {
                const V4* r = reinterpret_cast<const V4*>(rec + (size_t)(base + (int64_t)(q0 + u) * n + lane) * 8);
                ra[u] = r[0];
                if (ACC) rb[u] = r[1];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (q0 + u < D) {
                W0 += ra[u].x;
                V0[0] += ra[u].y;
                V0[1] += ra[u].z;
                V0[2] += ra[u].w;
                if (ACC) {
                    W1 += rb[u].x;
                    V1[0] += rb[u].y;
                    V1[1] += rb[u].z;
                    V1[2] += rb[u].w;
                }
            }
        }
    }
}

// Candidate pair record (l^(k+1) candidate, partition id, l^k) of iteration k.
__device__ __forceinline__ void write_cand_pair(const Params& p, int k, int cand, int li, const double* ln,
                                                double beta_bits, const double* lk) {
    double2* q = reinterpret_cast<double2*>(p.lcp[k & 1][cand] + (size_t)li * kLmPair);
    q[0] = make_double2(ln[0], ln[1]);
    q[1] = make_double2(ln[2], beta_bits);
    q[2] = make_double2(lk[0], lk[1]);
    q[3] = make_double2(lk[2], 0.0);
    if (p.fp32) {
        float4* f = reinterpret_cast<float4*>(p.lcp32[k & 1][cand] + (size_t)li * kLmPair);
        f[0] = make_float4((float)ln[0], (float)ln[1], (float)ln[2], __int_as_float((int)__double_as_longlong(beta_bits)));
        f[1] = make_float4((float)lk[0], (float)lk[1], (float)lk[2], 0.0f);
    }
}

// Landmark subproblems of one block: one wave per group of equal track
// length, one lane per landmark (the records it reads are consecutive
// across the wave's lanes).
template <typename RT, bool ACC>
__device__ __forceinline__ void landmark_role(const Params& p, int k, int lb, double (*sred)[4]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const double xi = p.xi;
    const int g = p.lmblock_g0[lb] + wv;
    // l^k and l^(k-1): the candidate of iteration k - 1 chosen for this
    // block's partition
    const int lcc = p.restart[p.lmblock_part[lb]] ? 0 : 1;
    double dmm = 0.0, dacc = 0.0;
    if (g < p.lmblock_g1[lb]) {
        const int n = p.group_n[g], D = p.group_deg[g];
        const int li = p.group_lm0[g] + lane;
        const int64_t base = p.group_base[g];
        if (lane < n) {
            double W0 = 0, V0[3] = {0, 0, 0}, W1 = 0, V1[3] = {0, 0, 0};
            sum_records<RT, ACC>(rec_base<RT>(p), base, n, lane, D, W0, V0, W1, V1);
            const LmRead<double> L = read_pair(p.lcp[(k + 1) & 1][lcc], li);
            double dl[3], nm = 0.0, dv = 0.0;
            const double den0 = 2.0 * W0 + xi;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dl[a] = V0[a] / den0;
                nm += dl[a] * dl[a];
                dv += dl[a] * V0[a];
            }
            dmm = (W0 + 0.5 * xi) * nm - dv;
            const double beta_bits = __longlong_as_double((long long)L.beta);
            const double lm[3] = {L.lk[0] + dl[0], L.lk[1] + dl[1], L.lk[2] + dl[2]};
            write_cand_pair(p, k, 0, li, lm, beta_bits, L.lk);
            if (ACC) {
                const double gam = p.st[k & 1].gamma;
                const double den1 = 2.0 * W1 + xi;
                double la[3], na = 0.0, va = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    double lbar = L.lk[a] + gam * (L.lk[a] - L.lp[a]);
                    la[a] = lbar + V1[a] / den1;
                    const double da = la[a] - L.lk[a];
                    na += da * da;
                    va += da * V0[a];
                }
                dacc = (W0 + 0.5 * xi) * na - va;
                write_cand_pair(p, k, 1, li, la, beta_bits, L.lk);
            }
        }
    }
    dmm = wave_sum(dmm);
    dacc = wave_sum(dacc);
    if (lane == 0) {
        sred[wv][0] = dmm;
        sred[wv][1] = dacc;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += sred[w][threadIdx.x];
        p.lmblk_vals[(size_t)lb * 2 + threadIdx.x] = s;
    }
}

// One launch, three kinds of blocks: camera subproblems, column sums of the
// per-tile partition bins, and landmark subproblems (in that order, so that
// the short column sums are not queued behind the landmark blocks).  The
// roles are independent, so the camera solves (long serial chains on few
// threads) overlap the landmark pass.
template <typename RT, bool ACC>
__global__ __launch_bounds__(256) void k_entity(Params p, int k) {
    __shared__ CamLds sh;
    __shared__ double sred[4][4];  // block reductions
    __shared__ double fshl[kMaxPart];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    if ((int)blockIdx.x < p.nCamBlocks) {
        camera_role<ACC>(p, k, blockIdx.x, sh, sred);
        return;
    }
    const int cb = blockIdx.x - p.nCamBlocks;
    if (cb < 2 * p.S) {
        // column sums of the per-tile partition bins
        const double* src = p.tile_bins + (size_t)cb * p.T;
        double s = 0.0;
        for (int t = threadIdx.x; t < p.T; t += 256) s += src[t];
        s = wave_sum(s);
        if (lane == 0) sred[wv][0] = s;
        __syncthreads();
        if (threadIdx.x == 0) p.colsum[cb] = sred[0][0] + sred[1][0] + sred[2][0] + sred[3][0];
        // F(x^(k-1)) from the shares this iteration's restart test stored
        if (cb == 0) store_trace(p, k, fshl);
        return;
    }
    const int lb = cb - 2 * p.S;
    if (lb == 0 && threadIdx.x == 0) p.st[0].decided = 0;
    landmark_role<RT, ACC>(p, k, lb, sred);
}

// ------------------------------------------------------- select and roll

// End of a call, after the restart test of iteration k - 1 (launched just
// before): the chosen candidates written into both candidate slots and the
// camera generation k % 3, so that x^k is stored plainly whichever slot is
// read; block 0 also stores F(x^(k-1)) in the trace.
__global__ __launch_bounds__(256) void k_finalize(Params p, int k) {
    __shared__ double sh[kMaxPart];
    if (blockIdx.x == 0) {
        store_trace(p, k, sh);
        if (threadIdx.x == 0) p.st[0].decided = 1;
    }
    const uint64_t restart = restart_mask(p);
    const int par = (k + 1) & 1;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < p.M) {
        const int ci = (int)i;
        const int c = chosen(restart, p.cam_part[ci]);
        const size_t o = (size_t)ci * kCamRec;
        // per-lane choice between two uniform pointers (indexing the
        // argument's pointer table per lane would copy it to scratch)
        const double* xc = c ? p.ccand[par][1] : p.ccand[par][0];
        const double* xbc = c ? p.cbar[par][1] : p.cbar[par][0];
        double2 x[8], xb[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            x[a] = reinterpret_cast<const double2*>(xc + o)[a];
            xb[a] = reinterpret_cast<const double2*>(xbc + o)[a];
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            reinterpret_cast<double2*>(p.ccand[par][0] + o)[a] = x[a];
            reinterpret_cast<double2*>(p.ccand[par][1] + o)[a] = x[a];
            reinterpret_cast<double2*>(p.cbar[par][0] + o)[a] = xb[a];
            reinterpret_cast<double2*>(p.cbar[par][1] + o)[a] = xb[a];
            reinterpret_cast<double2*>(p.cams[k % 3] + o)[a] = x[a];
        }
        return;
    }
    const int64_t j = i - p.M;
    if (j < p.N) {
        const int li = (int)j;
        const int c = chosen(restart, p.lm_part[li]);
        const size_t o = (size_t)li * kLmPair;
        const double* qc = c ? p.lcp[par][1] : p.lcp[par][0];
        double2 q[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) q[a] = reinterpret_cast<const double2*>(qc + o)[a];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            reinterpret_cast<double2*>(p.lcp[par][0] + o)[a] = q[a];
            reinterpret_cast<double2*>(p.lcp[par][1] + o)[a] = q[a];
        }
        if (p.fp32) {
            float4 f[2];
            const float* fc = c ? p.lcp32[par][1] : p.lcp32[par][0];
#pragma unroll
            for (int a = 0; a < 2; ++a) f[a] = reinterpret_cast<const float4*>(fc + o)[a];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                reinterpret_cast<float4*>(p.lcp32[par][0] + o)[a] = f[a];
                reinterpret_cast<float4*>(p.lcp32[par][1] + o)[a] = f[a];
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_extrapolate_cams(Params p, int k) {
    const int ci = blockIdx.x * 256 + threadIdx.x;
    if (ci >= p.M) return;
    double cb[16];
    extrapolate_cam(p.cams[k % 3] + (size_t)ci * kCamRec, p.cams[(k + 2) % 3] + (size_t)ci * kCamRec,
                    p.st[k & 1].gamma, cb);
    const int par = (k + 1) & 1;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
        p.cbar[par][0][(size_t)ci * kCamRec + a] = cb[a];
        p.cbar[par][1][(size_t)ci * kCamRec + a] = cb[a];
    }
}

// ------------------------------------------------------- objective shares

// Per tile: sum of F_ij / 2 over the tile (camera side) and the landmark-side
// halves binned by landmark partition (or plain totals when bins is null).
template <typename R, int LOSS>
__global__ __launch_bounds__(kObsWaves* kWave) void k_objective(Params p, const double* __restrict__ cams,
                                                                const double* __restrict__ lpair,
                                                                const double2* __restrict__ uv,
                                                                double* __restrict__ tile_F, double* __restrict__ bins_out) {
    __shared__ double bins[kObsWaves][2][kMaxPart];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int t = uniform_int(blockIdx.x * kObsWaves + wv);
    const bool active = t < p.T;
    const int S = p.S;
    for (int b = lane; b < S; b += kWave) bins[wv][0][b] = bins[wv][1][b] = 0.0;
    __syncthreads();
    if (!active) return;
    const int ci = uniform_int(p.tile_cam[t]);
    const int beg = uniform_int(p.tile_begin[t]), end = uniform_int(p.tile_end[t]);
    const CamT<R> c = load_cam<R>(cams + (size_t)ci * kCamRec);
    const R delta = (R)p.delta;
    double acc = 0.0;
    bool bad = false;
    for (int base = beg; base < end; base += kWave) {
        const int o = base + lane;
        double hF = 0.0;
        int key = -1;
        if (o < end) {
            const double2 u2 = uv[o];
            const R ux = (R)u2.x, uy = (R)u2.y;
            const LmRead<double> L = read_pair(lpair, p.obs_lm[o] & kLmMask);
            const R r2u = ux * ux + uy * uy;
            ObsEvalCF<LOSS, R> e;
            eval_obs_cf<LOSS, R>(c, (R)L.lk[0], (R)L.lk[1], (R)L.lk[2], ux, uy, r2u, r2u * r2u, delta, e);
            bad |= !(e.r2 > (R)1e-24);
            hF = (double)((R)0.25 * e.rho);
            key = L.beta;
        }
        acc += hF;
        if (bins_out) bin_add_sorted(hF, 0.0, key, lane, bins[wv][0], bins[wv][1]);
    }
    if (bad) p.st[0].err = -5;
    acc = wave_sum(acc);
    if (lane == 0) tile_F[t] = acc;
    if (bins_out)
        for (int b = lane; b < S; b += kWave) bins_out[(size_t)b * p.T + t] = bins[wv][0][b];
}

// Fsh^a = sum over the tiles of a's cameras of the camera halves + column sum
// of a's landmark halves; F = sum_a Fsh^a.  One block, fixed order.
__global__ __launch_bounds__(256) void k_objective_reduce(Params p, const double* __restrict__ tile_F,
                                                          const double* __restrict__ bins,
                                                          double* __restrict__ part_out, double* __restrict__ F_out) {
    __shared__ double sp[kMaxPart];
    __shared__ double sw[4];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int S = p.S;
    if (!bins) {
        double s = 0.0;
        for (int t = threadIdx.x; t < p.T; t += 256) s += tile_F[t];
        s = wave_sum(s);
        if (lane == 0) sw[wv] = s;
        __syncthreads();
        if (threadIdx.x == 0) *F_out = 2.0 * (sw[0] + sw[1] + sw[2] + sw[3]);
        return;
    }
    for (int a = wv; a < S; a += 4) {
        // camera side: tiles of cameras in partition a are contiguous
        const int t0 = p.cam_tile_off[p.part_cam[a]], t1 = p.cam_tile_off[p.part_cam[a + 1]];
        double s = 0.0;
        for (int t = t0 + lane; t < t1; t += kWave) s += tile_F[t];
        double s2 = 0.0;
        for (int t = lane; t < p.T; t += kWave) s2 += bins[(size_t)a * p.T + t];
        s = wave_sum(s);
        s2 = wave_sum(s2);
        if (lane == 0) sp[a] = s + s2;
    }
    __syncthreads();
    if (threadIdx.x < S) part_out[threadIdx.x] = sp[threadIdx.x];
    if (threadIdx.x == 0) {
        double F = 0.0;
        for (int a = 0; a < S; ++a) F += sp[a];
        *F_out = F;
        if (!isfinite(F) && p.st[0].err == 0) p.st[0].err = -4;
    }
}

// ------------------------------------------------------------- import point

// Caller arrays (caller order and units) -> internal scratch records.
__global__ __launch_bounds__(256) void k_import(Params p, const double* __restrict__ cams,
                                                const double* __restrict__ lms, const double* __restrict__ uv) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double sc = p.scale;
    if (i < p.M) {
        const double* src = cams ? cams + (size_t)p.cam_ext[i] * 15 : nullptr;
        double* dst = p.tmp_cams + (size_t)i * kCamRec;
        if (src) {
            for (int a = 0; a < 12; ++a) dst[a] = src[a];
            dst[12] = src[12] / sc;
            dst[13] = src[13] * sc;
            dst[14] = src[14] * sc * sc * sc;
            dst[15] = 0.0;
        }
    }
    if (i < p.N) {
        double* dst = p.tmp_lpair + (size_t)i * kLmPair;
        const double beta = __longlong_as_double((long long)p.lm_part[i]);
        if (lms) {
            const double* src = lms + (size_t)p.lm_ext[i] * 3;
            dst[0] = src[0];
            dst[1] = src[1];
            dst[2] = src[2];
        }
        dst[3] = beta;
    }
    if (i < p.K && uv) {
        const int oi = p.obs_orig[i];
        p.tmp_uv[i] = make_double2(uv[2 * (size_t)oi] / sc, uv[2 * (size_t)oi + 1] / sc);
    }
}

// ------------------------------------------------------------------ adjoint

// App. D, eq. DFij: per observation grad_R = -w lambda m e^T (camera-frame e),
// grad_t = w lambda R e, grad_l = -w lambda R e, grad_d = w e_z (1, |u|^2, |u|^4),
// grad_u = w (e_xy + e_z (2 d2 + 4 d3 |u|^2) u); camera sums per tile, landmark
// parts to the observation's slot, pixel parts to the caller's index.
template <typename R, int LOSS>
__global__ __launch_bounds__(kObsWaves* kWave) void k_grad_obs(Params p, const double* __restrict__ cams,
                                                               const double* __restrict__ lpair,
                                                               const double2* __restrict__ uv,
                                                               double* __restrict__ g_uv) {
    __shared__ double red[kObsWaves][16 * (kWave + 1)];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int t = uniform_int(blockIdx.x * kObsWaves + wv);
    const bool active = t < p.T;
    double acc[15];
#pragma unroll
    for (int a = 0; a < 15; ++a) acc[a] = 0.0;
    int beg = 0, end = 0, ci = 0;
    if (active) {
        ci = uniform_int(p.tile_cam[t]);
        beg = uniform_int(p.tile_begin[t]);
        end = uniform_int(p.tile_end[t]);
    }
    const CamT<R> c = load_cam<R>(cams + (size_t)ci * kCamRec);
    const R delta = (R)p.delta;
    for (int base = beg; base < end; base += kWave) {
        const int o = base + lane;
        if (o < end) {
            const double2 u2 = uv[o];
            const R ux = (R)u2.x, uy = (R)u2.y;
            const LmRead<double> L = read_pair(lpair, p.obs_lm[o] & kLmMask);
            const R r2u = ux * ux + uy * uy;
            ObsEvalCF<LOSS, R> e;
            eval_obs_cf<LOSS, R>(c, (R)L.lk[0], (R)L.lk[1], (R)L.lk[2], ux, uy, r2u, r2u * r2u, delta, e);
            const R* ec = e.e;
            const R wl = e.w * e.lam;
            // grad_R = -w (m m^T / |m|^2) R (e p^T + p e^T)
            //        = -(w / |m|^2) m ((n . e) p^T + (n . p) e^T), exact for any 3x3 R
            const R ne = e.n[0] * ec[0] + e.n[1] * ec[1] + e.n[2] * ec[2];
            const R np = e.lam * e.r2;
            const R wr = e.w / e.r2;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
                    acc[3 * a + bb] += (double)(-wr * e.m[a] * (ne * e.p[bb] + np * ec[bb]));
            // grad_t = w lambda R e,  grad_l = -w lambda R e
            R Re[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) Re[a] = c.r[3 * a] * ec[0] + c.r[3 * a + 1] * ec[1] + c.r[3 * a + 2] * ec[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[9 + a] += (double)(wl * Re[a]);
            acc[12] += (double)(e.w * ec[2]);
            acc[13] += (double)(e.w * ec[2] * r2u);
            acc[14] += (double)(e.w * ec[2] * r2u * r2u);
            double* lr = p.rec + (size_t)p.obs_slot[o] * 8;
            lr[0] = (double)(-wl * Re[0]);
            lr[1] = (double)(-wl * Re[1]);
            lr[2] = (double)(-wl * Re[2]);
            if (g_uv) {
                const R dz = (R)2 * c.d[1] + (R)4 * c.d[2] * r2u;
                const int oi = p.obs_orig[o];
                // caller units: dF_px/du_px = s dF/du
                g_uv[2 * (size_t)oi] = p.scale * (double)(e.w * (ec[0] + ec[2] * dz * ux));
                g_uv[2 * (size_t)oi + 1] = p.scale * (double)(e.w * (ec[1] + ec[2] * dz * uy));
            }
        }
    }
    double* rw = red[wv];
#pragma unroll
    for (int v = 0; v < 15; ++v) rw[v * (kWave + 1) + lane] = acc[v];
    __syncthreads();
    if (active && lane < 15) {
        double s = 0.0;
        for (int q = 0; q < kWave; ++q) s += rw[lane * (kWave + 1) + q];
        p.grad_tile[(size_t)t * 16 + lane] = s;
    }
}

__global__ __launch_bounds__(256) void k_grad_entities(Params p, double* __restrict__ g_cams,
                                                       double* __restrict__ g_lms) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double sc = p.scale, s2 = sc * sc;
    if (i < p.M && g_cams) {
        double acc[15];
#pragma unroll
        for (int a = 0; a < 15; ++a) acc[a] = 0.0;
        for (int t = p.cam_tile_off[i]; t < p.cam_tile_off[i + 1]; ++t)
#pragma unroll
            for (int a = 0; a < 15; ++a) acc[a] += p.grad_tile[(size_t)t * 16 + a];
        double* g = g_cams + (size_t)p.cam_ext[i] * 15;
        for (int a = 0; a < 12; ++a) g[a] = s2 * acc[a];
        g[12] = s2 * acc[12] / sc;
        g[13] = s2 * acc[13] * sc;
        g[14] = s2 * acc[14] * sc * sc * sc;
    }
    const int64_t j = i - p.M;
    if (j >= 0 && j < p.N && g_lms) {
        // landmark li = j: its slots are in its group
        const int li = (int)j;
        // find the group by the per-landmark table packed in group arrays:
        // groups are contiguous in landmark id; binary search
        int lo = 0, hi = p.G - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (p.group_lm0[mid] <= li) lo = mid;
            else hi = mid - 1;
        }
        const int g = lo, n = p.group_n[g], D = p.group_deg[g], lane = li - p.group_lm0[g];
        double a0 = 0, a1 = 0, a2 = 0;
        for (int q = 0; q < D; ++q) {
            const double* r = p.rec + (size_t)(p.group_base[g] + (int64_t)q * n + lane) * 8;
            a0 += r[0];
            a1 += r[1];
            a2 += r[2];
        }
        double* gl = g_lms + (size_t)p.lm_ext[li] * 3;
        gl[0] = s2 * a0;
        gl[1] = s2 * a1;
        gl[2] = s2 * a2;
    }
}

// -------------------------------------------------------------- launchers

#define DABA_LOSS_SWITCH(LOSS_VAR, BODY)        \
    switch (LOSS_VAR) {                         \
    case 1: { constexpr int LS = 1; BODY; } break; \
    case 2: { constexpr int LS = 2; BODY; } break; \
    default: { constexpr int LS = 0; BODY; } break; \
    }

hipError_t launch_obs_pass(const Params& p, int k, hipStream_t s) {
    if (p.T == 0) return hipSuccess;
    const int T1 = p.T;
    dim3 grid((T1 + kObsWaves - 1) / kObsWaves), block(kObsWaves * kWave);
    DABA_LOSS_SWITCH(p.loss, {
        if (p.fp32) {
            if (p.accelerate) hipLaunchKernelGGL((k_obs_dma<float, LS, true>), dim3(T1), dim3(kWave), 0, s, p, k);
            else hipLaunchKernelGGL((k_obs_dma<float, LS, false>), dim3(T1), dim3(kWave), 0, s, p, k);
        } else {
            if (p.accelerate) hipLaunchKernelGGL((k_obs_dma<double, LS, true>), dim3(T1), dim3(kWave), 0, s, p, k);
            else hipLaunchKernelGGL((k_obs_dma<double, LS, false>), dim3(T1), dim3(kWave), 0, s, p, k);
        }
    });
    return hipGetLastError();
}

hipError_t launch_entity(const Params& p, int k, hipStream_t s) {
    dim3 grid(p.nCamBlocks + p.nLmBlocks + 2 * p.S), block(256);
    if (p.fp32) {
        if (p.accelerate) hipLaunchKernelGGL((k_entity<float, true>), grid, block, 0, s, p, k);
        else hipLaunchKernelGGL((k_entity<float, false>), grid, block, 0, s, p, k);
    } else {
        if (p.accelerate) hipLaunchKernelGGL((k_entity<double, true>), grid, block, 0, s, p, k);
        else hipLaunchKernelGGL((k_entity<double, false>), grid, block, 0, s, p, k);
    }
    return hipGetLastError();
}

hipError_t launch_decide(const Params& p, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(p.S), dim3(256), 0, s, p, k, 1);
    return hipGetLastError();
}

hipError_t launch_finalize(const Params& p, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(p.S), dim3(256), 0, s, p, k, 0);
    const int64_t n = p.M + p.N;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, k);
    return hipGetLastError();
}

hipError_t launch_extrapolate_cams(const Params& p, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_extrapolate_cams, dim3((unsigned)((p.M + 255) / 256)), dim3(256), 0, s, p, k);
    return hipGetLastError();
}

hipError_t launch_objective(const Params& p, const double* cams, const double* lpair, const double2* uv,
                            double* part_out, double* F_out, hipStream_t s) {
    double* tile_F = p.tile_vals;                       // reuse: T doubles
    double* bins = part_out ? p.tile_bins : nullptr;    // reuse: S * T doubles
    if (p.T > 0) {
        dim3 grid((p.T + kObsWaves - 1) / kObsWaves), block(kObsWaves * kWave);
        DABA_LOSS_SWITCH(p.loss, {
            if (p.fp32) hipLaunchKernelGGL((k_objective<float, LS>), grid, block, 0, s, p, cams, lpair, uv, tile_F, bins);
            else hipLaunchKernelGGL((k_objective<double, LS>), grid, block, 0, s, p, cams, lpair, uv, tile_F, bins);
        });
    }
    hipLaunchKernelGGL(k_objective_reduce, dim3(1), dim3(256), 0, s, p, tile_F, bins, part_out, F_out);
    return hipGetLastError();
}

hipError_t launch_import_point(const Params& p, const double* cams, const double* lms, const double* uv,
                               hipStream_t s) {
    int64_t n = p.M;
    if (p.N > n) n = p.N;
    if (p.K > n) n = p.K;
    hipLaunchKernelGGL(k_import, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, cams, lms, uv);
    return hipGetLastError();
}

hipError_t launch_grad(const Params& p, const double* cams, const double* lpair, const double2* uv,
                       double* g_cams, double* g_lms, double* g_uv, hipStream_t s) {
    if (p.T > 0) {
        dim3 grid((p.T + kObsWaves - 1) / kObsWaves), block(kObsWaves * kWave);
        DABA_LOSS_SWITCH(p.loss, {
            if (p.fp32) hipLaunchKernelGGL((k_grad_obs<float, LS>), grid, block, 0, s, p, cams, lpair, uv, g_uv);
            else hipLaunchKernelGGL((k_grad_obs<double, LS>), grid, block, 0, s, p, cams, lpair, uv, g_uv);
        });
    }
    const int64_t n = p.M + p.N;
    hipLaunchKernelGGL(k_grad_entities, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g_cams, g_lms);
    return hipGetLastError();
}

}  // namespace daba
