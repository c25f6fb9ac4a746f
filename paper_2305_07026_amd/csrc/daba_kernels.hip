// gfx950 kernels of one DABA iteration (Fan et al., Algorithm 1, Sec. VI)
// with every observation majorized (Prop. 1): the surrogate separates per
// camera and per landmark, and camera partitions act as the devices of the
// adaptive restart (Sec. V).
//
// Per iteration k (k mod 3 picks the camera generation, k mod 2 the parity
// of the candidate buffers), four launches:
//   k_decide   (one block per partition) the restart test of iteration
//              k - 1 (eq. Fak, lFak, Eak), which picks each partition's
//              candidate (eq. update_amm or update_mm) as x^k;
//   k_tiles    one wave per camera tile: evaluates its camera's
//              observations at x^k (taken from the chosen candidate), at
//              the extrapolated x-bar^k and at x^(k-1); accumulates the
//              camera moments of both surrogates (FP64), the F share and
//              the surrogate-gap share, and bins the landmark-side shares
//              per partition;
//   k_lms      one wave per landmark block walks the same observations
//              landmark-major, one lane per landmark: the pixel and camera
//              index of each of its observations read coalesced, the two
//              cameras gathered (their records stay in cache), the
//              landmark-side sums of both surrogates formed in registers
//              and the landmark subproblems solved in closed form;
//   k_entity   camera subproblems (Levenberg-Marquardt on the moments, and
//              the next extrapolation of each candidate, eq. nesterov_x) and
//              the column sums of the partition bins (the first also sums
//              the objective the restart test split by partition).
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
#include "daba_eval.h"
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

// A 64-byte FP64 pair record from LDS.
__device__ __forceinline__ LmRead<double> lds_pair(const char* rec) {
    const double2* q = reinterpret_cast<const double2*>(rec);
    const double2 a = q[0], b = q[1], c = q[2], d = q[3];
    LmRead<double> o;
    o.lk[0] = a.x; o.lk[1] = a.y; o.lk[2] = b.x;
    o.beta = (int)__double_as_longlong(b.y);
    o.lp[0] = c.x; o.lp[1] = c.y; o.lp[2] = d.x;
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

// v plus the value that DPP control CTRL moves into this lane, or plus zero
// where the lane has no source or its row is masked off (a 64-bit value moves
// as its two 32-bit halves from the same source lane).  With every row
// enabled a lane without a source reads zero (bound_ctrl), so the move needs
// no zeroed destination.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
    const long long b = __double_as_longlong(v);
    int lo, hi;
    if constexpr (ROW_MASK == 0xf) {
        lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    }
    return v + __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Inclusive prefix sum over the 64 lanes of a wave (every lane active):
// shifts by 1, 2, 4 and 8 within each row of 16 lanes (a Hillis-Steele
// scan), then lane 15's row total into rows 1 and 3 and lane 31's into rows
// 2 and 3.  Cross-lane moves by DPP, with no LDS round trip.
__device__ __forceinline__ double wave_scan(double v) {
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31
    return v;
}

// Segmented sum over the lanes of a wave (every lane active) whose keys are
// sorted (equal keys contiguous; key < 0 adds nothing): with P the inclusive
// prefix sum, a run [a, b] of key k sums to P[b] - P[a - 1], so the last lane
// of each run adds P to bins[key], then subtracts it from the bins of the next
// run's key.  Within each of the two updates the lanes name distinct bins, and
// a wave's LDS operations complete in order.
__device__ __forceinline__ void bin_add_sorted(double v0, double v1, int key, int lane, double* bins0,
                                               double* bins1) {
    const double P0 = wave_scan(v0), P1 = wave_scan(v1);
    // the shuffle with every lane active (an inactive source lane reads as 0)
    int nk = __shfl_down(key, 1, kWave);
    if (lane == kWave - 1) nk = -1;
    if (nk != key) {
        if (key >= 0) {
            bins0[key] += P0;
            bins1[key] += P1;
        }
        // another lane's bin: the compiler must not move these reads above
        // the writes (it may assume key != nk in this thread)
        asm volatile("" ::: "memory");
        if (nk >= 0) {
            bins0[nk] -= P0;
            bins1[nk] -= P1;
        }
    }
}

// The same segmented sum through LDS permutes (fewer VALU instructions, more
// LDS traffic): a segmented Hillis-Steele scan, the last lane of each run
// adding the run's sum into bins[key].
__device__ __forceinline__ void bin_add_sorted_lds(double v0, double v1, int key, int lane, double* bins0,
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

// The observation pass's segmented sum, each form where it is the faster
// one (measured): FP64, whose LDS also serves the 64-byte pair records, bins
// by DPP; FP32, whose VALU is the busier unit, through LDS permutes.
template <typename R>
__device__ __forceinline__ void bin_runs(double v0, double v1, int key, int lane, double* bins0, double* bins1) {
    if constexpr (sizeof(R) == 8) bin_add_sorted(v0, v1, key, lane, bins0, bins1);
    else bin_add_sorted_lds(v0, v1, key, lane, bins0, bins1);
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

// --------------------------------------------- observation pass: camera tiles
// One camera tile of the fused pass, with its memory traffic arranged for
// gfx950 (FP64, and FP32-mixed with 32-byte pair records): a step's 64
// landmark pair records are fetched straight into LDS (global_load_lds, no
// VGPRs), several lanes per record (16 bytes each) so that a wave
// instruction touches a few cache lines instead of 64; pixels come the same
// way.  The fetch for step s + 1 is issued while step s computes, into the
// other of two buffers, and the landmark indices it needs are loaded one
// step earlier still.  Every wave waits for its vector memory operations
// at the start of a step, explicitly: the compiler does not order an LDS
// read after an LDS DMA into the same object.  The buffers are separate
// objects, so that reading one while another is being filled needs no
// wait.  No LDS instruction may run while a DMA is in flight unless it
// names its object: the compiler would order it after every outstanding
// DMA (vmcnt(0)), so the landmark indices travel between lanes by DPP.
// The tile writes nothing per observation: the landmark side of each pair
// is evaluated again by the landmark blocks.
//
// Pair records in LDS: wave instruction i of a fetch brings the records of
// observations kNI a + i (a = 0 .. kRPI - 1), kLPR lanes per record in order,
// into the 1 KB at 1040 i, so the record of lane M starts at
// 1040 (M mod kNI) + kRecB (M / kNI): the 16-byte skew between the slabs
// makes the lanes' reads of their own records conflict free.
constexpr int kRedHalf = 7;  // rows of the reduction transpose per buffer (7 x 65 <= 512)
template <typename R>
struct ObsBuf;
template <>
struct __align__(16) ObsBuf<double> {
    char pair[1040 * 3 + 1024 + 16];  // pair records of a step (4 slabs)
    double2 uv[kWave];
    __device__ double* red() { return reinterpret_cast<double*>(pair); }  // reused for the tile reduction
};
template <>
struct __align__(16) ObsBuf<float> {
    char pair[1040 + 1024 + 16];  // 2 slabs
    float ux[kWave], uy[kWave];
    double red_[kRedHalf * (kWave + 1)];
    __device__ double* red() { return red_; }
};
static_assert(kRedHalf * (kWave + 1) * sizeof(double) <= sizeof(ObsBuf<double>::pair), "reduction fits a pair buffer");

// Lane j of the lane's quad (j < 4 a compile-time constant) by DPP, and the
// lane 2 (q / 2) + j of its pair for FP32 records (two lanes per record).
template <int J>
__device__ __forceinline__ int quad_lane(int v) {
    return __builtin_amdgcn_mov_dpp(v, J | (J << 2) | (J << 4) | (J << 6), 0xF, 0xF, false);
}
template <int J>
__device__ __forceinline__ int pair_lane(int v) {
    return __builtin_amdgcn_mov_dpp(v, J | (J << 2) | ((2 + J) << 4) | ((2 + J) << 6), 0xF, 0xF, false);
}

typedef __attribute__((address_space(3))) void* lds_ptr;
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
// the 32-bit LDS address of a __shared__ object
__device__ __forceinline__ unsigned lds_addr(const void* p) {
    return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}
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
// LDS of the fused pass (separate objects, so that the compiler can see
// that a read of one buffer does not depend on a DMA into the other).
template <typename R>
struct TileLds {
    ObsBuf<R>& A;
    ObsBuf<R>& B;
    ObsBuf<R>& C;
    double (&bins)[2][kMaxPart];
    double* cprev;  // x^(k-1) of the tile's camera (used by the gap only)
    double* cbarl;  // x-bar^k of the tile's camera
};

// vmcnt(n) with expcnt and lgkmcnt left alone (gfx9 encoding: vmcnt bits
// 3:0 and 15:14)
template <int N>
__device__ __forceinline__ void wait_vmem_n() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

template <typename R, int LOSS, bool ACC>
__device__ __forceinline__ void tile_role(const Params& p, int k, int t, const TileLds<R>& sh) {
    constexpr int kRecB = 8 * (int)sizeof(R);  // bytes of a pair record
    constexpr int kLPR = kRecB / 16;           // lanes per record
    constexpr int kRPI = kWave / kLPR;         // records per wave instruction
    constexpr int kNI = kWave / kRPI;          // instructions per step
    // memory instructions of one step's fetch: the pair records, then the pixels
    constexpr int kNF = kNI + (sizeof(R) == 8 ? 1 : 2);
    ObsBuf<R>& A = sh.A;
    ObsBuf<R>& B = sh.B;
    ObsBuf<R>& C = sh.C;
    double (&bins)[2][kMaxPart] = sh.bins;
    double* const cprev = sh.cprev;
    double* const cbarl = sh.cbarl;
    const int lane = threadIdx.x;
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
    bool bad = false;
    int run_key = -1;  // this lane's current run: key and sums
    double run0 = 0.0, run1 = 0.0;
    __syncthreads();

    const int last = end - 1;  // tiles are never empty
    const int ns = active ? (end - beg + kWave - 1) / kWave : 0;
    // Three buffers: step s computes from buffer s mod 3 while the fetches of
    // steps s + 1 and s + 2 are in flight.  The landmark index (with its
    // partition in the top bits) of each lane's observation in step s is
    // loaded into li[s mod 3] at step s - 3, before that step's fetch, so
    // that a step's wait can leave exactly the newest fetch outstanding.
    // Lane kLPR r + c fetches chunk c of record kRPI i + r in instruction i.
    int li0 = 0, li1 = 0, li2 = 0;
    auto load_li = [&](int st, int& dst) { dst = (int)p.obs_lm[min(beg + kWave * st + lane, last)]; };
    // Lane-derived offsets are recomputed inside each step from a lane index
    // the optimizer cannot see through: hoisted out of the loop they would
    // hold VGPRs for its whole length.
    auto opaque_lane = [&]() {
        int l = lane;
        asm volatile("" : "+v"(l));
        return l;
    };
    // the landmark index of observation kNI (lane / kLPR) + i: lane i of the
    // lane's quad (FP64, kNI = kLPR = 4) or of its pair (FP32, kNI = kLPR = 2)
    auto owner_li = [&](int v, auto ic) -> unsigned {
        constexpr int i = decltype(ic)::value;
        if constexpr (sizeof(R) == 8) return (unsigned)quad_lane<i>(v);
        else return (unsigned)pair_lane<i>(v);
    };
    static_assert(kNI == kLPR && (kLPR == 4 || kLPR == 2), "record mapping");
    auto fetch = [&](int st, ObsBuf<R>& D, int li_st) {
        const int ln = opaque_lane(), qc = ln % kLPR;
        auto one = [&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const unsigned lp = owner_li(li_st, ic);
            const unsigned li = lp & kLmMask;
            const uint64_t off = (uint64_t)chosen(restart, (int)(lp >> kLmBits)) * cand_stride +
                                 (uint64_t)li * kRecB + 16u * qc;
            dma16(pbase + off, D.pair + 1040 * i);
        };
        one(std::integral_constant<int, 0>{});
        one(std::integral_constant<int, 1>{});
        if constexpr (kNI == 4) {
            one(std::integral_constant<int, 2>{});
            one(std::integral_constant<int, 3>{});
        }
        const unsigned o = (unsigned)min(beg + kWave * st + ln, last);
        if constexpr (sizeof(R) == 8) {
            dma16(reinterpret_cast<const char*>(p.uv) + 16u * o, &D.uv[0]);
        } else {
            dma4(reinterpret_cast<const char*>(p.uv32) + 8u * o, &D.ux[0]);
            dma4(reinterpret_cast<const char*>(p.uv32) + 8u * o + 4u, &D.uy[0]);
        }
    };
    // step st computes from buffer Cur; step st + 2's data goes to F, with
    // the landmark indices in liF; step st + 3's indices are loaded into liL
    // Every step issues the same memory operations, also past the tile's
    // end (then every lane names the tile's last observation: one cache
    // line), so that the compiler's wait counts stay exact.
    auto step = [&](int st, const ObsBuf<R>& Cur, ObsBuf<R>& F, const int& liF, int& liL) {
        // this step's fetch (issued two steps ago) and the indices of step
        // st + 2 have arrived; step st + 1's fetch may still be in flight
        wait_vmem_n<kNF>();
        load_li(st + 3, liL);
        // the indices before the fetch, so that the fetch is the newest kNF
        // operations when the next step waits
        __builtin_amdgcn_sched_barrier(0);
        fetch(st + 2, F, liF);
        __builtin_amdgcn_sched_barrier(0);
        const int ln = opaque_lane();
        const int o = beg + kWave * st + ln;
        const bool on = o < end;
        double hF = 0.0, gp = 0.0;
        int key = -1;
        if (on) {
            R ux, uy, lk0, lk1, lk2, lp0, lp1, lp2;
            int beta;
            // The step's own buffer is read in one asm block that waits for its
            // reads: written as plain loads, the compiler would order them
            // after every DMA still in flight into the other buffers.
            const unsigned pr = lds_addr(Cur.pair) + 1040u * (unsigned)(ln % kNI) + (unsigned)(kRecB * (ln / kNI));
            if constexpr (sizeof(R) == 8) {
                const unsigned ua = lds_addr(Cur.uv) + 16u * (unsigned)ln;
                v2d u2, q0, q1, q2;
                double q3;
                asm volatile(
                    "ds_read_b128 %0, %5\n\t"
                    "ds_read_b128 %1, %6\n\t"
                    "ds_read_b128 %2, %6 offset:16\n\t"
                    "ds_read_b128 %3, %6 offset:32\n\t"
                    "ds_read_b64 %4, %6 offset:48\n\t"
                    "s_waitcnt lgkmcnt(0)"
                    : "=&v"(u2), "=&v"(q0), "=&v"(q1), "=&v"(q2), "=&v"(q3)
                    : "v"(ua), "v"(pr)
                    : "memory");
                ux = u2[0];
                uy = u2[1];
                lk0 = q0[0]; lk1 = q0[1]; lk2 = q1[0];
                beta = (int)__double_as_longlong(q1[1]);
                lp0 = q2[0]; lp1 = q2[1]; lp2 = q3;
            } else {
                const unsigned xa = lds_addr(Cur.ux) + 4u * (unsigned)ln, ya = lds_addr(Cur.uy) + 4u * (unsigned)ln;
                v4f f0, f1;
                float fx, fy;
                asm volatile(
                    "ds_read_b32 %0, %4\n\t"
                    "ds_read_b32 %1, %5\n\t"
                    "ds_read_b128 %2, %6\n\t"
                    "ds_read_b128 %3, %6 offset:16\n\t"
                    "s_waitcnt lgkmcnt(0)"
                    : "=&v"(fx), "=&v"(fy), "=&v"(f0), "=&v"(f1)
                    : "v"(xa), "v"(ya), "v"(pr)
                    : "memory");
                ux = fx;
                uy = fy;
                lk0 = f0[0]; lk1 = f0[1]; lk2 = f0[2];
                beta = __float_as_int(f0[3]);
                lp0 = f1[0]; lp1 = f1[1]; lp2 = f1[2];
            }
            const R r2u = ux * ux + uy * uy, r4u = r2u * r2u;
            const R r6u = r4u * r2u, r8u = r4u * r4u;
            ObsEval<LOSS, R> ek;
            eval_obs<LOSS, R>(ck, lk0, lk1, lk2, ux, uy, r2u, r4u, delta, ek);
            bad |= !(ek.r2 > (R)1e-24);
            add_moments<R>(acc, ek.w, ek.lam, ux, uy, r2u, r4u, r6u, r8u, ek.e);
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
            }
        }
        // landmark-side shares by landmark partition.  Within a camera the
        // observations are sorted by landmark partition, so the lanes' keys
        // are sorted within a step and each lane's keys never decrease from
        // step to step.  Each lane sums its own run of one key; when any
        // lane's key changes, the finished runs (keyed by the lanes' previous
        // keys, sorted too) are binned by one segmented sum.
        if (__any(key != run_key)) {
            const bool done = key != run_key;
            bin_runs<R>(done ? run0 : 0.0, done ? run1 : 0.0, run_key, lane, bins[0], bins[1]);
            if (done) {
                run0 = 0.0;
                run1 = 0.0;
                run_key = key;
            }
        }
        run0 += hF;
        run1 -= gp;
    };

    if (ns > 0) {
        load_li(0, li0);
        wait_vmem();
        load_li(1, li1);
        __builtin_amdgcn_sched_barrier(0);
        fetch(0, A, li0);
        wait_vmem_n<kNF>();  // li1 has arrived
        load_li(2, li2);
        __builtin_amdgcn_sched_barrier(0);
        fetch(1, B, li1);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int st = 0; st < ns; st += 3) {
        step(st, A, C, li2, li0);
        if (st + 1 < ns) step(st + 1, B, A, li0, li1);
        if (st + 2 < ns) step(st + 2, C, B, li1, li2);
    }
    bin_runs<R>(run0, run1, run_key, lane, bins[0], bins[1]);
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

// -------------------------------------------- observation pass: landmarks

// One observation's landmark-side terms of one surrogate (eq. Q): with the
// pair evaluated at the linearization point, W += w lambda^2 and
// V += w lambda e_w.  The products are formed in the evaluation type and
// summed in FP64.
template <int LOSS, typename R>
__device__ __forceinline__ void lm_terms(const CamT<R>& c, R l0, R l1, R l2, R ux, R uy, R delta, double& W,
                                         double* V) {
    const R r2u = ux * ux + uy * uy, r4u = r2u * r2u;
    ObsEval<LOSS, R> e;
    eval_obs<LOSS, R>(c, l0, l1, l2, ux, uy, r2u, r4u, delta, e);
    const R wl = e.w * e.lam;
    W += (double)(wl * e.lam);
    V[0] += (double)(wl * e.e[0]);
    V[1] += (double)(wl * e.e[1]);
    V[2] += (double)(wl * e.e[2]);
}

// The observations of a landmark block, one lane per landmark: slot s of
// landmark lane holds the pixel and the observing camera (with its
// partition, which picks the candidate the restart test chose).
template <typename R>
struct SlotObs {
    R ux, uy;
    unsigned cam;
};
template <typename R>
__device__ __forceinline__ SlotObs<R> read_slot(const Params& p, int64_t s);
template <>
__device__ __forceinline__ SlotObs<double> read_slot<double>(const Params& p, int64_t s) {
    const double2 u = p.luv[s];
    return {u.x, u.y, p.slot_cam[s]};
}
template <>
__device__ __forceinline__ SlotObs<float> read_slot<float>(const Params& p, int64_t s) {
    const float2 u = p.luv32[s];
    return {u.x, u.y, p.slot_cam[s]};
}

// Camera records of a landmark step in LDS.  Each lane's camera arrives as
// one or two 128-byte records: in FP64 the x^k record (16 doubles) and, for
// the accelerated surrogate, the x-bar^k record, one slab apart; in
// FP32-mixed one record holding both FP32 copies (x^k in the first 64
// bytes, x-bar^k in the second).  The 64 records of a slab (one per lane)
// arrive by LDS DMA in eight wave instructions, eight lanes per record, each
// lane of a group loading the next 16 bytes of the record, so that the
// addresser sees in-order runs and a wave instruction touches 8 cache
// lines.  Instruction i brings the records of lanes i, 8 + i, ..., 56 + i
// into the 1 KB at 1040 i: the record of lane M starts at
// 1040 (M mod 8) + 128 (M / 8).  The 16-byte skew between the slabs puts
// chunk j of the records of any 16 consecutive lanes in 16 different bank
// groups, so that every lane reading chunk j of its own record is conflict
// free, and chunk j is an immediate offset from the lane's base.  `rec` is
// the lane's record index in the candidate pair of allocations
// (candidate * M + camera).
constexpr int kCamSlab = 7 * 1040 + 1024 + 16;
template <int NSETS>
__device__ __forceinline__ void dma_cams(const void* __restrict__ base0, const void* __restrict__ base1, unsigned rec,
                                         char* lds) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const unsigned w = (unsigned)__shfl((int)rec, (lane & ~7) + i);
        const unsigned off = w * 128u + 16u * (unsigned)(lane & 7);
        dma16(reinterpret_cast<const char*>(base0) + off, lds + 1040 * i);
        if constexpr (NSETS == 2) dma16(reinterpret_cast<const char*>(base1) + off, lds + kCamSlab + 1040 * i);
    }
}
// Version v (0: x^k, 1: x-bar^k) of the lane's camera from LDS (rb: the
// lane's record offset), in the evaluation type.
template <typename R>
__device__ __forceinline__ CamT<R> lds_cam(const char* lds, int rb, int v) {
    typedef typename std::conditional<std::is_same<R, double>::value, double, float>::type T;
    constexpr int C = (int)sizeof(T);  // chunks of one version
    const char* src = sizeof(T) == 8 ? lds + kCamSlab * v + rb : lds + rb + 64 * v;
    T x[16];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const float4 c = *reinterpret_cast<const float4*>(src + 16 * j);
        __builtin_memcpy(&x[j * (16 / C)], &c, 16);
    }
    CamT<R> o;
#pragma unroll
    for (int a = 0; a < 9; ++a) o.r[a] = (R)x[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.t[a] = (R)x[9 + a];
#pragma unroll
    for (int a = 0; a < 3; ++a) o.d[a] = (R)x[12 + a];
    return o;
}
// lgkmcnt(0) with vmcnt and expcnt left alone: every LDS read of a step has
// returned before the next step's DMA overwrites the records
__device__ __forceinline__ void wait_lds() {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// The candidate pair records (the candidate l^(k+1), the partition id, l^k)
// of a landmark group (n <= 64 consecutive landmarks from lm0) written by
// iteration k, stored cooperatively: each lane's records go to LDS,
// then every store instruction writes 1 KB of consecutive bytes, 16 per
// lane, in whole lines, instead of each lane's own record in strided 16-byte
// pieces (those partial-line stores took about a quarter of the landmark
// pass at 60M observations).  The LDS (at least 8 KB) is free: the group's
// last step has read its camera records.  A wave's LDS operations complete
// in program order, so a later staging write cannot overtake an earlier
// read.  Lanes past n stage lane 0's landmark and store nothing.
template <bool ACC>
__device__ __forceinline__ void store_group_pairs(const Params& p, int k, int lm0, int n, char* lds,
                                                  const double* lm, const double* la, double beta_bits,
                                                  const double* lk) {
    const int lane = threadIdx.x;
    constexpr int kC = ACC ? 2 : 1;
    {
        double2* s0 = reinterpret_cast<double2*>(lds + 64 * lane);
        s0[0] = make_double2(lm[0], lm[1]);
        s0[1] = make_double2(lm[2], beta_bits);
        s0[2] = make_double2(lk[0], lk[1]);
        s0[3] = make_double2(lk[2], 0.0);
        if constexpr (ACC) {
            double2* s1 = reinterpret_cast<double2*>(lds + 4096 + 64 * lane);
            s1[0] = make_double2(la[0], la[1]);
            s1[1] = make_double2(la[2], beta_bits);
            s1[2] = make_double2(lk[0], lk[1]);
            s1[3] = make_double2(lk[2], 0.0);
        }
    }
    const int bytes = 64 * n;
#pragma unroll
    for (int c = 0; c < kC; ++c) {
        char* dst = reinterpret_cast<char*>(p.lcp[k & 1][c] + (size_t)lm0 * kLmPair);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int off = 1024 * i + 16 * lane;
            const float4 v = *reinterpret_cast<const float4*>(lds + 4096 * c + off);
            if (off < bytes) *reinterpret_cast<float4*>(dst + off) = v;
        }
    }
    if (p.fp32) {  // the 32-byte FP32 copies, staged over the first 4 KB
        const float bf = __int_as_float((int)__double_as_longlong(beta_bits));
        float4* s0 = reinterpret_cast<float4*>(lds + 32 * lane);
        s0[0] = make_float4((float)lm[0], (float)lm[1], (float)lm[2], bf);
        s0[1] = make_float4((float)lk[0], (float)lk[1], (float)lk[2], 0.0f);
        if constexpr (ACC) {
            float4* s1 = reinterpret_cast<float4*>(lds + 2048 + 32 * lane);
            s1[0] = make_float4((float)la[0], (float)la[1], (float)la[2], bf);
            s1[1] = make_float4((float)lk[0], (float)lk[1], (float)lk[2], 0.0f);
        }
        const int bytes32 = 32 * n;
#pragma unroll
        for (int c = 0; c < kC; ++c) {
            char* dst = reinterpret_cast<char*>(p.lcp32[k & 1][c] + (size_t)lm0 * kLmPair);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int off = 1024 * i + 16 * lane;
                const float4 v = *reinterpret_cast<const float4*>(lds + 2048 * c + off);
                if (off < bytes32) *reinterpret_cast<float4*>(dst + off) = v;
            }
        }
    }
}

// Landmark subproblems of one block of whole groups (one partition, about
// a tile's worth of observations), one kernel of one-wave blocks: for each
// group of equal track length D, lane q takes landmark group_lm0 + q and
// walks its D slots, one per step.  A step brings the 64 observing cameras
// (x^k and, accelerated, x-bar^k) into LDS together; the pixel and camera
// index of each slot are loaded two steps ahead, after the step's DMAs, so
// that the step's wait leaves them in flight.  Each observation is
// evaluated at x^k and at x-bar^k (the camera's stored extrapolation and
// l-bar = l^k + gamma (l^k - l^(k-1)), eq. nesterov_x).  The sums run in
// slot order, which is the camera-major order of the landmark's
// observations.  Then the closed forms (both candidates) and the block's
// surrogate changes for the restart test.
template <typename R, int LOSS, bool ACC>
__device__ __forceinline__ void lm_role(const Params& p, int k, int lb, char* lds) {
    const int lane = threadIdx.x;
    const double xi = p.xi;
    const uint64_t restart = restart_mask(p);
    const int par = (k + 1) & 1;
    const int lcc = chosen(restart, uniform_int(p.lmblock_part[lb]));
    const double* __restrict__ lpb = p.lcp[par][lcc];
    // the records of the parity's candidates, and how many per camera
    constexpr bool kF64 = sizeof(R) == 8;
    constexpr int kSets = (kF64 && ACC) ? 2 : 1;
    const void* ckb = kF64 ? (const void*)p.ccand[par][0] : (const void*)p.cpk32[par];
    const void* cbb = p.cbar[par][0];
    const unsigned M = (unsigned)p.M;
    const double gam = ACC ? p.st[k & 1].gamma : 0.0;
    const R gamr = (R)gam;
    const R delta = (R)p.delta;
    // where this lane's camera records sit in LDS
    const int rb = 1040 * (lane & 7) + 128 * (lane >> 3);
    const int g0 = uniform_int(p.lmblock_g0[lb]), g1 = uniform_int(p.lmblock_g1[lb]);
    double dmm = 0.0, dacc = 0.0;
    for (int g = g0; g < g1; ++g) {
        const int n = uniform_int(p.group_n[g]), D = uniform_int(p.group_deg[g]);
        const bool on = lane < n;
        const int ln = on ? lane : 0;  // lanes past n read lane 0's data and discard it
        const int li0 = uniform_int(p.group_lm0[g]);
        const int64_t base = p.group_base[g] + ln;
        // slot q of the lane's landmark, clamped to the group's last slot and
        // to the slot arrays (which hold at least one slot), so that every
        // group issues the same loads, also one with no observations
        const int64_t slot_max = p.K > 0 ? p.K - 1 : 0;
        auto slot_at = [&](int q) { return min(base + (int64_t)min(q, max(D - 1, 0)) * n, slot_max); };
        // the first two slots' addresses before any DMA is in flight (the
        // compiler would wait for every outstanding DMA before using a value
        // loaded earlier)
        const int64_t sl0 = slot_at(0), sl1 = slot_at(1);
        __builtin_amdgcn_sched_barrier(0);
        // the group's pair records (consecutive landmarks) arrive in LDS as
        // 1 KB runs, 16 bytes per lane, rather than as each lane's own record
        // in strided pieces; lanes past the group's records re-read its last
        // 16 bytes into slots nobody reads
        {
            const char* src = reinterpret_cast<const char*>(lpb + (size_t)li0 * kLmPair);
            const int last = 64 * n - 16;
#pragma unroll
            for (int i = 0; i < 4; ++i) dma16(src + min(1024 * i + 16 * lane, last), lds + 1024 * i);
        }
        __builtin_amdgcn_sched_barrier(0);
        SlotObs<R> s0 = read_slot<R>(p, sl0);
        SlotObs<R> s1 = read_slot<R>(p, sl1);
        wait_vmem_n<4>();  // the pair records; slots 0 and 1 stay in flight
        const LmRead<double> L = lds_pair(lds + 64 * ln);
        wait_lds();  // the record is in registers before the cameras' DMA reuses the LDS
        // the evaluation points in the evaluation type (as the camera tiles
        // form them from the pair records)
        const R lk0 = (R)L.lk[0], lk1 = (R)L.lk[1], lk2 = (R)L.lk[2];
        const R lp0 = (R)L.lp[0], lp1 = (R)L.lp[1], lp2 = (R)L.lp[2];
        const R lb0 = lk0 + gamr * (lk0 - lp0), lb1 = lk1 + gamr * (lk1 - lp1), lb2 = lk2 + gamr * (lk2 - lp2);
        double W0 = 0.0, V0[3] = {0.0, 0.0, 0.0}, W1 = 0.0, V1[3] = {0.0, 0.0, 0.0};
        // slot q of this lane's landmark at base + q n
        // Step q's camera records wait in LDS when the step starts; they are
        // read into registers, and step q + 1's DMA is issued before step q
        // is evaluated, so that the DMA's latency overlaps the arithmetic.
        // Slot q + 1 is in s0 and slot q + 2 in s1 (loaded during step
        // q - 1); the prefetch past the last slot re-reads it, so that every
        // step issues the same loads and the compiler's wait counts stay
        // exact.
        auto rec_of = [&](unsigned cam) {
            // the record of the candidate the camera's partition chose
            return (unsigned)chosen(restart, (int)(cam >> kCamBits)) * M + (cam & kCamMask);
        };
        if (D > 0) {
            R ux = s0.ux, uy = s0.uy;
            dma_cams<kSets>(ckb, cbb, rec_of(on ? s0.cam : 0u), lds);
            __builtin_amdgcn_sched_barrier(0);
            s0 = s1;
            s1 = read_slot<R>(p, slot_at(2));
            wait_vmem_n<2>();  // step 0's records; slot 2 stays in flight
            for (int q = 0; q < D; ++q) {
                const CamT<R> xk = lds_cam<R>(lds, rb, 0);
                CamT<R> xb;
                if constexpr (ACC) xb = lds_cam<R>(lds, rb, 1);
                const R cux = ux, cuy = uy;
                wait_lds();  // the records are in registers; the LDS is free
                if (q + 1 < D) dma_cams<kSets>(ckb, cbb, rec_of(on ? s0.cam : 0u), lds);
                ux = s0.ux;
                uy = s0.uy;
                __builtin_amdgcn_sched_barrier(0);
                s0 = s1;
                s1 = read_slot<R>(p, slot_at(q + 3));
                __builtin_amdgcn_sched_barrier(0);
                if (on) {
                    lm_terms<LOSS, R>(xk, lk0, lk1, lk2, cux, cuy, delta, W0, V0);
                    if constexpr (ACC) lm_terms<LOSS, R>(xb, lb0, lb1, lb2, cux, cuy, delta, W1, V1);
                }
                wait_vmem_n<2>();  // step q + 1's records; slot q + 3 stays in flight
            }
        }
        // closed forms: l = l^y + V / (2W + xi) about each linearization
        // point (every lane: a lane past n repeats lane 0's landmark, counts
        // nothing and stores nothing)
        double dl[3], nm = 0.0, dv = 0.0;
        const double den0 = 2.0 * W0 + xi;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dl[a] = V0[a] / den0;
            nm += dl[a] * dl[a];
            dv += dl[a] * V0[a];
        }
        if (on) dmm += (W0 + 0.5 * xi) * nm - dv;
        const double beta_bits = __longlong_as_double((long long)L.beta);
        const double lm[3] = {L.lk[0] + dl[0], L.lk[1] + dl[1], L.lk[2] + dl[2]};
        double la[3] = {lm[0], lm[1], lm[2]};
        if constexpr (ACC) {
            const double den1 = 2.0 * W1 + xi;
            double na = 0.0, va = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double lbar = L.lk[a] + gam * (L.lk[a] - L.lp[a]);
                la[a] = lbar + V1[a] / den1;
                const double da = la[a] - L.lk[a];
                na += da * da;
                va += da * V0[a];
            }
            // the accelerated candidate measured on the surrogate about x^k
            if (on) dacc += (W0 + 0.5 * xi) * na - va;
        }
        store_group_pairs<ACC>(p, k, li0, n, lds, lm, la, beta_bits, L.lk);
    }
    dmm = wave_sum(dmm);
    dacc = wave_sum(dacc);
    if (lane == 0) {
        p.lmblk_vals[(size_t)lb * 2] = dmm;
        p.lmblk_vals[(size_t)lb * 2 + 1] = dacc;
    }
}

// The observation pass, two kernels of one-wave blocks on the same stream:
// camera tiles, then landmark blocks.  Each is bound by the memory requests
// it keeps in flight (random pair gathers from HBM; camera gathers from
// cache), so each gets the LDS and registers that maximize that.
template <typename R, int LOSS, bool ACC>
__global__ __launch_bounds__(kWave) void k_tiles(Params p, int k) {
    __shared__ ObsBuf<R> A;
    __shared__ ObsBuf<R> B;
    __shared__ ObsBuf<R> C;
    __shared__ double bins[2][kMaxPart];
    __shared__ double cprev[kCamRec];
    __shared__ double cbarl[kCamRec];
    const TileLds<R> sh{A, B, C, bins, cprev, cbarl};
    tile_role<R, LOSS, ACC>(p, k, blockIdx.x, sh);
}

template <typename R, int LOSS, bool ACC>
__global__ __launch_bounds__(kWave) void k_lms(Params p, int k) {
    __shared__ __align__(16) char cams[(sizeof(R) == 8 && ACC ? 2 : 1) * kCamSlab];
    lm_role<R, LOSS, ACC>(p, k, blockIdx.x, cams);
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
// A camera record (16 doubles) as its FP32 copy (16 floats).
__device__ __forceinline__ void store_rec32(float* __restrict__ d, const double* __restrict__ c) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
        reinterpret_cast<float4*>(d)[a] =
            make_float4((float)c[4 * a], (float)c[4 * a + 1], (float)c[4 * a + 2], (float)c[4 * a + 3]);
}
__device__ __forceinline__ void store_camd(double* __restrict__ c, const CamD& o);
__device__ __forceinline__ void store_cam32(float* __restrict__ d, const CamD& o) {
    double c[16];
    store_camd(c, o);
    store_rec32(d, c);
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
        if (p.fp32) store_cam32(p.cpk32[k & 1] + ((size_t)surr * p.M + ci) * 2 * kCamRec, c);
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
            if (p.fp32) store_rec32(p.cpk32[k & 1] + ((size_t)surr * p.M + ci) * 2 * kCamRec + kCamRec, cbar);
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

// One launch, two kinds of blocks: camera subproblems, then the column sums
// of the per-tile partition bins (the first of which also stores F of the
// previous iterate and clears the decided flag).  It runs after the fused
// pass, which has solved the landmark subproblems, so the camera role's
// register use (the LM solve) sets only this launch's occupancy.
template <bool ACC>
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
    // column sums of the per-tile partition bins
    const double* src = p.tile_bins + (size_t)cb * p.T;
    double s = 0.0;
    for (int t = threadIdx.x; t < p.T; t += 256) s += src[t];
    s = wave_sum(s);
    if (lane == 0) sred[wv][0] = s;
    __syncthreads();
    if (threadIdx.x == 0) p.colsum[cb] = sred[0][0] + sred[1][0] + sred[2][0] + sred[3][0];
    // F(x^(k-1)) from the shares this iteration's restart test stored
    if (cb == 0) {
        store_trace(p, k, fshl);
        if (threadIdx.x == 0) p.st[0].decided = 0;
    }
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
        if (p.fp32) {
            float4* r0 = reinterpret_cast<float4*>(p.cpk32[par] + (size_t)ci * 2 * kCamRec);
            float4* r1 = reinterpret_cast<float4*>(p.cpk32[par] + ((size_t)p.M + ci) * 2 * kCamRec);
            float4 y[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) y[a] = c ? r1[a] : r0[a];
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                r0[a] = y[a];
                r1[a] = y[a];
            }
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
    if (p.fp32) {
        store_rec32(p.cpk32[par] + (size_t)ci * 2 * kCamRec + kCamRec, cb);
        store_rec32(p.cpk32[par] + ((size_t)p.M + ci) * 2 * kCamRec + kCamRec, cb);
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
// grad_u = w (e_xy + e_z (2 d2 + 4 d3 |u|^2) u); camera sums per tile, pixel
// parts to the caller's index (the landmark parts: k_grad_lms).
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

__global__ __launch_bounds__(256) void k_grad_entities(Params p, double* __restrict__ g_cams) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double sc = p.scale, s2 = sc * sc;
    if (i < p.M) {
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
}

// Landmark parts of eq. DFij, grad_l = -w lambda R e (camera-frame e), one
// lane per landmark over its slots (camera-major order of its observations);
// each slot names the observation, whose pixel comes from uv.
template <typename R, int LOSS>
__global__ __launch_bounds__(256) void k_grad_lms(Params p, const double* __restrict__ cams,
                                                  const double* __restrict__ lpair, const double2* __restrict__ uv,
                                                  double* __restrict__ g_lms) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= p.N) return;
    const int li = (int)j;
    // the landmark's group: groups are contiguous in landmark id
    int lo = 0, hi = p.G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.group_lm0[mid] <= li) lo = mid;
        else hi = mid - 1;
    }
    const int g = lo, n = p.group_n[g], D = p.group_deg[g], lane = li - p.group_lm0[g];
    const LmRead<double> L = read_pair(lpair, li);
    const R delta = (R)p.delta;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int q = 0; q < D; ++q) {
        const int64_t s = p.group_base[g] + (int64_t)q * n + lane;
        const double2 u2 = uv[p.slot_obs[s]];
        const CamT<R> c = load_cam<R>(cams + (size_t)(p.slot_cam[s] & kCamMask) * kCamRec);
        const R ux = (R)u2.x, uy = (R)u2.y;
        const R r2u = ux * ux + uy * uy;
        ObsEvalCF<LOSS, R> e;
        eval_obs_cf<LOSS, R>(c, (R)L.lk[0], (R)L.lk[1], (R)L.lk[2], ux, uy, r2u, r2u * r2u, delta, e);
        const R wl = e.w * e.lam;
        R Re[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) Re[a] = c.r[3 * a] * e.e[0] + c.r[3 * a + 1] * e.e[1] + c.r[3 * a + 2] * e.e[2];
        a0 += (double)(-wl * Re[0]);
        a1 += (double)(-wl * Re[1]);
        a2 += (double)(-wl * Re[2]);
    }
    const double s2 = p.scale * p.scale;
    double* gl = g_lms + (size_t)p.lm_ext[li] * 3;
    gl[0] = s2 * a0;
    gl[1] = s2 * a1;
    gl[2] = s2 * a2;
}

// -------------------------------------------------------------- launchers

#define DABA_LOSS_SWITCH(LOSS_VAR, BODY)        \
    switch (LOSS_VAR) {                         \
    case 1: { constexpr int LS = 1; BODY; } break; \
    case 2: { constexpr int LS = 2; BODY; } break; \
    default: { constexpr int LS = 0; BODY; } break; \
    }

hipError_t launch_tiles(const Params& p, int k, hipStream_t s) {
    if (p.T == 0) return hipSuccess;
    const dim3 grid(p.T), block(kWave);
    DABA_LOSS_SWITCH(p.loss, {
        if (p.fp32) {
            if (p.accelerate) hipLaunchKernelGGL((k_tiles<float, LS, true>), grid, block, 0, s, p, k);
            else hipLaunchKernelGGL((k_tiles<float, LS, false>), grid, block, 0, s, p, k);
        } else {
            if (p.accelerate) hipLaunchKernelGGL((k_tiles<double, LS, true>), grid, block, 0, s, p, k);
            else hipLaunchKernelGGL((k_tiles<double, LS, false>), grid, block, 0, s, p, k);
        }
    });
    return hipGetLastError();
}

hipError_t launch_landmarks(const Params& p, int k, hipStream_t s) {
    const dim3 grid(p.nLmBlocks), block(kWave);
    DABA_LOSS_SWITCH(p.loss, {
        if (p.fp32) {
            if (p.accelerate) hipLaunchKernelGGL((k_lms<float, LS, true>), grid, block, 0, s, p, k);
            else hipLaunchKernelGGL((k_lms<float, LS, false>), grid, block, 0, s, p, k);
        } else {
            if (p.accelerate) hipLaunchKernelGGL((k_lms<double, LS, true>), grid, block, 0, s, p, k);
            else hipLaunchKernelGGL((k_lms<double, LS, false>), grid, block, 0, s, p, k);
        }
    });
    return hipGetLastError();
}

hipError_t launch_entity(const Params& p, int k, hipStream_t s) {
    dim3 grid(p.nCamBlocks + 2 * p.S), block(256);
    if (p.accelerate) hipLaunchKernelGGL((k_entity<true>), grid, block, 0, s, p, k);
    else hipLaunchKernelGGL((k_entity<false>), grid, block, 0, s, p, k);
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
    if (p.T > 0 && (g_cams || g_uv)) {
        dim3 grid((p.T + kObsWaves - 1) / kObsWaves), block(kObsWaves * kWave);
        DABA_LOSS_SWITCH(p.loss, {
            if (p.fp32) hipLaunchKernelGGL((k_grad_obs<float, LS>), grid, block, 0, s, p, cams, lpair, uv, g_uv);
            else hipLaunchKernelGGL((k_grad_obs<double, LS>), grid, block, 0, s, p, cams, lpair, uv, g_uv);
        });
    }
    if (g_cams)
        hipLaunchKernelGGL(k_grad_entities, dim3((unsigned)((p.M + 255) / 256)), dim3(256), 0, s, p, g_cams);
    if (g_lms) {
        const dim3 grid((unsigned)((p.N + 255) / 256)), block(256);
        DABA_LOSS_SWITCH(p.loss, {
            if (p.fp32) hipLaunchKernelGGL((k_grad_lms<float, LS>), grid, block, 0, s, p, cams, lpair, uv, g_lms);
            else hipLaunchKernelGGL((k_grad_lms<double, LS>), grid, block, 0, s, p, cams, lpair, uv, g_lms);
        });
    }
    return hipGetLastError();
}

}  // namespace daba
