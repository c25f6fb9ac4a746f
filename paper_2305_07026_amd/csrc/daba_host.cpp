// Host layer of the DABA library: validation, the device data layout, the
// workspace carve-up and the C ABI declared in include/daba.h.
#include "daba.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "daba_internal.h"

using namespace daba;

namespace {

constexpr int kTraceCap = 4096;
thread_local std::string g_create_error = "no error";

// Host-side description of the layout built from the observation lists.
struct Layout {
    int64_t M = 0, N = 0, K = 0;
    int S = 1;
    std::vector<int> cpart, lpart;              // caller index -> partition
    std::vector<int> cam_ext, cam_int;          // internal <-> caller
    std::vector<int> lm_ext, lm_int;
    std::vector<int> part_cam;                  // [S+1]
    std::vector<int> group_lm0, group_n, group_deg;
    std::vector<int64_t> group_base;
    std::vector<int> obs_order;                 // internal obs -> caller obs
    std::vector<uint32_t> obs_lm;               // internal obs: landmark | partition << kLmBits
    std::vector<int> obs_slot;                  // internal obs -> landmark-major slot
    std::vector<int> slot_obs;                  // slot -> internal obs
    std::vector<uint32_t> slot_cam;             // slot: camera | partition << kCamBits
    std::vector<int> cam_off;                   // [M+1] internal obs offsets
    std::vector<int> tile_cam, tile_begin, tile_end, cam_tile_off;
    std::vector<int> camblock_c0, camblock_c1, part_camblk;
    std::vector<int> lmblock_g0, lmblock_g1, part_lmblk, lmblock_part;
    int T = 0, G = 0;
    int block_obs = kTileMax;                   // observations per landmark block, about
};

// Landmark blocks of the fused pass: consecutive whole groups of one
// partition, closed once they hold at least `obs_per_block` observations (a
// group of landmarks nobody observes counts as one); one wave per block.
void build_lm_blocks(Layout& L, int64_t obs_per_block) {
    L.lmblock_g0.clear();
    L.lmblock_g1.clear();
    L.lmblock_part.clear();
    L.part_lmblk.assign(L.S + 1, 0);
    int g = 0;
    for (int a = 0; a < L.S; ++a) {
        L.part_lmblk[a] = (int)L.lmblock_g0.size();
        int g0 = g;
        while (g < L.G && L.lpart[L.lm_ext[L.group_lm0[g]]] == a) ++g;
        int64_t held = 0;
        int open = g0;
        for (int q = g0; q < g; ++q) {
            held += std::max<int64_t>((int64_t)L.group_n[q] * L.group_deg[q], 1);
            if (held >= obs_per_block || q + 1 == g) {
                L.lmblock_g0.push_back(open);
                L.lmblock_g1.push_back(q + 1);
                L.lmblock_part.push_back(a);
                open = q + 1;
                held = 0;
            }
        }
    }
    L.part_lmblk[L.S] = (int)L.lmblock_g0.size();
}

std::string vformat(const char* fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    return buf;
}

struct Fail {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::string m = vformat(fmt, ap);
    va_end(ap);
    throw Fail{code, m};
}

void hipcheck(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(DABA_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

void validate_sizes(const daba_problem* p) {
    if (!p) fail(DABA_E_INVAL, "problem is NULL");
    if (p->n_cameras < 1 || p->n_landmarks < 1 || p->n_obs < 0) fail(DABA_E_INVAL, "need M >= 1, N >= 1, K >= 0");
    if (p->n_cameras > (int64_t)kMaxCameras || p->n_landmarks > (int64_t)kLmMask || p->n_obs > 2000000000LL)
        fail(DABA_E_INVAL, "problem too large (at most %d cameras, 2^%d - 1 landmarks, 2e9 observations)",
             kMaxCameras, kLmBits);
    if (p->n_partitions < 1 || p->n_partitions > DABA_MAX_PARTITIONS)
        fail(DABA_E_INVAL, "n_partitions must be in [1, %d]", DABA_MAX_PARTITIONS);
    if (p->n_obs > 0 && (!p->obs_camera || !p->obs_landmark)) fail(DABA_E_INVAL, "observation lists are NULL");
}

// Builds the internal order of cameras, landmarks and observations.
void build_layout(const daba_problem* p, Layout& L) {
    validate_sizes(p);
    const int64_t M = p->n_cameras, N = p->n_landmarks, K = p->n_obs;
    const int S = p->n_partitions;
    L.M = M; L.N = N; L.K = K; L.S = S;
    for (int64_t o = 0; o < K; ++o) {
        if (p->obs_camera[o] < 0 || p->obs_camera[o] >= M) fail(DABA_E_INVAL, "obs_camera[%lld] out of range", (long long)o);
        if (p->obs_landmark[o] < 0 || p->obs_landmark[o] >= N)
            fail(DABA_E_INVAL, "obs_landmark[%lld] out of range", (long long)o);
    }
    // partitions: contiguous camera blocks; a landmark goes with the lowest
    // camera id that observes it
    L.cpart.assign(M, 0);
    const int64_t blk = (M + S - 1) / S;
    for (int64_t i = 0; i < M; ++i) {
        int a = p->camera_partition ? p->camera_partition[i] : (int)(i / blk);
        if (a < 0 || a >= S) fail(DABA_E_INVAL, "camera_partition[%lld] out of range", (long long)i);
        L.cpart[i] = a;
    }
    std::vector<int> deg(N, 0), lowcam(N, -1);
    for (int64_t o = 0; o < K; ++o) {
        int j = p->obs_landmark[o], i = p->obs_camera[o];
        deg[j]++;
        if (lowcam[j] < 0 || i < lowcam[j]) lowcam[j] = i;
    }
    L.lpart.assign(N, 0);
    for (int64_t j = 0; j < N; ++j) {
        int a = p->landmark_partition ? p->landmark_partition[j] : (lowcam[j] < 0 ? 0 : L.cpart[lowcam[j]]);
        if (a < 0 || a >= S) fail(DABA_E_INVAL, "landmark_partition[%lld] out of range", (long long)j);
        L.lpart[j] = a;
    }
    // cameras: stable order by partition
    L.part_cam.assign(S + 1, 0);
    for (int64_t i = 0; i < M; ++i) L.part_cam[L.cpart[i] + 1]++;
    for (int a = 0; a < S; ++a) L.part_cam[a + 1] += L.part_cam[a];
    {
        std::vector<int> fill(L.part_cam.begin(), L.part_cam.end() - 1);
        L.cam_ext.assign(M, 0);
        L.cam_int.assign(M, 0);
        for (int64_t i = 0; i < M; ++i) {
            int ci = fill[L.cpart[i]]++;
            L.cam_ext[ci] = (int)i;
            L.cam_int[i] = ci;
        }
    }
    // landmarks: stable order by (partition, track length)
    int maxdeg = 0;
    for (int64_t j = 0; j < N; ++j) maxdeg = std::max(maxdeg, deg[j]);
    {
        std::vector<int64_t> cnt((size_t)S * (maxdeg + 1) + 1, 0);
        for (int64_t j = 0; j < N; ++j) cnt[(size_t)L.lpart[j] * (maxdeg + 1) + deg[j] + 1]++;
        for (size_t q = 1; q < cnt.size(); ++q) cnt[q] += cnt[q - 1];
        L.lm_ext.assign(N, 0);
        L.lm_int.assign(N, 0);
        for (int64_t j = 0; j < N; ++j) {
            int64_t li = cnt[(size_t)L.lpart[j] * (maxdeg + 1) + deg[j]]++;
            L.lm_ext[li] = (int)j;
            L.lm_int[j] = (int)li;
        }
    }
    // groups of <= 64 landmarks with one partition and one track length
    int64_t base = 0;
    for (int64_t li = 0; li < N;) {
        int j = L.lm_ext[li];
        int a = L.lpart[j], D = deg[j];
        int64_t e = li;
        while (e < N && e - li < kWave && L.lpart[L.lm_ext[e]] == a && deg[L.lm_ext[e]] == D) ++e;
        L.group_lm0.push_back((int)li);
        L.group_n.push_back((int)(e - li));
        L.group_deg.push_back(D);
        L.group_base.push_back(base);
        base += (e - li) * (int64_t)D;
        li = e;
    }
    L.G = (int)L.group_lm0.size();
    // observations: camera-major (internal camera, internal landmark, caller index)
    {
        std::vector<int> by_lm(K), cntl(N + 1, 0);
        for (int64_t o = 0; o < K; ++o) cntl[L.lm_int[p->obs_landmark[o]] + 1]++;
        for (int64_t j = 0; j < N; ++j) cntl[j + 1] += cntl[j];
        for (int64_t o = 0; o < K; ++o) by_lm[cntl[L.lm_int[p->obs_landmark[o]]]++] = (int)o;
        L.cam_off.assign(M + 1, 0);
        for (int64_t o = 0; o < K; ++o) L.cam_off[L.cam_int[p->obs_camera[o]] + 1]++;
        for (int64_t i = 0; i < M; ++i) L.cam_off[i + 1] += L.cam_off[i];
        std::vector<int> fill(L.cam_off.begin(), L.cam_off.end() - 1);
        L.obs_order.assign(K, 0);
        for (int64_t q = 0; q < K; ++q) {
            int o = by_lm[q];
            L.obs_order[fill[L.cam_int[p->obs_camera[o]]]++] = o;
        }
    }
    // slots: the k-th observation of landmark li (in camera-major order) goes
    // to group_base + k * n + lane
    {
        std::vector<int> gid(N), lane(N), used(N, 0);
        for (int g = 0; g < L.G; ++g)
            for (int q = 0; q < L.group_n[g]; ++q) {
                gid[L.group_lm0[g] + q] = g;
                lane[L.group_lm0[g] + q] = q;
            }
        L.obs_lm.assign(K, 0);
        L.obs_slot.assign(K, 0);
        L.slot_obs.assign(K, 0);
        L.slot_cam.assign(K, 0);
        for (int64_t q = 0; q < K; ++q) {
            const int o = L.obs_order[q];
            const int li = L.lm_int[p->obs_landmark[o]];
            const int g = gid[li];
            L.obs_lm[q] = (uint32_t)li | ((uint32_t)L.lpart[L.lm_ext[li]] << kLmBits);
            const int slot = (int)(L.group_base[g] + (int64_t)used[li]++ * L.group_n[g] + lane[li]);
            L.obs_slot[q] = slot;
            L.slot_obs[slot] = (int)q;
            const int i = p->obs_camera[o];
            L.slot_cam[slot] = (uint32_t)L.cam_int[i] | ((uint32_t)L.cpart[i] << kCamBits);
        }
    }
    // tiles: each camera's observations in near-equal pieces of at most
    // kTileMax observations.  Landmark blocks hold about K / 4096
    // observations, rounded up to whole steps, within [kTileMin, kTileMax],
    // so that a small problem still has a few thousand landmark blocks.
    const int cap = kTileMax;
    L.block_obs = (int)std::min<int64_t>(kTileMax, std::max<int64_t>(kTileMin, (K / 4096 + kWave - 1) / kWave * kWave));
    L.cam_tile_off.assign(M + 1, 0);
    for (int64_t ci = 0; ci < M; ++ci) {
        int n = L.cam_off[ci + 1] - L.cam_off[ci];
        int nt = (n + cap - 1) / cap;
        int b = L.cam_off[ci];
        for (int q = 0; q < nt; ++q) {
            int sz = n / nt + (q < n % nt ? 1 : 0);
            L.tile_cam.push_back((int)ci);
            L.tile_begin.push_back(b);
            L.tile_end.push_back(b + sz);
            b += sz;
        }
        L.cam_tile_off[ci + 1] = (int)L.tile_cam.size();
    }
    L.T = (int)L.tile_cam.size();
    // camera-solve blocks and landmark-pass blocks, never straddling partitions
    L.part_camblk.assign(S + 1, 0);
    for (int a = 0; a < S; ++a) {
        L.part_camblk[a] = (int)L.camblock_c0.size();
        for (int c = L.part_cam[a]; c < L.part_cam[a + 1]; c += kCamBlock) {
            L.camblock_c0.push_back(c);
            L.camblock_c1.push_back(std::min(c + kCamBlock, L.part_cam[a + 1]));
        }
    }
    L.part_camblk[S] = (int)L.camblock_c0.size();
    build_lm_blocks(L, L.block_obs);
}

// Workspace carve-up: every array 256-byte aligned.
struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

void carve(const Layout& L, bool fp32, Carver& c, Params& p) {
    const size_t M = L.M, N = L.N, K = L.K, S = L.S, T = L.T, G = L.G;
    p.uv = c.take<double2>(K);
    p.uv32 = fp32 ? c.take<float2>(K) : nullptr;
    p.obs_lm = c.take<unsigned>(K);
    p.obs_orig = c.take<int>(K);
    // at least one slot, so that the landmark pass may read a slot it
    // discards even when nothing is observed
    const int64_t K1 = std::max<int64_t>(K, 1);
    p.luv = c.take<double2>(K1);
    p.luv32 = fp32 ? c.take<float2>(K1) : nullptr;
    p.slot_cam = c.take<unsigned>(K1);
    p.slot_obs = c.take<int>(K);
    p.tile_cam = c.take<int>(T);
    p.tile_begin = c.take<int>(T);
    p.tile_end = c.take<int>(T);
    p.cam_tile_off = c.take<int>(M + 1);
    p.cam_part = c.take<int>(M);
    p.part_cam = c.take<int>(S + 1);
    p.group_lm0 = c.take<int>(G);
    p.group_n = c.take<int>(G);
    p.group_deg = c.take<int>(G);
    p.group_base = c.take<int64_t>(G);
    p.lmblock_g0 = c.take<int>(L.lmblock_g0.size());
    p.lmblock_g1 = c.take<int>(L.lmblock_g0.size());
    p.lmblock_part = c.take<int>(L.lmblock_g0.size());
    p.cam_ext = c.take<int>(M);
    p.lm_ext = c.take<int>(N);
    p.lm_part = c.take<int>(N);
    for (int g = 0; g < 3; ++g) p.cams[g] = c.take<double>(M * kCamRec);
    // the two candidates of a parity are one allocation (the landmark pass
    // addresses candidate 1 as candidate 0 plus M records), and so are
    // their extrapolations
    for (int par = 0; par < 2; ++par) {
        double* b = c.take<double>(2 * M * kCamRec);
        p.ccand[par][0] = b;
        p.ccand[par][1] = b ? b + M * kCamRec : nullptr;
        double* e = c.take<double>(2 * M * kCamRec);
        p.cbar[par][0] = e;
        p.cbar[par][1] = e ? e + M * kCamRec : nullptr;
        p.cpk32[par] = fp32 ? c.take<float>(2 * M * 2 * kCamRec) : nullptr;
    }
    // the two candidates of a parity are one allocation (the observation
    // pass addresses candidate 1 as candidate 0 plus N records)
    for (int par = 0; par < 2; ++par) {
        double* b = c.take<double>(2 * N * kLmPair);
        p.lcp[par][0] = b;
        p.lcp[par][1] = b ? b + N * kLmPair : nullptr;
        float* bf = fp32 ? c.take<float>(2 * N * kLmPair) : nullptr;
        p.lcp32[par][0] = bf;
        p.lcp32[par][1] = bf ? bf + N * kLmPair : nullptr;
    }
    p.restart = c.take<int>(S);
    p.tile_vals = c.take<double>(std::max<size_t>(T * kTileVals, 1));
    p.tile_bins = c.take<double>(2 * S * std::max<size_t>(T, 1));
    p.camblk_vals = c.take<double>(L.camblock_c0.size() * 4);
    p.lmblk_vals = c.take<double>(L.lmblock_g0.size() * 2);
    p.colsum = c.take<double>(2 * S);
    p.Fbar = c.take<double>(2 * S);
    p.E = c.take<double>(2 * S);
    p.EE = c.take<double>(2 * S);
    p.Fprev = c.take<double>(2 * S);
    p.metrics = c.take<double>(4 * S);
    p.fsh = c.take<double>(S);
    p.st = c.take<DevState>(2);
    p.trace = c.take<double>(kTraceCap);
    p.trace_cap = kTraceCap;
    p.tmp_cams = c.take<double>(M * kCamRec);
    p.tmp_lpair = c.take<double>(N * kLmPair);
    p.tmp_uv = c.take<double2>(K);
    p.grad_tile = c.take<double>(std::max<size_t>(T, 1) * 16);
    (void)c.take<double>(S + 1);  // objective outputs (recomputed below)
}

double* objective_scratch(const Layout& L, bool fp32, char* base) {
    Carver c{base};
    Params p{};
    carve(L, fp32, c, p);
    c.off -= (L.S + 1) * sizeof(double);
    return reinterpret_cast<double*>(base + c.off);
}

bool rotation_ok(const double* R) {
    double err = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = R[a] * R[b] + R[3 + a] * R[3 + b] + R[6 + a] * R[6 + b];
            err = std::max(err, std::fabs(s - (a == b ? 1.0 : 0.0)));
        }
    double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                 R[2] * (R[3] * R[7] - R[4] * R[6]);
    return err <= 1e-6 && det > 0.0;
}

void validate_options(const daba_options* o) {
    if (!o) fail(DABA_E_INVAL, "options are NULL");
    if (o->loss < 0 || o->loss > 2) fail(DABA_E_INVAL, "unknown loss %d", o->loss);
    if (o->loss != DABA_LOSS_TRIVIAL && !(o->loss_delta > 0.0 && std::isfinite(o->loss_delta)))
        fail(DABA_E_INVAL, "loss_delta must be positive");
    if (!(o->xi > 0.0 && std::isfinite(o->xi))) fail(DABA_E_INVAL, "xi must be positive");
    if (!(o->eta > 0.0 && o->eta <= 1.0)) fail(DABA_E_INVAL, "eta must be in (0, 1]");
    if (o->precision != DABA_FP64 && o->precision != DABA_FP32_MIXED) fail(DABA_E_INVAL, "unknown precision");
}

void cam_to_internal(const double* in, double s, double* out) {
    for (int a = 0; a < 12; ++a) out[a] = in[a];
    out[12] = in[12] / s;
    out[13] = in[13] * s;
    out[14] = in[14] * s * s * s;
    out[15] = 0.0;
}
void cam_to_caller(const double* in, double s, double* out) {
    for (int a = 0; a < 12; ++a) out[a] = in[a];
    out[12] = in[12] * s;
    out[13] = in[13] / s;
    out[14] = in[14] / (s * s * s);
}

}  // namespace

struct daba_handle {
    Params p{};
    Layout L;
    daba_options opt{};
    hipStream_t stream = nullptr;
    int64_t k = 0;
    double* d_obj = nullptr;  // [S+1] device scratch for objective outputs
    std::string err = "no error";
    // six iterations (one period of the buffer rotation) as a HIP graph
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t period = nullptr;
    bool graphs = true;
    ~daba_handle() {
        if (period) (void)hipGraphExecDestroy(period);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

int guard(daba_handle* h, int (*fn)(daba_handle*, void*), void* ctx) {
    try {
        return fn(h, ctx);
    } catch (const Fail& f) {
        if (h) h->err = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        if (h) h->err = "host allocation failed";
        return DABA_E_NOMEM;
    }
}

void upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    hipcheck(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync H2D");
}
void download(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    hipcheck(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
}

void sync_and_check(daba_handle* h) {
    DevState st;
    download(&st, h->p.st, sizeof st, h->stream);
    hipcheck(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (st.err == DABA_E_DEGENERATE) fail(DABA_E_DEGENERATE, "an observation has |l_j - t_i| <= 1e-12 (Assumption 2)");
    if (st.err == DABA_E_NONFINITE) fail(DABA_E_NONFINITE, "a non-finite objective value appeared");
    if (st.err != 0) fail(DABA_E_HIP, "device error %d", st.err);
}

// Buffers the current point lives in between calls (iteration counter k):
// cameras in generations k % 3 (x^k) and (k + 2) % 3 (x^(k-1)), landmark pair
// records (l^k, partition, l^(k-1)) in candidate slot 0 of parity (k + 1) & 1.
const double* cur_pair(const daba_handle* h) { return h->p.lcp[(h->k + 1) & 1][0]; }

// x^k and x^(k-1) (caller order and units, all four arrays) into every buffer
// iteration k reads: camera generations k % 3 and (k + 2) % 3, both camera
// candidate slots of parity (k + 1) & 1, and both landmark candidate slots as
// pair records (l^k, partition, l^(k-1)); both x-bar slots follow from
// gamma^(k) in the state.  Marks the restart test as taken.
void write_point(daba_handle* h, const double* cams, const double* lms, const double* cams_prev,
                 const double* lms_prev) {
    const Layout& L = h->L;
    Params& p = h->p;
    const double s = p.scale;
    const int k = (int)(h->k % 6);
    const int par = (k + 1) & 1;
    hipStream_t st = h->stream;
    std::vector<double> buf(L.M * kCamRec);
    for (int which = 0; which < 2; ++which) {
        const double* src = which == 0 ? cams : cams_prev;
        for (int64_t ci = 0; ci < L.M; ++ci) {
            const double* c = src + (size_t)L.cam_ext[ci] * 15;
            for (int a = 0; a < 15; ++a)
                if (!std::isfinite(c[a])) fail(DABA_E_INVAL, "camera %d has a non-finite entry", L.cam_ext[ci]);
            if (!rotation_ok(c)) fail(DABA_E_INVAL, "camera %d: R is not a rotation", L.cam_ext[ci]);
            cam_to_internal(c, s, &buf[(size_t)ci * kCamRec]);
        }
        const size_t bytes = buf.size() * sizeof(double);
        if (which == 0) {
            upload(p.cams[k % 3], buf.data(), bytes, st);
            upload(p.ccand[par][0], buf.data(), bytes, st);
            upload(p.ccand[par][1], buf.data(), bytes, st);
            if (h->opt.precision == DABA_FP32_MIXED) {
                // both candidates' FP32 halves; the extrapolated halves follow
                // from the extrapolation launch below
                std::vector<float> bf(2 * L.M * 2 * kCamRec, 0.0f);
                for (int c = 0; c < 2; ++c)
                    for (int64_t ci = 0; ci < L.M; ++ci)
                        for (int a = 0; a < kCamRec; ++a)
                            bf[((size_t)c * L.M + ci) * 2 * kCamRec + a] = (float)buf[(size_t)ci * kCamRec + a];
                upload(p.cpk32[par], bf.data(), bf.size() * sizeof(float), st);
                hipcheck(hipStreamSynchronize(st), "sync");
            }
        } else {
            upload(p.cams[(k + 2) % 3], buf.data(), bytes, st);
        }
        hipcheck(hipStreamSynchronize(st), "sync");
    }
    std::vector<double> pair(L.N * kLmPair);
    for (int64_t li = 0; li < L.N; ++li) {
        double* q = &pair[(size_t)li * kLmPair];
        const int j = L.lm_ext[li];
        for (int a = 0; a < 3; ++a) {
            q[a] = lms[3 * (size_t)j + a];
            q[4 + a] = lms_prev[3 * (size_t)j + a];
            if (!std::isfinite(q[a]) || !std::isfinite(q[4 + a]))
                fail(DABA_E_INVAL, "landmark %d has a non-finite entry", j);
        }
        long long beta = L.lpart[j];
        std::memcpy(&q[3], &beta, sizeof beta);
        q[7] = 0.0;
    }
    upload(p.lcp[par][0], pair.data(), pair.size() * sizeof(double), st);
    upload(p.lcp[par][1], pair.data(), pair.size() * sizeof(double), st);
    std::vector<float> pf;
    if (h->opt.precision == DABA_FP32_MIXED) {
        pf.resize(L.N * kLmPair);
        for (int64_t li = 0; li < L.N; ++li) {
            const double* q = &pair[(size_t)li * kLmPair];
            float* fq = &pf[(size_t)li * kLmPair];
            for (int a = 0; a < 3; ++a) {
                fq[a] = (float)q[a];
                fq[4 + a] = (float)q[4 + a];
            }
            int beta = L.lpart[L.lm_ext[li]];
            std::memcpy(&fq[3], &beta, sizeof beta);
            fq[7] = 0.0f;
        }
        upload(p.lcp32[par][0], pf.data(), pf.size() * sizeof(float), st);
        upload(p.lcp32[par][1], pf.data(), pf.size() * sizeof(float), st);
    }
    hipcheck(launch_extrapolate_cams(p, k, st), "extrapolate");
    DevState s0;
    download(&s0, p.st, sizeof s0, st);
    hipcheck(hipStreamSynchronize(st), "sync");
    s0.decided = 1;
    upload(p.st, &s0, sizeof s0, st);
    hipcheck(hipStreamSynchronize(st), "sync");
}

// The current x^k and x^(k-1) in caller order and units; any output may be
// empty.  Synchronizes.
void read_point(daba_handle* h, std::vector<double>* cams, std::vector<double>* lms, std::vector<double>* cams_prev,
                std::vector<double>* lms_prev) {
    const Layout& L = h->L;
    Params& p = h->p;
    const double sc = p.scale;
    const int k = (int)(h->k % 6);
    hipStream_t st = h->stream;
    for (int which = 0; which < 2; ++which) {
        std::vector<double>* dst = which == 0 ? cams : cams_prev;
        if (!dst) continue;
        std::vector<double> buf(L.M * kCamRec);
        download(buf.data(), which == 0 ? p.cams[k % 3] : p.cams[(k + 2) % 3], buf.size() * sizeof(double), st);
        hipcheck(hipStreamSynchronize(st), "sync");
        dst->assign(L.M * 15, 0.0);
        for (int64_t ci = 0; ci < L.M; ++ci) cam_to_caller(&buf[(size_t)ci * kCamRec], sc, dst->data() + (size_t)L.cam_ext[ci] * 15);
    }
    if (lms || lms_prev) {
        std::vector<double> pair(L.N * kLmPair);
        download(pair.data(), cur_pair(h), pair.size() * sizeof(double), st);
        hipcheck(hipStreamSynchronize(st), "sync");
        if (lms) lms->assign(L.N * 3, 0.0);
        if (lms_prev) lms_prev->assign(L.N * 3, 0.0);
        for (int64_t li = 0; li < L.N; ++li) {
            const int j = L.lm_ext[li];
            for (int a = 0; a < 3; ++a) {
                if (lms) (*lms)[3 * (size_t)j + a] = pair[(size_t)li * kLmPair + a];
                if (lms_prev) (*lms_prev)[3 * (size_t)j + a] = pair[(size_t)li * kLmPair + 4 + a];
            }
        }
    }
}

// Assumption 2 at the current point, checked on the host from the caller's arrays
void check_assumption2(const daba_problem* pr) {
    for (int64_t o = 0; o < pr->n_obs; ++o) {
        const double* c = pr->cameras + 15 * (size_t)pr->obs_camera[o];
        const double* l = pr->landmarks + 3 * (size_t)pr->obs_landmark[o];
        double m0 = l[0] - c[9], m1 = l[1] - c[10], m2 = l[2] - c[11];
        if (!(m0 * m0 + m1 * m1 + m2 * m2 > 1e-24))
            fail(DABA_E_DEGENERATE, "observation %lld: |l - t| <= 1e-12 (Assumption 2)", (long long)o);
    }
}

void init_metrics(daba_handle* h) {
    // eq. Fainit: F^a(-1) = E^a(x^0 | x^0) = sum of each pair's halves of F
    Params& p = h->p;
    const int k = (int)h->k;
    hipcheck(launch_objective(p, p.cams[k % 3], cur_pair(h), p.uv, h->d_obj, h->d_obj + h->L.S, h->stream),
             "objective");
    std::vector<double> part(h->L.S + 1);
    download(part.data(), h->d_obj, part.size() * sizeof(double), h->stream);
    sync_and_check(h);
    const int S = h->L.S;
    const size_t slot = (size_t)(h->k & 1) * S;
    upload(p.Fbar + slot, part.data(), S * sizeof(double), h->stream);
    upload(p.E + slot, part.data(), S * sizeof(double), h->stream);
    upload(p.EE + slot, part.data(), S * sizeof(double), h->stream);
    upload(p.Fprev + slot, part.data(), S * sizeof(double), h->stream);
    hipcheck(hipStreamSynchronize(h->stream), "sync");
}

}  // namespace

extern "C" {

size_t daba_workspace_bytes(const daba_problem* prob, const daba_options* opt) {
    try {
        validate_options(opt);
        Layout L;
        build_layout(prob, L);
        Carver c{nullptr};
        Params p{};
        carve(L, opt->precision == DABA_FP32_MIXED, c, p);
        return c.off + 256;
    } catch (...) {
        return 0;
    }
}

static bool ensure_period_graph(daba_handle* h);

int daba_create(const daba_problem* prob, const daba_options* opt, void* dev_workspace, size_t workspace_bytes,
                void* hip_stream, daba_handle** out) {
    if (!out) {
        g_create_error = "out is NULL";
        return DABA_E_INVAL;
    }
    *out = nullptr;
    daba_handle* h = nullptr;
    try {
        validate_options(opt);
        validate_sizes(prob);
        if (!prob->cameras || !prob->landmarks || (prob->n_obs > 0 && !prob->obs_uv))
            fail(DABA_E_INVAL, "problem arrays are NULL");
        if (!(prob->unit_scale > 0.0 && std::isfinite(prob->unit_scale))) fail(DABA_E_INVAL, "unit_scale must be positive");
        for (int64_t o = 0; o < 2 * prob->n_obs; ++o)
            if (!std::isfinite(prob->obs_uv[o])) fail(DABA_E_INVAL, "obs_uv has a non-finite entry");
        for (int64_t i = 0; i < prob->n_cameras; ++i) {
            const double* c = prob->cameras + 15 * (size_t)i;
            for (int a = 0; a < 15; ++a)
                if (!std::isfinite(c[a])) fail(DABA_E_INVAL, "camera %lld has a non-finite entry", (long long)i);
            if (!rotation_ok(c)) fail(DABA_E_INVAL, "camera %lld: R is not a rotation", (long long)i);
        }
        for (int64_t j = 0; j < 3 * prob->n_landmarks; ++j)
            if (!std::isfinite(prob->landmarks[j])) fail(DABA_E_INVAL, "landmarks have a non-finite entry");
        h = new daba_handle();
        h->opt = *opt;
        h->stream = (hipStream_t)hip_stream;
        if (const char* ng = std::getenv("DABA_NO_GRAPH")) h->graphs = !(ng[0] == '1');
        build_layout(prob, h->L);
        const Layout& L = h->L;
        const bool fp32 = opt->precision == DABA_FP32_MIXED;
        Carver c{nullptr};
        Params tmp{};
        carve(L, fp32, c, tmp);
        if (!dev_workspace) fail(DABA_E_INVAL, "workspace is NULL");
        if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) fail(DABA_E_INVAL, "workspace must be 256-byte aligned");
        if (workspace_bytes < c.off) fail(DABA_E_NOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, c.off);
        Carver cv{static_cast<char*>(dev_workspace)};
        Params& p = h->p;
        carve(L, fp32, cv, p);
        h->d_obj = objective_scratch(L, fp32, static_cast<char*>(dev_workspace));
        p.M = L.M; p.N = L.N; p.K = L.K; p.S = L.S; p.T = L.T; p.G = L.G;
        p.nCamBlocks = (int)L.camblock_c0.size();
        for (int a = 0; a <= L.S; ++a) {
            p.pcb[a] = L.part_camblk[a];
            p.plb[a] = L.part_lmblk[a];
            p.pcam[a] = L.part_cam[a];
        }
        p.nLmBlocks = (int)L.lmblock_g0.size();
        p.loss = opt->loss;
        p.scale = prob->unit_scale;
        p.delta = opt->loss == DABA_LOSS_TRIVIAL ? 1.0 : opt->loss_delta / prob->unit_scale;
        p.xi = opt->xi;
        p.eta = opt->eta;
        p.accelerate = opt->accelerate ? 1 : 0;
        p.inner_steps = opt->inner_steps;
        p.fp32 = fp32 ? 1 : 0;
        p.flags = opt->debug_flags;
        check_assumption2(prob);
        // device work starts here

        hipStream_t s = h->stream;
        const int64_t K = L.K;
        // observations
        std::vector<double2> uv(K);
        std::vector<int> orig(K);
        for (int64_t q = 0; q < K; ++q) {
            int o = L.obs_order[q];
            orig[q] = o;
            uv[q] = make_double2(prob->obs_uv[2 * (size_t)o] / p.scale, prob->obs_uv[2 * (size_t)o + 1] / p.scale);
        }
        upload((void*)p.uv, uv.data(), K * sizeof(double2), s);
        // the same pixels landmark-major, at their slots
        std::vector<double2> luv(K);
        for (int64_t q = 0; q < K; ++q) luv[L.obs_slot[q]] = uv[q];
        upload((void*)p.luv, luv.data(), K * sizeof(double2), s);
        if (fp32) {
            std::vector<float2> uvf(K), luvf(K);
            for (int64_t q = 0; q < K; ++q) {
                uvf[q] = make_float2((float)uv[q].x, (float)uv[q].y);
                luvf[L.obs_slot[q]] = uvf[q];
            }
            upload((void*)p.uv32, uvf.data(), K * sizeof(float2), s);
            upload((void*)p.luv32, luvf.data(), K * sizeof(float2), s);
            hipcheck(hipStreamSynchronize(s), "sync");
        }
        upload((void*)p.obs_lm, L.obs_lm.data(), K * sizeof(uint32_t), s);
        upload((void*)p.obs_orig, orig.data(), K * sizeof(int), s);
        upload((void*)p.slot_cam, L.slot_cam.data(), K * sizeof(uint32_t), s);
        upload((void*)p.slot_obs, L.slot_obs.data(), K * sizeof(int), s);
        upload((void*)p.tile_cam, L.tile_cam.data(), L.T * sizeof(int), s);
        upload((void*)p.tile_begin, L.tile_begin.data(), L.T * sizeof(int), s);
        upload((void*)p.tile_end, L.tile_end.data(), L.T * sizeof(int), s);
        upload((void*)p.cam_tile_off, L.cam_tile_off.data(), (L.M + 1) * sizeof(int), s);
        std::vector<int> cpart_int(L.M);
        for (int64_t ci = 0; ci < L.M; ++ci) cpart_int[ci] = L.cpart[L.cam_ext[ci]];
        upload((void*)p.cam_part, cpart_int.data(), L.M * sizeof(int), s);
        upload((void*)p.part_cam, L.part_cam.data(), (L.S + 1) * sizeof(int), s);
        upload((void*)p.group_lm0, L.group_lm0.data(), L.G * sizeof(int), s);
        upload((void*)p.group_n, L.group_n.data(), L.G * sizeof(int), s);
        upload((void*)p.group_deg, L.group_deg.data(), L.G * sizeof(int), s);
        upload((void*)p.group_base, L.group_base.data(), L.G * sizeof(int64_t), s);
        upload((void*)p.lmblock_g0, L.lmblock_g0.data(), L.lmblock_g0.size() * sizeof(int), s);
        upload((void*)p.lmblock_g1, L.lmblock_g1.data(), L.lmblock_g1.size() * sizeof(int), s);
        upload((void*)p.lmblock_part, L.lmblock_part.data(), L.lmblock_part.size() * sizeof(int), s);
        upload((void*)p.cam_ext, L.cam_ext.data(), L.M * sizeof(int), s);
        upload((void*)p.lm_ext, L.lm_ext.data(), L.N * sizeof(int), s);
        std::vector<int> lpart_int(L.N);
        for (int64_t li = 0; li < L.N; ++li) lpart_int[li] = L.lpart[L.lm_ext[li]];
        upload((void*)p.lm_part, lpart_int.data(), L.N * sizeof(int), s);
        hipcheck(hipStreamSynchronize(s), "sync");
        // state: x^(-1) = x^(0), s = 1, gamma = 0
        DevState st[2]{};
        st[0].s = 1.0;
        st[0].gamma = 0.0;
        st[0].k = 0;
        upload(p.st, st, sizeof st, s);
        std::vector<double> zero(std::max<int64_t>(4 * L.S, 1), 0.0);
        upload(p.metrics, zero.data(), 4 * L.S * sizeof(double), s);
        upload(p.fsh, zero.data(), L.S * sizeof(double), s);
        std::vector<int> zeroi(L.S, 0);
        upload(p.restart, zeroi.data(), L.S * sizeof(int), s);
        hipcheck(hipStreamSynchronize(s), "sync");
        h->k = 0;
        write_point(h, prob->cameras, prob->landmarks, prob->cameras, prob->landmarks);
        init_metrics(h);
        // capture the replayed period now, so that no later call pays for it
        ensure_period_graph(h);
        *out = h;
        return DABA_OK;
    } catch (const Fail& f) {
        g_create_error = f.msg;
        delete h;
        return f.code;
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        delete h;
        return DABA_E_NOMEM;
    }
}

// One iteration on stream s: the restart test of the previous iteration (one
// block per partition), the camera tiles, the landmark blocks, the camera
// solves; ev (optional, kEv events) brackets each launch.
constexpr int kEv = 5;
static void launch_iteration(daba_handle* h, int k, hipStream_t s, hipEvent_t* ev = nullptr) {
    const Params& p = h->p;
    if (ev) hipcheck(hipEventRecord(ev[0], s), "event");
    hipcheck(launch_decide(p, k, s), "k_decide");
    if (ev) hipcheck(hipEventRecord(ev[1], s), "event");
    hipcheck(launch_tiles(p, k, s), "k_tiles");
    if (ev) hipcheck(hipEventRecord(ev[2], s), "event");
    hipcheck(launch_landmarks(p, k, s), "k_lms");
    if (ev) hipcheck(hipEventRecord(ev[3], s), "event");
    hipcheck(launch_entity(p, k, s), "k_entity");
    if (ev) hipcheck(hipEventRecord(ev[4], s), "event");
}

// Captures iterations with k mod 6 = 0..5 once; replaying the graph runs one
// full period of the buffer rotation.
static bool ensure_period_graph(daba_handle* h) {
    if (h->period) return true;
    if (!h->graphs) return false;
    hipcheck(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    hipcheck(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    for (int k = 0; k < 6; ++k) launch_iteration(h, k, h->cap_stream);
    hipGraph_t g = nullptr;
    hipcheck(hipStreamEndCapture(h->cap_stream, &g), "hipStreamEndCapture");
    hipError_t e = hipGraphInstantiate(&h->period, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hipcheck(e, "hipGraphInstantiate");
    return true;
}

static int iterate_impl(daba_handle* h, int n, double* F_trace, double* ms) {
    if (n < 0) fail(DABA_E_INVAL, "n_iters < 0");
    Params& p = h->p;
    hipStream_t s = h->stream;
    const int64_t k0 = h->k;
    // per-kernel timing: events for up to kPool iterations, drained in batches
    constexpr int kPool = 64;
    std::vector<hipEvent_t> ev;
    hipEvent_t fin[2] = {nullptr, nullptr};
    int pooled = 0;
    // ms[0]: camera tiles, ms[1]: landmark blocks, ms[2]: camera solves,
    // ms[3]: restart tests (one per iteration) and the closing k_finalize
    auto drain = [&]() {
        if (pooled == 0) return;
        hipcheck(hipEventSynchronize(ev[kEv * (pooled - 1) + kEv - 1]), "event sync");
        constexpr int slot[kEv - 1] = {3, 0, 1, 2};
        for (int q = 0; q < pooled; ++q)
            for (int e = 0; e < kEv - 1; ++e) {
                float t = 0.f;
                hipcheck(hipEventElapsedTime(&t, ev[kEv * q + e], ev[kEv * q + e + 1]), "elapsed");
                ms[slot[e]] += t;
            }
        pooled = 0;
    };
    if (ms) {
        ev.resize(kEv * kPool);
        for (auto& e : ev) hipcheck(hipEventCreate(&e), "hipEventCreate");
        for (auto& e : fin) hipcheck(hipEventCreate(&e), "hipEventCreate");
        for (int e = 0; e < kEv - 1; ++e) ms[e] = 0.0;
    }
    int done = 0;
    while (done < n) {
        const int chunk = std::min(n - done, kTraceCap - 1);
        for (int it = 0; it < chunk; ++it) {
            if (!ms && h->k % 6 == 0 && chunk - it >= 6 && ensure_period_graph(h)) {
                hipcheck(hipGraphLaunch(h->period, s), "hipGraphLaunch");
                h->k += 6;
                it += 5;
                continue;
            }
            const int k = (int)(h->k % 6);
            launch_iteration(h, k, s, ms ? &ev[kEv * pooled] : nullptr);
            if (ms && ++pooled == kPool) drain();
            h->k++;
        }
        // the restart test of the chunk's last iteration, and x^k stored plainly
        if (ms) hipcheck(hipEventRecord(fin[0], s), "event");
        hipcheck(launch_finalize(p, (int)(h->k % 6), s), "k_finalize");
        if (ms) {
            hipcheck(hipEventRecord(fin[1], s), "event");
            hipcheck(hipEventSynchronize(fin[1]), "event sync");
            float t = 0.f;
            hipcheck(hipEventElapsedTime(&t, fin[0], fin[1]), "elapsed");
            ms[3] += t;
        }
        if (F_trace) {
            // entries k0+done+1 .. k0+done+chunk-1 were written by this chunk
            std::vector<double> ring(kTraceCap);
            download(ring.data(), p.trace, kTraceCap * sizeof(double), s);
            sync_and_check(h);
            const double s2 = p.scale * p.scale;
            for (int i = done; i < done + chunk - 1; ++i) F_trace[i] = s2 * ring[(k0 + i + 1) % kTraceCap];
            if (done > 0) F_trace[done - 1] = s2 * ring[(k0 + done) % kTraceCap];
        }
        done += chunk;
    }
    if (F_trace && n > 0) {
        // F(x^(k0+n)): one objective pass at the new iterate
        const int k = (int)(h->k % 6);
        hipcheck(launch_objective(p, p.cams[k % 3], cur_pair(h), p.uv, nullptr, h->d_obj, s), "objective");
        double F;
        download(&F, h->d_obj, sizeof F, s);
        sync_and_check(h);
        F_trace[n - 1] = p.scale * p.scale * F;
    }
    if (ms) {
        drain();
        for (auto& e : ev) (void)hipEventDestroy(e);
        for (auto& e : fin) (void)hipEventDestroy(e);
    }
    return DABA_OK;
}

int daba_iterate(daba_handle* h, int n_iters, double* F_trace) {
    if (!h) return DABA_E_INVAL;
    struct C { int n; double* F; } c{n_iters, F_trace};
    return guard(h, [](daba_handle* hh, void* v) -> int {
        C* cc = static_cast<C*>(v);
        return iterate_impl(hh, cc->n, cc->F, nullptr);
    }, &c);
}

int daba_iterate_timed(daba_handle* h, int n_iters, double* ms_out) {
    if (!h || !ms_out) return DABA_E_INVAL;
    struct C { int n; double* ms; } c{n_iters, ms_out};
    return guard(h, [](daba_handle* hh, void* v) -> int {
        C* cc = static_cast<C*>(v);
        int r = iterate_impl(hh, cc->n, nullptr, cc->ms);
        sync_and_check(hh);
        return r;
    }, &c);
}

// Point for objective / gradient: caller arrays imported into scratch, or the
// current iterate.
static void prepare_point(daba_handle* h, const double* cams, const double* lms, const double* uv,
                          const double** pc, const double** pl, const double2** pu) {
    Params& p = h->p;
    const int k = (int)(h->k % 6);
    hipStream_t s = h->stream;
    if (!cams && !lms && !uv) {
        *pc = p.cams[k % 3];
        *pl = cur_pair(h);
        *pu = p.uv;
        return;
    }
    if (!cams)
        hipcheck(hipMemcpyAsync(p.tmp_cams, p.cams[k % 3], h->L.M * kCamRec * sizeof(double), hipMemcpyDeviceToDevice, s),
                 "copy");
    if (!lms)
        hipcheck(hipMemcpyAsync(p.tmp_lpair, cur_pair(h), h->L.N * kLmPair * sizeof(double),
                                hipMemcpyDeviceToDevice, s), "copy");
    if (!uv && h->L.K > 0)
        hipcheck(hipMemcpyAsync(p.tmp_uv, p.uv, h->L.K * sizeof(double2), hipMemcpyDeviceToDevice, s), "copy");
    hipcheck(launch_import_point(p, cams, lms, uv, s), "import");
    *pc = p.tmp_cams;
    *pl = p.tmp_lpair;
    *pu = p.tmp_uv;
}

int daba_objective(daba_handle* h, const double* cams, const double* lms, const double* uv, double* F_out) {
    if (!h || !F_out) return DABA_E_INVAL;
    struct C { const double *c, *l, *u; double* F; } c{cams, lms, uv, F_out};
    return guard(h, [](daba_handle* hh, void* v) -> int {
        C* cc = static_cast<C*>(v);
        const double *pc, *pl;
        const double2* pu;
        prepare_point(hh, cc->c, cc->l, cc->u, &pc, &pl, &pu);
        hipcheck(launch_objective(hh->p, pc, pl, pu, nullptr, hh->d_obj, hh->stream), "objective");
        double F;
        download(&F, hh->d_obj, sizeof F, hh->stream);
        sync_and_check(hh);
        *cc->F = hh->p.scale * hh->p.scale * F;
        return DABA_OK;
    }, &c);
}

int daba_grad(daba_handle* h, const double* cams, const double* lms, const double* uv, double* g_cams,
              double* g_lms, double* g_uv) {
    if (!h) return DABA_E_INVAL;
    struct C { const double *c, *l, *u; double *gc, *gl, *gu; } c{cams, lms, uv, g_cams, g_lms, g_uv};
    return guard(h, [](daba_handle* hh, void* v) -> int {
        C* cc = static_cast<C*>(v);
        const double *pc, *pl;
        const double2* pu;
        prepare_point(hh, cc->c, cc->l, cc->u, &pc, &pl, &pu);
        hipcheck(launch_grad(hh->p, pc, pl, pu, cc->gc, cc->gl, cc->gu, hh->stream), "grad");
        return DABA_OK;
    }, &c);
}

int daba_get_state(daba_handle* h, double* cams, double* lms, double* cams_prev, double* lms_prev, double* part4,
                   double* scalars2) {
    if (!h) return DABA_E_INVAL;
    struct C { double *c, *l, *cp, *lp, *p4, *sc; } c{cams, lms, cams_prev, lms_prev, part4, scalars2};
    return guard(h, [](daba_handle* hh, void* v) -> int {
        C* cc = static_cast<C*>(v);
        const Layout& L = hh->L;
        Params& p = hh->p;
        const int64_t k = hh->k;
        hipStream_t s = hh->stream;
        sync_and_check(hh);
        const double s2 = p.scale * p.scale;
        std::vector<double> vc, vl, vcp, vlp;
        read_point(hh, cc->c ? &vc : nullptr, cc->l ? &vl : nullptr, cc->cp ? &vcp : nullptr, cc->lp ? &vlp : nullptr);
        if (cc->c) std::memcpy(cc->c, vc.data(), vc.size() * sizeof(double));
        if (cc->l) std::memcpy(cc->l, vl.data(), vl.size() * sizeof(double));
        if (cc->cp) std::memcpy(cc->cp, vcp.data(), vcp.size() * sizeof(double));
        if (cc->lp) std::memcpy(cc->lp, vlp.data(), vlp.size() * sizeof(double));
        if (cc->p4) {
            const int S = L.S;
            std::vector<double> a(S), b(S), c2(S), d(S);
            const size_t slot = (size_t)(k & 1) * S;
            download(a.data(), p.Fbar + slot, S * sizeof(double), s);
            download(b.data(), p.E + slot, S * sizeof(double), s);
            download(c2.data(), p.EE + slot, S * sizeof(double), s);
            download(d.data(), p.Fprev + slot, S * sizeof(double), s);
            hipcheck(hipStreamSynchronize(s), "sync");
            for (int q = 0; q < S; ++q) {
                cc->p4[4 * q] = s2 * a[q];
                cc->p4[4 * q + 1] = s2 * b[q];
                cc->p4[4 * q + 2] = s2 * c2[q];
                cc->p4[4 * q + 3] = s2 * d[q];
            }
        }
        if (cc->sc) {
            DevState st;
            download(&st, p.st + (k & 1), sizeof st, s);
            hipcheck(hipStreamSynchronize(s), "sync");
            cc->sc[0] = st.s;
            cc->sc[1] = (double)st.k;
        }
        return DABA_OK;
    }, &c);
}

int daba_set_state(daba_handle* h, const double* cams, const double* lms, const double* cams_prev,
                   const double* lms_prev, const double* part4, const double* scalars2) {
    if (!h) return DABA_E_INVAL;
    struct C { const double *c, *l, *cp, *lp, *p4, *sc; } c{cams, lms, cams_prev, lms_prev, part4, scalars2};
    return guard(h, [](daba_handle* hh, void* v) -> int {
        C* cc = static_cast<C*>(v);
        Params& p = hh->p;
        hipStream_t s = hh->stream;
        const Layout& L = hh->L;
        hipcheck(hipStreamSynchronize(s), "sync");
        // the point as it is, with the parts the caller gives replaced
        std::vector<double> vc, vl, vcp, vlp;
        read_point(hh, &vc, &vl, &vcp, &vlp);
        if (cc->c) std::memcpy(vc.data(), cc->c, vc.size() * sizeof(double));
        if (cc->l) std::memcpy(vl.data(), cc->l, vl.size() * sizeof(double));
        if (cc->cp) std::memcpy(vcp.data(), cc->cp, vcp.size() * sizeof(double));
        if (cc->lp) std::memcpy(vlp.data(), cc->lp, vlp.size() * sizeof(double));
        // every input is checked before anything is changed, so that a call
        // that fails leaves the handle as it was
        for (const std::vector<double>* cs : {&vc, &vcp})
            for (int64_t i = 0; i < L.M; ++i) {
                const double* c = cs->data() + 15 * (size_t)i;
                for (int a = 0; a < 15; ++a)
                    if (!std::isfinite(c[a])) fail(DABA_E_INVAL, "camera %lld has a non-finite entry", (long long)i);
                if (!rotation_ok(c)) fail(DABA_E_INVAL, "camera %lld: R is not a rotation", (long long)i);
            }
        for (const std::vector<double>* ls : {&vl, &vlp})
            for (double v : *ls)
                if (!std::isfinite(v)) fail(DABA_E_INVAL, "landmarks have a non-finite entry");
        if (cc->sc && !(std::isfinite(cc->sc[0]) && cc->sc[0] >= 1.0 && std::isfinite(cc->sc[1]) && cc->sc[1] >= 0))
            fail(DABA_E_INVAL, "bad scalars (s >= 1, k >= 0)");
        if (cc->p4)
            for (int q = 0; q < 4 * L.S; ++q)
                if (!std::isfinite(cc->p4[q])) fail(DABA_E_INVAL, "part4 has a non-finite entry");
        if (cc->sc) {
            const int64_t knew = (int64_t)cc->sc[1];
            DevState sts[2];
            download(sts, p.st, sizeof sts, s);
            hipcheck(hipStreamSynchronize(s), "sync");
            DevState st = sts[knew & 1];
            st.s = cc->sc[0];
            const double s1 = (std::sqrt(4.0 * st.s * st.s + 1.0) + 1.0) / 2.0;
            st.gamma = p.accelerate ? (st.s - 1.0) / s1 : 0.0;
            st.k = knew;
            if ((knew & 1) != (hh->k & 1)) {
                // the restart bookkeeping follows the counter's parity slot
                const int S = L.S;
                for (double* arr : {p.Fbar, p.E, p.EE, p.Fprev})
                    hipcheck(hipMemcpyAsync(arr + (size_t)(knew & 1) * S, arr + (size_t)(hh->k & 1) * S,
                                            S * sizeof(double), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
            }
            hh->k = knew;
            if ((knew & 1) == 0) st.decided = sts[0].decided, st.err = sts[0].err;
            upload(p.st + (knew & 1), &st, sizeof st, s);
            hipcheck(hipStreamSynchronize(s), "sync");
        }
        write_point(hh, vc.data(), vl.data(), vcp.data(), vlp.data());
        {
            // no restart test is stored for the new point: clear the F shares
            // the next iteration would otherwise sum into an unread trace slot
            std::vector<double> z(L.S, 0.0);
            upload(p.fsh, z.data(), L.S * sizeof(double), s);
            hipcheck(hipStreamSynchronize(s), "sync");
        }
        if (cc->p4) {
            const int S = L.S;
            const double s2 = p.scale * p.scale;
            std::vector<double> a(S), b(S), c2(S), d(S);
            for (int q = 0; q < S; ++q) {
                a[q] = cc->p4[4 * q] / s2;
                b[q] = cc->p4[4 * q + 1] / s2;
                c2[q] = cc->p4[4 * q + 2] / s2;
                d[q] = cc->p4[4 * q + 3] / s2;
            }
            const size_t slot = (size_t)(hh->k & 1) * S;
            upload(p.Fbar + slot, a.data(), S * sizeof(double), s);
            upload(p.E + slot, b.data(), S * sizeof(double), s);
            upload(p.EE + slot, c2.data(), S * sizeof(double), s);
            upload(p.Fprev + slot, d.data(), S * sizeof(double), s);
            hipcheck(hipStreamSynchronize(s), "sync");
        }
        return DABA_OK;
    }, &c);
}

int daba_get_metrics(daba_handle* h, double* metrics) {
    if (!h || !metrics) return DABA_E_INVAL;
    return guard(h, [](daba_handle* hh, void* v) -> int {
        double* m = static_cast<double*>(v);
        sync_and_check(hh);
        const int S = hh->L.S;
        download(m, hh->p.metrics, 4 * S * sizeof(double), hh->stream);
        hipcheck(hipStreamSynchronize(hh->stream), "sync");
        const double s2 = hh->p.scale * hh->p.scale;
        for (int q = 0; q < S; ++q)
            for (int a = 0; a < 3; ++a) m[4 * q + a] *= s2;
        return DABA_OK;
    }, metrics);
}

int daba_destroy(daba_handle* h) {
    delete h;
    return DABA_OK;
}

const char* daba_last_error(const daba_handle* h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
