// Internal layout shared by the host layer and the gfx950 kernels of the DABA
// library.  Not part of the ABI.
//
// Device data layout (all inside the caller's workspace):
//  * observations in camera-major order (internal camera id, then internal
//    landmark id): pixel uv (double2 / float2, internal units), internal
//    landmark id, original index;
//  * cameras in partition-major order, one 128-byte record each
//    (R row-major 9 | t 3 | d 3 | pad): three rotating generations of the
//    chosen iterate, and the two candidates of the last iteration (plain MM
//    and accelerated) with the extrapolation each would give;
//  * landmarks in (partition, track length) order; the two candidates of the
//    last iteration as 64-byte pair records (candidate xyz, partition id,
//    l^k xyz, pad), double-buffered by iteration parity, with FP32 copies;
//  * the landmark index of an observation carries its landmark's partition
//    in the top bits (kLmBits), so a fetch can pick the partition's
//    candidate without reading the record first;
//  * the same observations a second time in landmark-major order, at their
//    slot: groups of up to 64 landmarks with one track length D are stored
//    observation-major (slot = base + k * n + lane), and each slot holds the
//    pixel and the observing camera (partition in the top bits), so the
//    landmark pass reads them coalesced and gathers only camera records,
//    which stay in cache.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace daba {

constexpr int kWave = 64;
constexpr int kObsWaves = 4;         // waves (tiles) per block of the observation pass
constexpr int kTileMax = 1024;       // most observations per tile (16 per lane)
constexpr int kTileMin = 256;        // fewest observations per landmark block (target)
constexpr int kMom = 38;             // moments of one surrogate
constexpr int kTileVals = 80;        // 2 * 38 moments, F share, gap share, pad
constexpr int kCamRec = 16;          // doubles per camera record
constexpr int kLmPair = 8;           // doubles per landmark pair record
constexpr int kCamBlock = 128;       // cameras per block of the camera solve
constexpr int kMaxPart = 64;
constexpr int kLmBits = 26;              // landmark index bits in obs_lm (partition above)
constexpr unsigned kLmMask = (1u << kLmBits) - 1;
constexpr int kCamBits = 26;             // camera index bits in slot_cam (partition above)
constexpr unsigned kCamMask = (1u << kCamBits) - 1;
// the landmark pass addresses a candidate's camera record with a 32-bit
// byte offset, (candidate M + camera) * 128 < 2^32
constexpr int kMaxCameras = (1 << 24) - 1;

// Two slots, by iteration parity: the restart test of iteration k - 1 reads
// slot (k - 1) & 1 and writes slot k & 1, which iteration k then uses.  The
// sticky error code and the decided flag live in slot 0.
struct DevState {
    double s;        // s^(k)
    double gamma;    // gamma^(k) used by iteration k
    double F;        // F(x^(k-1)) (internal units)
    int64_t k;
    int32_t err;     // sticky error code (0 = none), slot 0 only
    int32_t decided; // slot 0: 1 if the restart test of the last iteration is stored
};

// Everything a kernel needs, passed by value.
struct Params {
    int64_t M, N, K;
    int S, T, G;
    int nCamBlocks, nLmBlocks;
    int loss;
    double delta;   // internal units
    double xi, eta;
    int accelerate, inner_steps, fp32;
    uint64_t flags;
    double scale;

    // observations (camera-major)
    const double2* uv;
    const float2* uv32;
    const unsigned* obs_lm;   // internal landmark | partition << kLmBits
    const int* obs_orig;
    // the observations again, landmark-major at their slots
    const double2* luv;
    const float2* luv32;
    const unsigned* slot_cam; // internal camera | partition << kCamBits
    const int* slot_obs;      // camera-major index of the slot's observation
    // tiles
    const int* tile_cam;
    const int* tile_begin;
    const int* tile_end;
    const int* cam_tile_off;  // [M+1]
    const int* cam_part;      // [M] internal camera -> partition
    const int* part_cam;      // [S+1] first internal camera of each partition
    // landmark groups
    const int* group_lm0;
    const int* group_n;
    const int* group_deg;
    const int64_t* group_base;
    const int* lmblock_g0;    // [nLmBlocks]
    const int* lmblock_g1;
    // first camera block, landmark block and camera of each partition (so
    // that a block finds its partition, and the restart test its block
    // sums, without a memory load)
    int pcb[kMaxPart + 1], plb[kMaxPart + 1], pcam[kMaxPart + 1];
    const int* lmblock_part;  // [nLmBlocks] partition of each landmark block
    const int* cam_ext;       // internal -> caller camera index
    const int* lm_ext;        // internal -> caller landmark index
    const int* lm_part;       // [N] partition of each internal landmark

    // state.  Iteration k reads the candidates of parity (k + 1) & 1 (those
    // of iteration k - 1, chosen by its restart test) and writes parity k & 1.
    double* cams[3];          // chosen x^k in generation k % 3
    double* ccand[2][2];      // [parity][0: plain MM, 1: accelerated] camera candidates
    double* cbar[2][2];       // x-bar the next iteration uses if that candidate is chosen
    // FP32-mixed: per parity, both candidates (candidate c of camera i at
    // c M + i), each a 128-byte line holding the candidate's FP32 record
    // (16 floats) and that of its extrapolation, as the landmark pass reads
    // them: one cache line per observation
    float* cpk32[2];
    double* lcp[2][2];        // [parity][candidate] landmark pair records
    float* lcp32[2][2];
    int* restart;             // [S] restart test of the last decided iteration
    double* tile_vals;        // [T * kTileVals]
    double* tile_bins;        // [2S * T], column q*S + beta
    double* camblk_vals;      // [nCamBlocks * 4]
    double* lmblk_vals;       // [nLmBlocks * 2]
    double* colsum;           // [2S]
    // restart bookkeeping, [2 * S]: slot k & 1 holds the values iteration k
    // starts from, slot (k + 1) & 1 receives the updated ones
    double* Fbar;             // Fbar^a(k-1)
    double* E;                // E^a(k)
    double* EE;               // E^a(x^k | x^(k-1))
    double* Fprev;            // F^a(k-1)
    double* metrics;          // [S*4] of the last iteration
    double* fsh;              // [S] partition shares of F at the last restart test
    DevState* st;             // [2]
    double* trace;            // [trace_cap]
    int trace_cap;
    // scratch for caller-supplied points (objective / gradient)
    double* tmp_cams;         // [M * kCamRec]
    double* tmp_lpair;        // [N * kLmPair]
    double2* tmp_uv;          // [K]
    double* grad_tile;        // [T * 16]
};
static_assert(sizeof(Params) <= 4096, "Params is passed as a kernel argument");

// Launchers (daba_kernels.hip).  k mod 3 selects the camera generation and
// k mod 2 the landmark pair buffer.
// Observation pass: camera tiles (moments, F and gap shares), then landmark
// blocks (landmark-side sums and the landmark subproblems).
hipError_t launch_tiles(const Params& p, int k, hipStream_t s);
hipError_t launch_landmarks(const Params& p, int k, hipStream_t s);
hipError_t launch_entity(const Params& p, int k, hipStream_t s);  // camera subproblems, bin column sums
// Restart test of iteration k - 1 unless already stored (one block).
hipError_t launch_decide(const Params& p, int k, hipStream_t s);
// Restart test of iteration k - 1 and the choice of its candidates, written
// into both candidate slots and the camera generation k % 3 (a call
// boundary: afterwards every buffer holds x^k).
hipError_t launch_finalize(const Params& p, int k, hipStream_t s);
// Objective shares at (cams, lpair, uv): tile F shares and bins -> Fsh^a and F.
hipError_t launch_objective(const Params& p, const double* cams, const double* lpair, const double2* uv,
                            double* part_out /*[S]*/, double* F_out /*[1]*/, hipStream_t s);
// Both x-bar candidates of parity (k + 1) & 1 from (x^k, x^(k-1)) with gamma^(k)
// read from the state.
hipError_t launch_extrapolate_cams(const Params& p, int k, hipStream_t s);
// Caller arrays -> internal scratch (units and order).
hipError_t launch_import_point(const Params& p, const double* cams, const double* lms, const double* uv,
                               hipStream_t s);
hipError_t launch_grad(const Params& p, const double* cams, const double* lpair, const double2* uv,
                       double* g_cams, double* g_lms, double* g_uv, hipStream_t s);

}  // namespace daba
