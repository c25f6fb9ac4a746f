/*
 * daba.h -- C ABI of the MI355X (gfx950) implementation of one DABA
 * iteration: decentralized, accelerated bundle adjustment (Fan, Ortiz, Hsiao,
 * Monge, Dong, Murphey, Mukadam, "Decentralization and Acceleration Enables
 * Large-Scale Bundle Adjustment").
 *
 * The problem is Problem 1 (Sec. II): cameras c_i = (R_i, t_i, d_i) and points
 * l_j (Sec. III), observations u_ij, a robust loss rho, and a partition of the
 * variables onto S devices.  Each camera partition plays one of the paper's
 * devices for the adaptive-restart bookkeeping of Sec. V; every observation
 * is majorized by Prop. 1, so the surrogate splits per camera and per
 * landmark.  One call to daba_iterate runs Algorithm 1's loop body once per
 * iteration on the GPU.
 *
 * Conventions.
 *  - Every function returns 0 (DABA_OK) or a negative DABA_E_* code; nothing
 *    throws across the ABI.  daba_last_error() describes the last failure of
 *    a handle.
 *  - The library never allocates device memory.  The caller allocates one
 *    device workspace of daba_workspace_bytes() bytes (256-byte aligned) and
 *    keeps it alive until daba_destroy.  The library allocates only host
 *    memory for the handle.
 *  - All device work is ordered on the caller's HIP stream (hipStream_t
 *    passed as void*; NULL = the default stream).  Calls that return host
 *    values synchronize that stream.
 *  - A handle is not thread-safe; calls on one handle must not overlap.
 *  - Caller units: pixels for u, f and the loss width; d = (f, f*k1, f*k2)
 *    with u in pixels (eq. ray).  Internally the library works in units of
 *    pixels / unit_scale (exact for a power-of-two unit_scale); objective
 *    values and gradients are returned in caller units.
 */
#ifndef DABA_H
#define DABA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DABA_OK = 0,
    DABA_E_INVAL = -1,      /* bad argument or problem                        */
    DABA_E_NOMEM = -2,      /* workspace too small or host allocation failed  */
    DABA_E_HIP = -3,        /* a HIP runtime call failed                      */
    DABA_E_NONFINITE = -4,  /* a non-finite value appeared on the device      */
    DABA_E_DEGENERATE = -5  /* |l_j - t_i| <= eps for an observation (Assumption 2) */
};

enum { DABA_LOSS_TRIVIAL = 0, DABA_LOSS_HUBER = 1, DABA_LOSS_WELSCH = 2 };
enum { DABA_FP64 = 0, DABA_FP32_MIXED = 1 };
/* debug_flags: force the restart test's outcome (tests of Sec. V only) */
enum { DABA_DEBUG_NEVER_RESTART = 1, DABA_DEBUG_ALWAYS_RESTART = 2 };

/* Largest number of partitions (camera blocks) a handle accepts. */
#define DABA_MAX_PARTITIONS 64

typedef struct daba_handle daba_handle;

/* Problem 1 (Sec. II) with the camera model of Sec. III.  Host pointers; the
 * caller keeps ownership and may free them after daba_create returns. */
typedef struct {
    int64_t n_cameras, n_landmarks, n_obs;  /* M >= 1, N >= 1, K >= 0          */
    const int32_t *obs_camera;   /* [K] camera index i of each observation, any order */
    const int32_t *obs_landmark; /* [K] landmark index j                           */
    const double *obs_uv;        /* [K*2] observed distorted pixel u_ij, from the image centre */
    const double *cameras;       /* [M*15] R_i row-major (9) | t_i (3) | d_i (3)      */
    const double *landmarks;     /* [N*3] l_j                                       */
    int32_t n_partitions;        /* S, 1 <= S <= DABA_MAX_PARTITIONS                */
    const int32_t *camera_partition;   /* [M] or NULL: blocks of ceil(M/S) consecutive ids */
    const int32_t *landmark_partition; /* [N] or NULL: partition of the lowest camera id observing j */
    double unit_scale;           /* s > 0; power of two recommended                */
} daba_problem;

/* Algorithm 1's inputs xi and eta, the loss, and how each subproblem is
 * solved. */
typedef struct {
    int32_t loss;        /* DABA_LOSS_*; rho satisfies Assumption 1                       */
    double loss_delta;   /* Huber / Welsch width in pixels                                 */
    double xi;           /* proximal weight xi > 0 of eq. Ealpha (internal units)          */
    double eta;          /* 0 < eta <= 1, eq. lFak                                         */
    int32_t accelerate;  /* 1: Nesterov + adaptive restart (DABA); 0: plain MM (eq. update_mm) */
    int32_t inner_steps; /* successful Levenberg-Marquardt steps per camera subproblem; 1 as in
                            the paper's experiments; <= 0 iterates to convergence (Assumption 4) */
    int32_t precision;   /* DABA_FP64 or DABA_FP32_MIXED                                   */
    uint64_t debug_flags;
} daba_options;

/* Bytes of device workspace daba_create needs for this problem and options
 * (0 if the problem is invalid).  Reads only the sizes, the partition count
 * and the observation lists. */
size_t daba_workspace_bytes(const daba_problem *prob, const daba_options *opt);

/* Validates the problem (indices, partitions, finite values, rotations,
 * Assumption 2 at x^(0)), lays it out in the workspace and initialises the
 * restart metrics of eq. Fainit: F^a(-1) = E^a(x^(0) | x^(0)),
 * Fbar^a(-1) = F^a(-1), E^a(0) = F^a(-1), x^(-1) = x^(0), s^a(0) = 1.
 * dev_workspace: device pointer, at least daba_workspace_bytes() bytes.
 * hip_stream: the stream all later calls enqueue on.  Synchronizes it. */
int daba_create(const daba_problem *prob, const daba_options *opt, void *dev_workspace,
                size_t workspace_bytes, void *hip_stream, daba_handle **out);

/* Runs n_iters iterations of Algorithm 1 (Sec. VI): Nesterov extrapolation
 * (eq. nesterov_x), majorization (Prop. 1, eq. Ealpha), the per-camera and
 * per-landmark minimizations of the extrapolated and plain surrogates
 * (eq. update_amm, eq. update_mm) and the per-partition restart test
 * (eq. Fak, lFak, Eak).  If F_trace is not NULL it receives (host, [n_iters])
 * the objective F after each iteration in pixels^2, and the call
 * synchronizes the stream; otherwise it only enqueues work. */
int daba_iterate(daba_handle *h, int n_iters, double *F_trace);

/* F (eq. Fobj) in pixels^2 at the given point.  cams [M*15], lms [N*3],
 * uv [K*2] are DEVICE pointers in caller units and caller order, or NULL for
 * the current iterate / stored pixels.  Synchronizes. */
int daba_objective(daba_handle *h, const double *cams, const double *lms, const double *uv,
                   double *F_out);

/* Euclidean gradient of F (App. D, eq. DFij, with the intrinsics row
 * transposed back: dF/dd = rho' e_z (1, |u|^2, |u|^4)) at the given point
 * (same conventions as daba_objective), written to DEVICE buffers in caller
 * units and order: g_cams [M*15] (d/dR entries as a free 3x3 matrix, d/dt,
 * d/dd), g_lms [N*3], g_uv [K*2]; any output may be NULL.  Enqueues only. */
int daba_grad(daba_handle *h, const double *cams, const double *lms, const double *uv,
              double *g_cams, double *g_lms, double *g_uv);

/* State at the start of the next iteration k, HOST buffers, caller units:
 * x^k (cams [M*15], lms [N*3]), x^(k-1) (cams_prev, lms_prev), per partition
 * part4 [S*4] = (Fbar^a(k-1), E^a(k), E^a(x^k | x^(k-1)), F^a(k-1)) and
 * scalars2 = (s^(k), k).  Any pointer may be NULL.  Synchronizes. */
int daba_get_state(daba_handle *h, double *cams, double *lms, double *cams_prev, double *lms_prev,
                   double *part4, double *scalars2);
/* Replaces the state (same layout; NULL leaves that part unchanged). */
int daba_set_state(daba_handle *h, const double *cams, const double *lms, const double *cams_prev,
                   const double *lms_prev, const double *part4, const double *scalars2);

/* Per-partition metrics of the last iteration, HOST [S*4]:
 * (F^a(k), Fbar^a(k), E^a(k+1), restarted 0/1).  Synchronizes. */
int daba_get_metrics(daba_handle *h, double *metrics);

/* Timing hook for measurement: runs n_iters iterations and returns, through
 * ms_out (host [4]), the summed GPU time in ms of the camera-tile passes, of
 * the landmark passes (landmark-side sums and landmark subproblems), of the
 * camera subproblems, and of the restart tests (one small launch per
 * iteration) together with the closing launch that stores the final
 * iterate, measured with HIP events on the handle's stream around each
 * launch.  Synchronizes. */
int daba_iterate_timed(daba_handle *h, int n_iters, double *ms_out);

/* Measurement only, not part of the method: enqueues a plain streaming copy
 * of `bytes` bytes (a multiple of 16; both DEVICE pointers 16-byte aligned,
 * not overlapping) from src to dst on hip_stream, with `blocks` blocks of
 * 256 threads, so that a caller can time the bandwidth the GPU attains next
 * to the kernels of the iteration.  Returns DABA_E_INVAL for a bad argument,
 * DABA_E_HIP if the launch fails. */
int daba_stream_copy(void *dst, const void *src, size_t bytes, int blocks, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the robust
 * objective F = sum_ij 1/2 rho(|e_ij|^2) of Problem 1, as daba_objective
 * computes it, at caller arrays, with no handle and no workspace.
 *   n_cameras, n_landmarks >= 1; 0 <= n_obs <= DABA_NOALLOC_MAX_OBS;
 *   obs_camera, obs_landmark: DEVICE int32 [n_obs]; obs_uv: DEVICE [n_obs*2]
 *   pixels, principal point subtracted; cameras: DEVICE [n_cameras*15] in
 *   the layout of daba_problem; landmarks: DEVICE [n_landmarks*3]; loss and
 *   loss_delta (pixels) as in daba_options; F_out: DEVICE, one double, in
 *   caller units.
 * Enqueues on hip_stream and returns; allocates nothing (no hipMalloc, no
 * host allocation).  Its only device memory beyond the arguments is a
 * static array of DABA_NOALLOC_BLOCKS doubles per GPU, which the library
 * holds until the process ends; every call on a GPU shares it, so calls
 * that overlap on one GPU race and must be ordered by the caller.  Each
 * call writes every entry it reads, so no clearing is needed.  An
 * observation with an index out of range or a landmark at its camera centre
 * (Assumption 2) makes *F_out NaN.  Returns DABA_E_INVAL for a bad size,
 * pointer or loss (before any device work), DABA_E_HIP if the launch fails. */
#define DABA_NOALLOC_BLOCKS 4096
#define DABA_NOALLOC_MAX_OBS 2000000000LL
int daba_objective_noalloc(int64_t n_cameras, int64_t n_landmarks, int64_t n_obs, const int32_t *obs_camera,
                           const int32_t *obs_landmark, const double *obs_uv, const double *cameras,
                           const double *landmarks, int loss, double loss_delta, double *F_out, void *hip_stream);

/* Releases the handle (host memory only; the workspace stays the caller's). */
int daba_destroy(daba_handle *h);

/* Text of the last error on this handle (or of the last failed create when
 * h is NULL); never NULL. */
const char *daba_last_error(const daba_handle *h);

#ifdef __cplusplus
}
#endif
#endif
