/*
 * daba_part.h -- C ABI of DABA with the paper's device-level surrogate on one
 * MI355X (gfx950).
 *
 * Sec. IV splits the observations into pairs whose camera and point lie on
 * the same device (kept exact) and pairs split between devices (majorized by
 * P_ij + Q_ij of Prop. 1); eq. Ealpha sums them, with a proximal term, into
 * one subproblem per device.  Here the devices are the S camera partitions of
 * one GPU.  Each device's subproblem is solved by Levenberg-Marquardt
 * (Sec. VII-B: one successful inner step) over all of its cameras and
 * landmarks at once: Gauss-Newton model with robust weights, the landmarks
 * eliminated by their 3x3 blocks (Schur complement), the reduced camera
 * system factorised densely by Cholesky.  Nesterov extrapolation and the
 * per-device adaptive restart (Sec. V, eq. Fak, lFak, Eak) are as in daba.h.
 *
 * Conventions are those of daba.h: int return codes (DABA_E_*), no device
 * allocation (one caller workspace), all work on the caller's stream, caller
 * units in and out.  The problem and option structs are daba.h's.  The
 * differences:
 *  - options.precision must be DABA_FP64 and options.inner_steps >= 1;
 *  - each partition's reduced camera system is a dense (9 M_a)^2 FP64 matrix
 *    in the workspace, M_a <= DABA_PART_MAX_CAMERAS;
 *  - daba_part_iterate synchronizes the stream once per LM attempt (the host
 *    loops until every device has its successful step or gives up).
 */
#ifndef DABA_PART_H
#define DABA_PART_H

#include "daba.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Largest number of cameras in one partition. */
#define DABA_PART_MAX_CAMERAS 2048

typedef struct daba_part_handle daba_part_handle;

/* Bytes of device workspace daba_part_create needs (0 if the problem or the
 * options are invalid).  Reads the sizes, the partitions and the observation
 * lists. */
size_t daba_part_workspace_bytes(const daba_problem *prob, const daba_options *opt);

/* Validates the problem and options, lays the problem out in the workspace
 * (256-byte aligned DEVICE pointer of at least daba_part_workspace_bytes()
 * bytes) and initialises eq. Fainit with the device surrogate:
 * F^a(-1) = Fbar^a(-1) = E^a(0) = E^a(x^(0) | x^(0)), x^(-1) = x^(0),
 * s^a = 1.  Synchronizes hip_stream. */
int daba_part_create(const daba_problem *prob, const daba_options *opt, void *dev_workspace,
                     size_t workspace_bytes, void *hip_stream, daba_part_handle **out);

/* n_iters iterations of Algorithm 1 with the device surrogate of eq. Ealpha.
 * F_trace (host [n_iters] or NULL) receives F after each iteration in
 * pixels^2.  Synchronizes. */
int daba_part_iterate(daba_part_handle *h, int n_iters, double *F_trace);

/* x^k in caller units (HOST cams [M*15], lms [N*3], either may be NULL) and
 * the metrics of the last iteration (HOST [S*4] or NULL):
 * (F^a(k), Fbar^a(k), E^a(k+1), restarted 0/1) in pixels^2.  Synchronizes. */
int daba_part_get_state(daba_part_handle *h, double *cams, double *lms, double *metrics);

/* Timing hook for measurement: runs n_iters iterations and returns through
 * ms_out (HOST [8]): [0..5] the summed GPU time in ms, from HIP events on
 * the handle's stream, of the objective and surrogate evaluations, the
 * normal-equation builds, the Schur-complement assembly, the Cholesky
 * factorisations, the triangular solves with the back-substitution, and the
 * rest (extrapolation, restart test, bookkeeping); [6] the LM attempts made;
 * [7] the Cholesky launches.  Synchronizes after every launch group, so the
 * total is slower than daba_part_iterate. */
int daba_part_iterate_timed(daba_part_handle *h, int n_iters, double *ms_out);

/* Checkpoint of everything the next iteration depends on (Sec. V): x^k and
 * x^(k-1) (HOST cams [M*15], lms [N*3], cams_prev, lms_prev; caller units
 * and order) and per partition part3 [S*3] = (Fbar^a(k-1), E^a(k) in
 * pixels^2, s^a(k)).  Any pointer may be NULL.  get synchronizes; set
 * replaces the given parts (rotations are not re-validated) and enqueues
 * the uploads, so that a handle created for the same problem and options
 * continues exactly where the checkpoint was taken. */
int daba_part_get_checkpoint(daba_part_handle *h, double *cams, double *lms, double *cams_prev,
                             double *lms_prev, double *part3);
int daba_part_set_checkpoint(daba_part_handle *h, const double *cams, const double *lms,
                             const double *cams_prev, const double *lms_prev, const double *part3);

int daba_part_destroy(daba_part_handle *h);

/* Text of the last error on this handle (or of the last failed create when h
 * is NULL); never NULL. */
const char *daba_part_last_error(const daba_part_handle *h);

#ifdef __cplusplus
}
#endif
#endif
