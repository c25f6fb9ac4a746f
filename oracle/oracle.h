/*
 * Plain CPU FP64 oracle of the DABA iteration (Fan et al., "Decentralization
 * and Acceleration Enables Large-Scale Bundle Adjustment").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * it.  It shares no code, header or table with the GPU library.
 *
 * Every quantity is computed from its definition in the paper by direct sums
 * over observations, in input order, in double precision:
 *   ray p, depth scalar lambda, residual e ........ Sec. III (eq. ray,
 *                                                   eq. lambdaij, eq. error)
 *   objective F = sum 1/2 rho(|e|^2) .............. Problem 1 (eq. Fij, Fobj)
 *   weights w, a, centre g, majorizers P, Q ........ Prop. 1 (eq. P, Q, a, w,
 *                                                   gamma, g)
 *   surrogate E^alpha with proximal term ........... eq. Ealpha
 *   Nesterov scalars and extrapolation ............. Sec. V (eq. nesterov_*)
 *   rotation projection onto SO(3) ................. eq. proj_rot3d
 *   surrogate gap and restart metrics .............. eq. DEalpha, Fainit, Fak,
 *                                                   lFak, Eak; Algorithm 1
 *   Euclidean gradient of F ........................ App. D, eq. DFij (the
 *                                                   intrinsics row corrected)
 *
 * Readings where the paper is silent (all observations majorized, camera
 * partitions as the devices for the restart bookkeeping, the per-camera
 * Levenberg-Marquardt specification, loss widths, units) are listed at the
 * top of oracle.c.
 *
 * All functions return 0 on success and a negative code on failure.
 */
#ifndef DABA_ORACLE_H
#define DABA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LOSS_TRIVIAL = 0, ORC_LOSS_HUBER = 1, ORC_LOSS_WELSCH = 2 };
enum { ORC_NEVER_RESTART = 1, ORC_ALWAYS_RESTART = 2 };

typedef struct orc_state orc_state;

/* Problem in caller units (pixels).  cameras [M*15] = R row-major | t | d with
 * d = (f, f*k1, f*k2); landmarks [N*3]; uv [K*2] pixels from the image
 * centre.  cam_part / lm_part may be NULL (contiguous camera blocks of
 * ceil(M/S); a landmark goes with the lowest camera id observing it).
 * unit_scale s: internal units are pixels / s.  delta is the loss width in
 * pixels, xi is in internal units.  frozen_partition >= 0 holds that
 * partition's variables fixed (a stalled device); -1 for none. */
int orc_create(int64_t M, int64_t N, int64_t K, const int32_t *obs_cam,
               const int32_t *obs_lm, const double *uv, const double *cameras,
               const double *landmarks, int S, const int32_t *cam_part,
               const int32_t *lm_part, double unit_scale, int loss, double delta,
               double xi, double eta, int accelerate, int inner_steps,
               uint64_t flags, int frozen_partition, orc_state **out);
void orc_destroy(orc_state *st);

/* n iterations of Algorithm 1.  F_trace[i] = F after iteration i (pixels^2);
 * metrics_trace[i*S*4 + a*4 + .] = (F^a(k), Fbar^a(k), E^a(k+1), restarted)
 * of iteration k; both may be NULL. */
int orc_iterate(orc_state *st, int n, double *F_trace, double *metrics_trace);

/* F at (cameras, landmarks) (caller units; NULL = current iterate). */
int orc_objective(orc_state *st, const double *cameras, const double *landmarks,
                  const double *uv, double *F_out);

/* Euclidean gradient of F (caller units) w.r.t. cameras [M*15], landmarks
 * [N*3] and pixels [K*2]; NULL inputs = current iterate / stored pixels. */
int orc_grad(orc_state *st, const double *cameras, const double *landmarks,
             const double *uv, double *g_cams, double *g_lms, double *g_uv);

/* State at the start of the next iteration k: x^k, x^(k-1) (caller units),
 * per partition (Fbar^a(k-1), E^a(k), E^a(x^k | x^(k-1)), F^a(k-1)), and
 * scalars (s^(k), k).  Any pointer may be NULL. */
int orc_get_state(const orc_state *st, double *cams, double *lms, double *cams_prev,
                  double *lms_prev, double *part4, double *scalars2);
int orc_set_state(orc_state *st, const double *cams, const double *lms,
                  const double *cams_prev, const double *lms_prev, const double *part4,
                  const double *scalars2);

/* Steps 1-2 of the next iteration without taking it (a probe of Sec. V):
 * gamma^a(k) per partition [S] (eq. nesterov_scalar) and the extrapolated
 * point x-bar^(k) of eq. nesterov_x (cameras [M*15] in caller units,
 * landmarks [N*3]).  The state is not changed.  Any pointer may be NULL. */
int orc_extrapolation(const orc_state *st, double *gamma_out, double *cams_bar, double *lms_bar);

/* Per-partition E^a(x | y) and DeltaE^a(x | y) (pixels^2) by direct sums;
 * x and y in caller units; out arrays [S]. */
int orc_surrogate(orc_state *st, const double *cams_x, const double *lms_x,
                  const double *cams_y, const double *lms_y, double *E_out,
                  double *dE_out);

/* Quantities of one observation at camera c[15], landmark l[3], pixel u[2]
 * in internal units: out = p[3], lambda, e[3], |e|^2, rho, w, a, g[3], F_ij. */
int orc_obs_eval(const orc_state *st, const double *c, const double *l, const double *u,
                 double *out16);

/* Majorizer pieces of one observation (internal units): P_ij(c | y) and
 * Q_ij(l | y) with the frozen quantities taken at (cy, ly). */
int orc_PQ(const orc_state *st, const double *u, const double *cy, const double *ly,
           const double *c, const double *l, double *P, double *Q);

/* Minimizers of one entity's share of E(. | y) (internal units):
 * landmark j closed form; camera i by the Levenberg-Marquardt specification.
 * y is given as full camera / landmark arrays in internal units. */
int orc_landmark_min(const orc_state *st, int64_t j, const double *cams_y,
                     const double *lms_y, double *l_out);
int orc_camera_min(const orc_state *st, int64_t i, const double *cams_y,
                   const double *lms_y, int inner_steps, double *c_out, int *n_success);
/* One camera's surrogate Phi_i(c | y) = sum_j P_ij(c | y) + prox (internal). */
int orc_camera_phi(const orc_state *st, int64_t i, const double *cams_y,
                   const double *lms_y, const double *c, double *phi);
int orc_landmark_phi(const orc_state *st, int64_t j, const double *cams_y,
                     const double *lms_y, const double *l, double *phi);

/* argmin over SO(3) of |R - M|_F (row-major 3x3), via an SVD built from a
 * cyclic Jacobi eigen-decomposition of M^T M. */
int orc_projrot3d(const double *M, double *R);

/* Internal <-> caller unit conversion of a camera array [M*15]. */
int orc_cams_to_internal(const orc_state *st, const double *in, double *out, int64_t M);

/* Threads of the OpenMP loops over entities: the current count, and a new
 * one (n < 1: one per processor).  The arithmetic and its order do not
 * depend on the count. */
int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
