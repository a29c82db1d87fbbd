/*
 * icp.h -- C ABI of the MI355X ICP registration library (libicp.so).
 *
 * Method (Open3D paper, Sec. 3.3 "Registration"): ICP refinement of a source
 * cloud onto a target cloud from an initial transform, keeping only pairs
 * closer than a maximum correspondence distance, with the point-to-plane or
 * point-to-point error [2, 4].  Each iteration is one Gauss-Newton step
 * x <- x - (J^T J)^{-1} J^T r on L(x) = sum_i r_i(x)^2 (Sec. 4, eqs. (1)-(2)),
 * with J^T J and J^T r formed as a parallel reduction over per-correspondence
 * contributions (Sec. 4, the reduction over a per-record function).
 *
 * Conventions shared by every entry point
 *   - Point clouds are row-major (N, 3) float32 arrays in DEVICE memory
 *     (x0 y0 z0 x1 y1 z1 ...), 4-byte aligned.  The library never retains a
 *     caller pointer after a call returns.
 *   - Transforms are row-major 4x4 float64 matrices in HOST memory mapping
 *     source coordinates to target coordinates (q = R s + t).  The last row
 *     must be (0, 0, 0, 1) and |R^T R - I| <= 1e-6 (max-abs).
 *   - Update: xi = (omega, v), rotation first, applied as a left perturbation
 *     T <- Exp(xi) T; xi solves (J^T J) xi = -J^T r (eq. (2)), no damping.
 *   - Correspondence: for each source point s, q = T s is evaluated in FP64
 *     without FMA as ((R_a0 sx + R_a1 sy) + R_a2 sz) + t_a and rounded to
 *     float32; the squared distance to a target p is
 *     (dx*dx + dy*dy) + dz*dz in float32 without FMA.  The match is the target
 *     with the smallest (distance, original index) pair among those with
 *     distance <= (float)(max_corr_dist^2).  Source -> target only.
 *   - Residuals: point-to-plane r = n . (q - p), J = [(q x n)^T, n^T];
 *     point-to-point r = q - p, J = [-[q]_x, I].
 *   - Pass k = 0..max_iter evaluates correspondences at T_k.  The loop stops
 *     with ICP_DEGENERATE when pass k has no inliers or a Cholesky pivot of
 *     J^T J is <= 1e-12 max(diag); with ICP_OK at k == max_iter; with
 *     ICP_CONVERGED when k >= 1 and both |n_k - n_{k-1}| <= rel_tol n_{k-1}
 *     and |rmse_k - rmse_{k-1}| <= rel_tol rmse_{k-1}.  Results are those of
 *     the last pass: fitness = n_k / n_src, inlier_rmse = sqrt(sum d^2 / n_k)
 *     (0 when n_k = 0), T = T_k.
 *   - Precision ICP_PREC_F32_KAHAN_F64: per-point residuals and Jacobian
 *     products in float32, partial sums with Kahan compensation in float32,
 *     cross-block reduction, solve and pose update in float64.
 *     ICP_PREC_F64: per-point terms and all sums in float64.
 *   - Return value: ICP_SUCCESS (0) or a negative ICP_E_* code; on error the
 *     outputs are untouched and icp_last_error() (thread-local) describes it.
 *     Arguments are validated on the host before any device work.
 *   - Calls on one context are serialised by the caller; a context is bound
 *     to one device and one HIP stream.  Plain and batched calls block until
 *     their (host) outputs are written.
 */
#ifndef ICP_H
#define ICP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define ICP_SUCCESS 0
#define ICP_E_INVALID_ARG (-1) /* null pointer, n < 1, bad r / max_iter / rel_tol / T, ... */
#define ICP_E_NONFINITE (-2)   /* NaN or Inf in a coordinate or normal (found on device) */
#define ICP_E_TOO_LARGE (-3)   /* N > 2^31 - 1, or a request larger than the budget */
#define ICP_E_OOM (-4)         /* device allocation failed */
#define ICP_E_DEVICE (-5)      /* HIP runtime error; text in icp_last_error() */
#define ICP_E_CANCELLED (-6)   /* request dropped by icp_server_destroy */
#define ICP_E_NOT_FOUND (-7)   /* unknown ticket */

/* icp_result_t.status (not errors) */
#define ICP_OK 0          /* stopped at max_iter */
#define ICP_CONVERGED 1   /* rel_tol test met */
#define ICP_DEGENERATE 2  /* no inliers, or J^T J not positive definite; T = last pose */

/* variant */
#define ICP_POINT_TO_POINT 0
#define ICP_POINT_TO_PLANE 1
/* precision */
#define ICP_PREC_F32_KAHAN_F64 0
#define ICP_PREC_F64 1

typedef struct {
  double T[16];        /* row-major final pose (source -> target) */
  double fitness;      /* inliers / n_src at T */
  double inlier_rmse;  /* sqrt(mean squared inlier distance) at T */
  int64_t n_inliers;
  int32_t n_iter;      /* number of pose updates applied */
  int32_t status;      /* ICP_OK / ICP_CONVERGED / ICP_DEGENERATE */
} icp_result_t;

typedef struct icp_ctx icp_ctx_t;

/* Version string of the library (static storage). */
const char *icp_version(void);

/* Text for a return code (static storage). */
const char *icp_strerror(int code);

/* Description of the last error raised on the calling thread ("" if none). */
const char *icp_last_error(void);

/* Creates a context on `device` bound to `hip_stream` (a hipStream_t; NULL
 * makes the context create and own a default-priority stream).  The context
 * owns its device workspace, which grows on demand and is reused across calls.
 * *out receives the handle.  Errors: INVALID_ARG (out NULL, bad device),
 * DEVICE. */
int icp_ctx_create(int device, void *hip_stream, icp_ctx_t **out);

/* Releases the context and all device memory it owns.  NULL is a no-op. */
int icp_ctx_destroy(icp_ctx_t *ctx);

/* Registers one pair (Sec. 3.3 ICP refinement; Sec. 4 eqs. (1)-(2)).
 *   ctx          context; NULL uses a per-thread default context on the
 *                current device
 *   src_xyz      device (n_src, 3) float32 source points
 *   tgt_xyz      device (n_tgt, 3) float32 target points
 *   tgt_normals  device (n_tgt, 3) float32 target normals (used as given, not
 *                renormalised); required for point-to-plane, ignored (may be
 *                NULL) for point-to-point
 *   T_init       host row-major 4x4 float64 initial pose
 *   max_corr_dist  > 0 with (float)(max_corr_dist^2) finite (metres); inliers
 *                have distance <= it
 *   max_iter     >= 0 pose updates at most (0 evaluates T_init only)
 *   rel_tol      >= 0 convergence threshold (0: stop only at an exact fixed point)
 *   variant      ICP_POINT_TO_PLANE or ICP_POINT_TO_POINT
 *   precision    ICP_PREC_F32_KAHAN_F64 or ICP_PREC_F64
 *   out          host result
 * Errors: INVALID_ARG, NONFINITE, TOO_LARGE, OOM, DEVICE. */
int icp_register(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const float *tgt_xyz,
                 const float *tgt_normals, int64_t n_tgt, const double T_init[16],
                 double max_corr_dist, int32_t max_iter, double rel_tol, int32_t variant,
                 int32_t precision, icp_result_t *out);

/* Test hook, same kernels as icp_register: the correspondence of every source
 * point at pose T (Sec. 3.3, pairs within max_corr_dist).
 *   idx_out  device int32[n_src]: original target index of the match, -1 if none
 *   d2_out   device float32[n_src]: pinned float32 squared distance of the match,
 *            +inf if none
 * Outputs are indexed by the ORIGINAL source index.  Errors as icp_register. */
int icp_correspondences(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const double T[16],
                        const float *tgt_xyz, int64_t n_tgt, double max_corr_dist,
                        int32_t *idx_out, float *d2_out);

/* Test hook, same kernels as icp_register: the Gauss-Newton normal equations
 * at pose T (Sec. 4, the J^T J / J^T r reduction of eq. (2)).
 *   AtA21    host float64[21]: upper triangle of J^T J, row-major
 *            ((0,0),(0,1),..,(0,5),(1,1),..,(5,5))
 *   Atb6     host float64[6]: J^T r
 *   sum_d2   host: sum over inliers of the squared distance
 *   n_in     host: number of inliers
 * Errors as icp_register. */
int icp_normal_equations(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const double T[16],
                         const float *tgt_xyz, const float *tgt_normals, int64_t n_tgt,
                         double max_corr_dist, int32_t variant, int32_t precision,
                         double AtA21[21], double Atb6[6], double *sum_d2, int64_t *n_in);

/* ---- batched form -------------------------------------------------------- */
typedef struct {
  const float *src_xyz;      /* device (n_src, 3) float32 */
  const float *tgt_xyz;      /* device (n_tgt, 3) float32 */
  const float *tgt_normals;  /* device (n_tgt, 3) float32; required for point-to-plane */
  int64_t n_src;
  int64_t n_tgt;
  double T_init[16];         /* row-major initial pose */
  double max_corr_dist;      /* as icp_register */
  double rel_tol;            /* as icp_register */
  int32_t max_iter;          /* as icp_register */
  int32_t reserved;          /* must be 0 */
} icp_pair_t;

/* Registers n_pairs independent pairs together (Sec. 3.3 ICP refinement, as
 * many fragment pairs are registered in the reconstruction pipeline of
 * Sec. 3.4).  Every pair runs exactly the per-pair computation of
 * icp_register (same stopping rules, its own max_corr_dist / max_iter /
 * rel_tol), but one launch per iteration covers the source tiles of all pairs
 * still running, and one launch solves all pairs' systems.  A pair's result is
 * independent of the other pairs in the batch (bitwise).
 *   pairs  host array of n_pairs descriptors (device point pointers)
 *   out    host array of n_pairs results
 * All pairs share `variant` and `precision`.  Errors: as icp_register; on any
 * error no result is written; icp_last_error() names the offending pair. */
int icp_register_batch(icp_ctx_t *ctx, const icp_pair_t *pairs, int32_t n_pairs, int32_t variant,
                       int32_t precision, icp_result_t *out);

/* ---- kernel timing (measurement support) --------------------------------
 * With profiling enabled, every registration call on the context records a
 * pair of HIP events around each launch of the fused correspondence /
 * normal-equation kernel on the context's stream and accumulates, after the
 * call's final synchronisation, the durations of the launches that did work
 * (passes 0..n_iter; launches skipped after the stopping rule fired are not
 * counted).  Costs one event pair per pass; off by default. */
typedef struct {
  double pass_ms;          /* summed duration of counted pass-kernel launches */
  int64_t pass_launches;   /* number of counted launches */
  int64_t pass_points;     /* sum of n_src over counted launches */
  double call_ms;          /* summed duration from first to last launch of each call */
  int64_t calls;
} icp_profile_t;

/* Enables (1) or disables (0) kernel timing on ctx; resets the counters.
 * Errors: INVALID_ARG (ctx NULL), DEVICE. */
int icp_ctx_set_profiling(icp_ctx_t *ctx, int enable);

/* Copies the accumulated counters to *out (host).  Errors: INVALID_ARG. */
int icp_ctx_get_profile(icp_ctx_t *ctx, icp_profile_t *out);

#ifdef __cplusplus
}
#endif

#endif /* ICP_H */
