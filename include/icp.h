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
/* robust loss of icp_register_robust / icp_normal_equations_robust */
#define ICP_LOSS_NONE 0
#define ICP_LOSS_HUBER 1
#define ICP_LOSS_TUKEY 2
#define ICP_LOSS_CAUCHY 3

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
 * owns its device workspace:
 *   arena_bytes == 0: buffers grow on demand (hipMalloc inside the calls that
 *                     need more than before) and are reused across calls;
 *   arena_bytes > 0:  one device allocation of arena_bytes now, and pinned
 *                     host staging of arena_bytes / 256 (at least 16 MiB, at
 *                     most 256 MiB); every call carves its buffers from
 *                     them afresh and allocates nothing, and a call that
 *                     does not fit returns ICP_E_OOM (the context stays
 *                     usable).  A 2M/2M point-to-plane registration needs
 *                     about 0.5 GB.
 * A context serves one call at a time: calls on one context from several
 * threads must be serialised by the caller (use one context per thread).
 * *out receives the handle.  Errors: INVALID_ARG (out NULL, bad device),
 * OOM (arena), DEVICE. */
int icp_ctx_create(int device, void *hip_stream, size_t arena_bytes, icp_ctx_t **out);

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

/* ---- robust variants -----------------------------------------------------
 * The paper's ICP module offers "other ICP variants" beside point-to-point and
 * point-to-plane (Sec. 3.3) without naming them; these are robust
 * (iteratively reweighted least squares) versions of both.  Each inlier's
 * terms of J^T J and J^T r are multiplied by w = rho'(s) / s at its residual
 * magnitude s at the current pose (|n . (q - p)| point-to-plane, |q - p|
 * point-to-point), so each Gauss-Newton step minimises the weighted squares
 * whose gradient is that of sum rho(s):
 *   ICP_LOSS_HUBER   w = 1 for s <= k, k / s beyond
 *   ICP_LOSS_TUKEY   w = (1 - (s/k)^2)^2 for s <= k, 0 beyond
 *   ICP_LOSS_CAUCHY  w = 1 / (1 + (s/k)^2)
 * The weight is computed in the precision of the terms (float32 in
 * ICP_PREC_F32_KAHAN_F64, float64 in ICP_PREC_F64).  Correspondences, inlier
 * gating by max_corr_dist, fitness, inlier_rmse (unweighted) and the stopping
 * rules are those of icp_register; ICP_LOSS_NONE gives icp_register exactly.
 *   loss    ICP_LOSS_*
 *   loss_k  scale k (metres): finite, > 0, also as float32 (ignored for NONE)
 * Other arguments, outputs and errors as icp_register / icp_normal_equations. */
int icp_register_robust(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const float *tgt_xyz,
                        const float *tgt_normals, int64_t n_tgt, const double T_init[16],
                        double max_corr_dist, int32_t max_iter, double rel_tol, int32_t variant,
                        int32_t precision, int32_t loss, double loss_k, icp_result_t *out);

int icp_normal_equations_robust(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src,
                                const double T[16], const float *tgt_xyz, const float *tgt_normals,
                                int64_t n_tgt, double max_corr_dist, int32_t variant,
                                int32_t precision, int32_t loss, double loss_k, double AtA21[21],
                                double Atb6[6], double *sum_d2, int64_t *n_in);

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
/* icp_register_batch with one robust loss for every pair (the IRLS weights of
 * icp_register_robust); a pair's result equals icp_register_robust's for it
 * alone, bitwise.  Errors: as icp_register_batch, INVALID_ARG for the loss. */
int icp_register_batch_robust(icp_ctx_t *ctx, const icp_pair_t *pairs, int32_t n_pairs, int32_t variant,
                              int32_t precision, int32_t loss, double loss_k, icp_result_t *out);

int icp_register_batch(icp_ctx_t *ctx, const icp_pair_t *pairs, int32_t n_pairs, int32_t variant,
                       int32_t precision, icp_result_t *out);

/* ---- voxel downsampling and multi-scale registration --------------------
 * Voxel downsampling (Sec. 3.3, voxel_down_sample before registration): the
 * cloud's box minimum o and the voxel edge v define voxel indices
 * floor((p - o) / v) per axis (float64); each occupied voxel yields the mean
 * of its points (float64 sum in original-index order, rounded to float32)
 * and, with normals, the normalised float64 sum of its points' normals (the
 * first point's normal if that sum is shorter than 1e-12).  Outputs are in
 * voxel-key order (x fastest, then y, then z). */

/* Downsamples one device cloud.
 *   pts, normals  device (n, 3) float32; normals may be NULL
 *   voxel         finite, > 0 (metres)
 *   out_pts, out_normals  device (cap, 3) float32 (out_normals required iff
 *                 normals given); cap = n always suffices
 *   n_out         host: number of occupied voxels
 * Errors: INVALID_ARG, NONFINITE, TOO_LARGE (more than 2^48 voxels in the box,
 * or cap < *n_out: then *n_out is set and no output beyond cap is written),
 * OOM, DEVICE. */
int icp_voxel_downsample(icp_ctx_t *ctx, const float *pts, const float *normals, int64_t n,
                         double voxel, float *out_pts, float *out_normals, int64_t cap,
                         int64_t *n_out);

/* ---- normal estimation ----------------------------------------------------
 * Normals of a point cloud with the hybrid neighbourhood that the paper's
 * workflow passes to estimate_normals (Sec. 3.2 Fig. 1 and Sec. 3.3: a search
 * radius and a maximum neighbour count), by the least-variance direction of
 * [16].  Point i's neighbourhood is the max_nn smallest (d2, original index)
 * among the points j, i included, with d2 <= (float)(radius^2), where d2 is
 * the float32 expression (dx*dx + dy*dy) + dz*dz of d = p_i - p_j (no FMA).
 * The normal is the unit eigenvector of the smallest eigenvalue of the
 * neighbourhood's float64 covariance (about its mean, divided by the count),
 * rounded to float32 and turned so that n . (viewpoint - p_i) >= 0.  Fewer than
 * three neighbours give (0, 0, 0); when the smallest eigenvalue is repeated
 * (collinear or isotropic neighbourhoods) any unit vector of its eigenspace
 * may be returned.
 *   pts          device (n, 3) float32, 4-byte aligned
 *   radius       finite, > 0, with a finite float32 square (metres)
 *   max_nn       1 .. 64
 *   viewpoint    host, 3 finite doubles
 *   normals_out  device (n, 3) float32, in the order of pts (caller-owned)
 *   counts_out   device (n) int32 neighbourhood sizes, or NULL
 * Synchronous on the context's stream.  Errors: INVALID_ARG, NONFINITE (a
 * coordinate), TOO_LARGE, OOM, DEVICE; nothing is written on argument errors. */
int icp_estimate_normals(icp_ctx_t *ctx, const float *pts, int64_t n, double radius, int32_t max_nn,
                         const double viewpoint[3], float *normals_out, int32_t *counts_out);

/* Coarse-to-fine registration (as in the fragment registration stage of the
 * reconstruction pipeline, Sec. 3.4): for each level l, both clouds are
 * downsampled with voxel[l] (0: the original clouds), then registered with
 * max_corr_dist[l] and max_iter[l] starting from the previous level's pose.
 * A DEGENERATE level ends the call.  `out` is the last level's result with
 * n_iter = the total number of pose updates.  n_levels in [1, 16]; arrays are
 * host memory.  Errors as icp_register / icp_voxel_downsample. */
/* icp_register_multiscale with a robust loss at every level (the IRLS
 * weights of icp_register_robust).  Errors: as icp_register_multiscale,
 * INVALID_ARG for the loss. */
int icp_register_multiscale_robust(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const float *tgt_xyz,
                                   const float *tgt_normals, int64_t n_tgt, const double T_init[16],
                                   int32_t n_levels, const double *voxel, const int32_t *max_iter,
                                   const double *max_corr_dist, double rel_tol, int32_t variant,
                                   int32_t precision, int32_t loss, double loss_k, icp_result_t *out);

int icp_register_multiscale(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const float *tgt_xyz,
                            const float *tgt_normals, int64_t n_tgt, const double T_init[16],
                            int32_t n_levels, const double *voxel, const int32_t *max_iter,
                            const double *max_corr_dist, double rel_tol, int32_t variant,
                            int32_t precision, icp_result_t *out);

/* ---- multiway registration: pose-graph optimisation ---------------------
 * Multiway registration (Sec. 3.3) by pose-graph optimisation with
 * Gauss-Newton or Levenberg-Marquardt (the in-house solvers of Sec. 2).  Node
 * k has pose T_k (node frame -> world, row-major 4x4); edge (i, j) holds a
 * measured relative pose Z ~ T_i^-1 T_j (e.g. an icp_register result that maps
 * fragment j onto fragment i) and a symmetric positive semi-definite 6x6
 * information matrix (row-major, twist order (omega, v)).  The residual is
 * e = Log(Z^-1 T_i^-1 T_j), the objective F = sum e^T information e.  Node 0
 * stays fixed; the others move by left perturbations T <- Exp(d) T with the
 * edge Jacobians +-Ad(T_j^-1) (exact where e = 0, so consistent graphs are
 * recovered exactly).  Gauss-Newton solves H d = -g; Levenberg-Marquardt
 * solves (H + lambda diag H) d = -g, lambda starting at 1e-4, keeps a step
 * that lowers F (lambda / 10) and otherwise refuses it (lambda * 10).  The run
 * stops after max_iter kept steps (ICP_OK), when a kept step changes F by at
 * most rel_tol * F or after 10 refusals in a row (ICP_CONVERGED), or on a
 * Cholesky pivot <= 1e-12 max diag (ICP_DEGENERATE, poses of the last kept
 * step).  Rotation angles of the residuals must stay below pi. */
#define ICP_PG_GAUSS_NEWTON 0
#define ICP_PG_LEVENBERG_MARQUARDT 1

typedef struct {
  int32_t i, j;           /* node indices, 0 <= i, j < n_nodes, i != j */
  double Z[16];           /* row-major rigid transform, ~ T_i^-1 T_j */
  double information[36]; /* row-major 6x6 */
} icp_pose_edge_t;

typedef struct {
  double F_initial;  /* objective at the given poses */
  double F_final;    /* objective at the returned poses */
  int32_t steps;     /* kept steps */
  int32_t status;    /* ICP_OK, ICP_CONVERGED or ICP_DEGENERATE */
} icp_pose_graph_result_t;

/* Optimises the poses in place.
 *   n_nodes  2 .. 256
 *   poses    host (n_nodes, 16) float64, finite rigid transforms; overwritten
 *   edges    host array of n_edges >= 1 edges
 *   method   ICP_PG_GAUSS_NEWTON or ICP_PG_LEVENBERG_MARQUARDT
 *   max_iter >= 0; rel_tol finite, >= 0
 *   out      host result
 * Synchronous on the context's stream.  Errors: INVALID_ARG (bad sizes,
 * indices, non-finite or non-rigid transforms, non-finite information, an
 * information matrix that is not exactly symmetric), OOM, DEVICE; on errors
 * the poses are untouched. */
int icp_pose_graph_optimize(icp_ctx_t *ctx, int32_t n_nodes, double *poses, int32_t n_edges,
                            const icp_pose_edge_t *edges, int32_t method, int32_t max_iter,
                            double rel_tol, icp_pose_graph_result_t *out);

/* ---- global registration: RANSAC on feature matches ---------------------
 * The global step of the pairwise workflow (Sec. 3.3, the RANSAC-based
 * registration on feature matches [17] that supplies ICP's initial pose, with
 * the point-to-point estimate, the edge-length and distance correspondence
 * checkers and the (max_iteration, max_validation) criterion; validating a
 * hypothesis dominates its cost).  Definitions:
 *   feature match  c(i) = argmin_j (D_ij, j), D_ij the float32 squared
 *                  feature distance summed over the dimensions in index
 *                  order without FMA (ties: smallest j);
 *   hypothesis h   ransac_n source indices from Philox4x64-10 (Salmon et al.,
 *                  SC'11), block b = Philox(counter (h, b, 0, 0), key (seed,
 *                  0)), draw k = word k % 4 of block k / 4 mapped to [0, n_src)
 *                  by ((z >> 32) * n_src) >> 32; the pairs (i, corr[i]);
 *                  rejected if an index repeats or corr[i] is outside
 *                  [0, n_tgt);
 *   edge length    for every two pairs a, b: ds2 >= sigma^2 dt2 and
 *                  dt2 >= sigma^2 ds2 (squared lengths in float64);
 *   fit            the rigid transform (no scale) minimising the sampled
 *                  pairs' squared distances;
 *   distance       every sampled pair within d under the fit (float64);
 *   validation     every source point matched to its nearest target point
 *                  under T by the same rule as icp_correspondences; score
 *                  (count, sumq), sumq = sum over inliers of
 *                  floor(d2 * 2^shift), shift = 40 - e with
 *                  fl32(max_corr_dist^2) = m 2^e, m in [0.5, 1): an exact
 *                  integer;
 *   selection      the first max_validation hypotheses (in h order) that
 *                  pass both checkers are validated; the loop ends there or
 *                  after max_iteration hypotheses; the best is the
 *                  lexicographic minimum of (-count, sumq, h). */
#define ICP_RANSAC_NO_HYPOTHESIS 3  /* no hypothesis passed the checkers; T = identity */

typedef struct {
  double max_corr_dist;    /* validation radius r > 0 */
  double edge_length;      /* edge-length similarity sigma (paper: 0.9); <= 0: checker off */
  double distance;         /* distance checker threshold d (paper: = r); <= 0: checker off */
  int64_t max_iteration;   /* >= 1 hypotheses at most */
  int32_t max_validation;  /* 1 .. 65535 validated hypotheses at most */
  int32_t ransac_n;        /* 3 .. 8 pairs per hypothesis */
  uint64_t seed;           /* Philox key word 0 */
} icp_ransac_params_t;

typedef struct {
  double T[16];             /* row-major transform of the best hypothesis (source -> target) */
  double fitness;           /* n_inliers / n_src */
  double inlier_rmse;       /* sqrt(sumq 2^-shift / n_inliers) */
  int64_t n_inliers;
  uint64_t sumq;            /* the best score's fixed-point sum */
  int32_t shift;
  int32_t status;           /* ICP_OK or ICP_RANSAC_NO_HYPOTHESIS */
  int64_t n_iterations;     /* hypotheses consumed: (h of the max_validation-th validated) + 1, else max_iteration */
  int64_t n_validated;
  int64_t best_hypothesis;  /* h of the best, -1 if none */
} icp_ransac_result_t;

/* Optional per-hypothesis outputs of icp_ransac_register: device arrays with
 * room for max_validation entries (any may be NULL), in validation order. */
typedef struct {
  int64_t *h;       /* hypothesis indices */
  double *T;        /* (16) row-major transforms */
  int64_t *count;   /* inlier counts */
  uint64_t *sumq;   /* fixed-point sums */
} icp_ransac_trace_t;

/* FPFH descriptors (Sec. 3.3, compute_fpfh_feature with a hybrid (radius,
 * max_nn) neighbourhood; the Fast Point Feature Histogram of [17]).  The
 * neighbourhood of point i is the normal estimation's: the max_nn smallest
 * (pinned float32 squared distance, index) within radius, i included.  For a
 * neighbour j != i at non-zero distance, in float64 from the float32 inputs:
 * the source s is the end whose normal makes the smaller angle with the line
 * to the other (s = i iff n_i . (p_j - p_i) >= -n_j . (p_j - p_i)), e the
 * unit line from s, u = n_s, v = unit(u x e) (pair skipped if u x e = 0),
 * w = u x v; alpha = v . n_t, phi = u . e, theta = atan2(w . n_t, u . n_t);
 * bins floor((alpha + 1) 5.5), 11 + floor((phi + 1) 5.5),
 * 22 + floor((theta + pi) 11 / (2 pi)), each sub-bin clamped to [0, 10].
 * SPFH(i) = bin counts * 100 / k_i (k_i pairs counted; zero if none);
 * FPFH(i) = SPFH(i) + (1 / k') sum over those neighbours of SPFH(j) / |p_j - p_i|
 * (k' their number), rounded to float32.
 *   pts, normals  device (n, 3) float32; normals unit length (not checked)
 *   radius > 0; max_nn 1 .. 128
 *   features_out  device (n, 33) float32 (caller-owned)
 *   nn_out        device (n) int32 neighbourhood sizes (i included), or NULL
 * Synchronous.  Errors: INVALID_ARG, NONFINITE (a coordinate), TOO_LARGE, OOM,
 * DEVICE. */
int icp_compute_fpfh(icp_ctx_t *ctx, const float *pts, const float *normals, int64_t n, double radius,
                     int32_t max_nn, float *features_out, int32_t *nn_out);

/* Nearest-feature matching (row-major float32 features, device memory).
 *   src_feat  (n_src, dim), tgt_feat (n_tgt, dim); n_src, n_tgt >= 0;
 *             dim 1 .. 64; features must be finite (not checked)
 *   match_out device (n_src) int32: c(i), -1 if n_tgt = 0
 *   dist_out  device (n_src) float32 D_i(c(i)), or NULL
 * Synchronous.  Errors: INVALID_ARG, TOO_LARGE, OOM, DEVICE. */
int icp_feature_match(icp_ctx_t *ctx, const float *src_feat, int64_t n_src, const float *tgt_feat,
                      int64_t n_tgt, int32_t dim, int32_t *match_out, float *dist_out);

/* icp_feature_match without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * icp_feature_match, with the context replaced by a stream:
 *   hip_stream  hipStream_t the kernels are enqueued on (NULL: the null
 *               stream) on the calling thread's current device
 * The call is asynchronous: it only enqueues kernels (no allocation, no
 * memset, no synchronisation), and match_out / dist_out are complete when
 * that stream's work is.  Its scratch (one 64-bit key per source feature) is
 * a static device array of 2^20 keys (8 MiB) that each device holds for the
 * life of the process: n_src > 2^20 gives ICP_E_TOO_LARGE.  Every call on a
 * device shares that array, so calls that may overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.  The
 * first call on a device looks the array's address up (hipGetSymbolAddress).
 * Errors: INVALID_ARG, TOO_LARGE, DEVICE. */
int icp_feature_match_noalloc(const float *src_feat, int64_t n_src, const float *tgt_feat, int64_t n_tgt,
                              int32_t dim, int32_t *match_out, float *dist_out, void *hip_stream);

/* Scores n_hyp given transforms (the validation step).
 *   src_xyz, tgt_xyz  device (n, 3) float32; 1 <= n_src <= 2^23
 *   T                 host (n_hyp, 16) rigid transforms, n_hyp 1 .. 65535
 *   count_out, sumq_out  host (n_hyp)
 * Synchronous.  Errors: INVALID_ARG, NONFINITE, TOO_LARGE, OOM, DEVICE. */
int icp_ransac_validate(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const float *tgt_xyz,
                        int64_t n_tgt, double max_corr_dist, int32_t n_hyp, const double *T,
                        int64_t *count_out, uint64_t *sumq_out);

/* RANSAC registration of src onto tgt from putative pairs (i, corr[i]).
 *   src_xyz, tgt_xyz  device (n, 3) float32 in original order; n_src <= 2^23
 *   corr              device (n_src) int32 target index per source point
 *                     (e.g. icp_feature_match's output; values outside
 *                     [0, n_tgt) mark a point without a match)
 *   prm, out          host; trace: optional device outputs, or NULL
 * Synchronous (one readback per chunk of hypotheses).  The context's device
 * workspace grows to about 100 B per hypothesis of the largest chunk (at
 * most 2^21 hypotheses, ~210 MB) plus the validation partials.  Run time
 * grows with max_iteration when few hypotheses pass the checkers.  Errors:
 * INVALID_ARG, NONFINITE, TOO_LARGE, OOM, DEVICE. */
int icp_ransac_register(icp_ctx_t *ctx, const float *src_xyz, int64_t n_src, const float *tgt_xyz,
                        int64_t n_tgt, const int32_t *corr, const icp_ransac_params_t *prm,
                        icp_ransac_result_t *out, const icp_ransac_trace_t *trace);

/* ---- served form: continuous batching of registration requests ----------
 * Requests (pairs of clouds, as produced one by one by a reconstruction
 * pipeline's fragment registration stage, Sec. 3.4) are submitted at any
 * time.  The server copies each request's inputs into its own device memory,
 * admits requests FIFO while registration slots are free and its device
 * memory budget allows, and advances every admitted request through a
 * coarse-to-fine schedule (voxel downsampling then ICP per level, as
 * icp_register_multiscale).  One server step runs `iters_per_step`
 * iterations of all running requests together (one HIP graph replay: per
 * iteration one batched pass launch over every running request's tiles and
 * one batched solve launch), then retires finished levels and requests.  A request's result is bitwise the
 * one icp_register_multiscale (icp_register_multiscale_robust with a loss)
 * gives for it alone.
 * Level l of a request uses max_corr_dist = corr_dist[l] if > 0, else
 * corr_factor * max(voxel[l], spacing) with the request's target spacing. */
typedef struct icp_server icp_server_t;

typedef struct {
  int32_t device;
  int32_t max_slots;          /* requests registered concurrently, >= 1 */
  uint64_t hbm_budget_bytes;  /* device memory for inputs and working data of all requests */
  int32_t n_levels;           /* 1..4 */
  int32_t iters[4];           /* max_iter per level */
  double voxel[4];            /* voxel edge per level (0: original clouds) */
  double corr_dist[4];        /* > 0: fixed max_corr_dist per level */
  double corr_factor;         /* rule factor for levels without corr_dist (e.g. 2) */
  int32_t variant;            /* ICP_POINT_TO_PLANE / ICP_POINT_TO_POINT */
  int32_t precision;          /* ICP_PREC_* */
  int32_t iters_per_step;     /* iterations per server step, 1..64 */
  int32_t background_thread;  /* 1: a server thread runs steps; 0: caller drives icp_server_step */
  int32_t loss;               /* ICP_LOSS_* for every request (0: plain ICP) */
  double loss_k;              /* its scale (ignored for ICP_LOSS_NONE) */
} icp_server_cfg_t;

typedef struct {
  const float *src_xyz;       /* (n_src, 3) float32, device or host (host_memory) */
  const float *tgt_xyz;       /* (n_tgt, 3) */
  const float *tgt_normals;   /* (n_tgt, 3); required for point-to-plane */
  int64_t n_src;
  int64_t n_tgt;
  double T_init[16];          /* host, row-major */
  double rel_tol;             /* >= 0, per level */
  double spacing;             /* mean target point spacing (m), 0 if unknown */
  int32_t host_memory;        /* 1: the three arrays are host memory */
  int32_t reserved;           /* must be 0 */
  uint64_t user_tag;
  void *stream;               /* device inputs: the hipStream_t whose work so far
                                 produces them (the copy waits for it), or NULL
                                 when they are already complete */
} icp_request_t;

typedef struct {
  uint64_t ticket;
  uint64_t user_tag;
  icp_result_t result;        /* valid when error == 0; n_iter = total pose updates */
  int32_t error;              /* 0 or a negative ICP_E_* code */
  int32_t reserved;
  int64_t t_submit_ns;        /* CLOCK_MONOTONIC, at icp_server_submit entry */
  int64_t t_admit_ns;         /* when a slot was assigned */
  int64_t t_done_ns;          /* when the result was posted */
} icp_completion_t;

/* Creates a server (its own context, stream, device memory pool of
 * hbm_budget_bytes, slot table and step graph).  Errors: INVALID_ARG, OOM,
 * DEVICE. */
int icp_server_create(const icp_server_cfg_t *cfg, icp_server_t **out);

/* Copies the request's inputs (device-to-device or host-to-device) into
 * server memory before returning -- the caller may free its buffers at once
 * -- and queues it.  The copy runs on the server's own stream: device inputs
 * still being written by queued work must name that work's stream in
 * req->stream (the copy is ordered after everything enqueued on it before
 * this call); with stream NULL they must be complete.  *ticket identifies the
 * completion.  Thread-safe.
 * Errors: INVALID_ARG, TOO_LARGE (inputs alone exceed the budget), DEVICE
 * (also once the server has stopped after a device error). */
int icp_server_submit(icp_server_t *srv, const icp_request_t *req, uint64_t *ticket);

/* Caller-driven mode: one server step (admission, level preparation,
 * iters_per_step iterations, retirement).  *n_busy (optional) receives the
 * number of queued + running requests after the step.  With a background
 * thread this is a no-op.  Errors: DEVICE.  After a failed step (here or on
 * the background thread) the server is stopped: every queued and running
 * request completes at once with error ICP_E_DEVICE, and later submits and
 * steps return ICP_E_DEVICE; only poll, wait (for the completions already
 * posted) and destroy remain useful. */
int icp_server_step(icp_server_t *srv, int32_t *n_busy);

/* Moves up to cap finished requests' completions to out (host), in
 * completion order; *n_out receives the count.  Non-blocking.  Thread-safe. */
int icp_server_poll(icp_server_t *srv, icp_completion_t *out, int32_t cap, int32_t *n_out);

/* Blocks until `ticket` has completed and moves its completion to *out (in
 * caller-driven mode it runs steps itself).  A request of a stopped server
 * is delivered with error ICP_E_DEVICE.  Errors: NOT_FOUND (unknown or
 * already delivered ticket), DEVICE (a step it ran failed). */
int icp_server_wait(icp_server_t *srv, uint64_t ticket, icp_completion_t *out);

/* Stops the server: requests not yet completed are completed with
 * ICP_E_CANCELLED (and dropped), all device memory is released.  NULL is a
 * no-op. */
int icp_server_destroy(icp_server_t *srv);

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
  double validate_ms;        /* RANSAC validation launches (pass and per-hypothesis sum) */
  int64_t validate_launches;
  int64_t validate_evals;    /* hypotheses x source points scored */
  double build_ms;           /* grid and source-order builds of registration calls */
  int64_t builds;
  int64_t build_points;      /* target points built (summed over the calls' pairs) */
  int64_t hashed_grids;      /* pairs whose target grid got a hashed cell table */
  int64_t fine_grids;        /* pairs whose grid took two cells per radius */
} icp_profile_t;

/* Enables (1) or disables (0) kernel timing on ctx; resets the counters.
 * Errors: INVALID_ARG (ctx NULL), DEVICE. */
int icp_ctx_set_profiling(icp_ctx_t *ctx, int enable);

/* Copies the accumulated counters to *out (host).  Errors: INVALID_ARG. */
int icp_ctx_get_profile(icp_ctx_t *ctx, icp_profile_t *out);

/* ---- device ceilings (measurement support) ------------------------------
 * Not part of the method: these run small dedicated kernels on `device` and
 * return the rates that the library's kernels are compared against, taken on
 * the same device in the same process.  Each allocates and frees its own
 * buffers and stream, and blocks until done.
 *
 * icp_measure_valu: issue rate of unpacked vector arithmetic, in lane
 * operations per second (one operation per lane per instruction), over
 * 8 waves per SIMD of 8 independent dependency chains each.
 *   kind 0  v_mul_f32 / v_add_f32 alternating
 *   kind 1  v_fma_f32
 *   kind 2  v_mul_f64 / v_add_f64 alternating
 *   kind 3  v_fma_f64
 *   kind 4  v_sub_f32 / v_mul_f32 / v_add_f32 of a 36-dimensional squared
 *           distance, two queries against a target in scalar registers (many
 *           independent instructions per wave: the highest unpacked rate)
 * *best_ms (may be NULL) receives the fastest of five timed launches.
 * Errors: INVALID_ARG (kind outside 0..4, lane_ops_per_s NULL), DEVICE. */
int icp_measure_valu(int device, int kind, double *lane_ops_per_s, double *best_ms);

/* icp_measure_copy: streaming bandwidth of device memory over a buffer of
 * `bytes` (>= 1 MiB; choose it above the 256 MiB last-level cache to measure
 * HBM).  kind 0: copy (read + write bytes counted), kind 1: read only (a
 * per-thread sum is written, negligible).  *gb_per_s is bytes moved / fastest
 * of five launches, in 1e9 B/s.  Errors: INVALID_ARG, OOM/DEVICE. */
int icp_measure_copy(int device, int64_t bytes, int kind, double *gb_per_s, double *best_ms);

#ifdef __cplusplus
}
#endif

#endif /* ICP_H */
