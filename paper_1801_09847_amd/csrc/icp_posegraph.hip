// Pose-graph optimisation (multiway registration) on gfx950.
//
// Method: Open3D paper Sec. 3.3 (multiway registration by pose-graph
// optimisation) with the in-house Gauss-Newton / Levenberg-Marquardt solvers
// of Sec. 2.  Nodes carry poses T_i (node frame -> world); an edge (i, j, Z, L)
// carries a measured relative pose Z ~ T_i^-1 T_j and a 6x6 information
// matrix L.  The residual is e = Log(Z^-1 T_i^-1 T_j) (rotation first, the
// twist order of the ICP step), the objective F = sum e^T L e; node 0 is held
// fixed and the others move by left perturbations T_k <- Exp(d_k) T_k, with
// de/dd_j = Ad(T_j^-1) and de/dd_i = -Ad(T_j^-1) (exact where e = 0).
//
// Per iteration: one thread per edge forms K = J^T L J, u = J^T L e and
// f = e^T L e in float64; the dense normal equations over the free nodes are
// assembled block by block from host-built incidence lists (fixed order, no
// atomics); F is a fixed-order reduction; the damped system is factorised by
// a right-looking blocked Cholesky (64x64 diagonal blocks factorised in
// registers by four wavefronts, each inside the trailing update before it;
// the panel solved with four lanes per row; the trailing update in 64x64
// tiles; the forward substitution rides along in the update) and solved by
// blocked backward substitution, on the context's stream, with the pivot
// rule checked on the factor; one thread per node applies the step.  The
// host keeps or refuses the step from F alone.

#include <math.h>

#include <algorithm>
#include <vector>

#include "icp_runtime.h"

#pragma clang fp contract(off)

using namespace icp;
using namespace icp_rt;

namespace {

constexpr int kTerms = 43;       // K (36), u (6), f
constexpr int kMaxPgNodes = 256;

struct PgEdge {
  int32_t i, j;
  double Z[16];
  double L[36];
};

struct PgBlock {  // one 6x6 block (a, b), a <= b, of H over the free nodes
  int32_t a, b;   // free-node indices (node - 1)
  int32_t start, count;  // contributions in the (edge, sign) list
};

__device__ inline void rigid_inverse(const double* T, double* Ti) {
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) Ti[4 * r + c] = T[4 * c + r];
    Ti[4 * r + 3] = -((T[4 * 0 + r] * T[3] + T[4 * 1 + r] * T[7]) + T[4 * 2 + r] * T[11]);
  }
  Ti[12] = 0.0; Ti[13] = 0.0; Ti[14] = 0.0; Ti[15] = 1.0;
}

__device__ inline void mul4(const double* X, const double* Y, double* Z) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = (X[4 * r] * Y[c] + X[4 * r + 1] * Y[4 + c]) + X[4 * r + 2] * Y[8 + c];
      if (c == 3) s += X[4 * r + 3];
      Z[4 * r + c] = s;
    }
  Z[12] = 0.0; Z[13] = 0.0; Z[14] = 0.0; Z[15] = 1.0;
}

// Log of a rigid transform (rotation angle below pi): omega from the
// antisymmetric part of R scaled by theta / (2 sin theta), v = V^-1 t with
// V^-1 = I - W / 2 + k W^2, k = (1 - theta sin theta / (2 (1 - cos theta))) / theta^2
// (series near 0).
__device__ inline void log_rigid(const double* E, double* e) {
  const double tr = (E[0] + E[5]) + E[10];
  const double c = fmin(fmax(0.5 * (tr - 1.0), -1.0), 1.0);
  const double th = acos(c);
  const double ax = E[9] - E[6], ay = E[2] - E[8], az = E[4] - E[1];
  double s, k;
  if (th < 1e-4) {
    s = 0.5 * (1.0 + th * th / 6.0);
    k = 1.0 / 12.0 + th * th / 720.0;
  } else {
    const double sn = sin(th);
    s = th / (2.0 * sn);
    k = (1.0 - th * sn / (2.0 * (1.0 - cos(th)))) / (th * th);
  }
  const double wx = s * ax, wy = s * ay, wz = s * az;
  const double tx = E[3], ty = E[7], tz = E[11];
  // W t and W (W t) with W = [w]_x
  const double p0 = wy * tz - wz * ty, p1 = wz * tx - wx * tz, p2 = wx * ty - wy * tx;
  const double q0 = wy * p2 - wz * p1, q1 = wz * p0 - wx * p2, q2 = wx * p1 - wy * p0;
  e[0] = wx; e[1] = wy; e[2] = wz;
  e[3] = (tx - 0.5 * p0) + k * q0;
  e[4] = (ty - 0.5 * p1) + k * q1;
  e[5] = (tz - 0.5 * p2) + k * q2;
}

// Exp of (omega, v) applied on the left of T (same closed form as the ICP
// pose update).
__device__ inline void exp_left(const double* xi, const double* T, double* out) {
  const double wx = xi[0], wy = xi[1], wz = xi[2];
  const double th2 = (wx * wx + wy * wy) + wz * wz;
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    const double sn = sin(th), sh = sin(0.5 * th);
    A = sn / th;
    B = 2.0 * sh * sh / th2;
    C = (th - sn) / (th2 * th);
  }
  const double W[3][3] = {{0.0, -wz, wy}, {wz, 0.0, -wx}, {-wy, wx, 0.0}};
  double E[16];
  for (int r = 0; r < 3; ++r) {
    double vr = 0.0;
    for (int c = 0; c < 3; ++c) {
      double w2 = 0.0;
      for (int m = 0; m < 3; ++m) w2 += W[r][m] * W[m][c];
      const double I = r == c ? 1.0 : 0.0;
      E[4 * r + c] = I + A * W[r][c] + B * w2;
      vr += (I + B * W[r][c] + C * w2) * xi[3 + c];
    }
    E[4 * r + 3] = vr;
  }
  E[12] = 0.0; E[13] = 0.0; E[14] = 0.0; E[15] = 1.0;
  mul4(E, T, out);
}

// One edge: e, J = Ad(T_j^-1) (rows of (omega, v) = [[R', 0], [[t']_x R', R']]
// with (R', t') = T_j^-1), K = J^T L J, u = J^T L e, f = e^T L e.
__global__ __launch_bounds__(64) void pg_edge_kernel(const double* __restrict__ poses,
                                                     const PgEdge* __restrict__ edges, int m,
                                                     double* __restrict__ terms) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const PgEdge& ed = edges[k];
  const double* Ti = poses + 16 * ed.i;
  const double* Tj = poses + 16 * ed.j;
  double Tii[16], Zi[16], A[16], E[16], Tji[16];
  rigid_inverse(Ti, Tii);
  mul4(Tii, Tj, A);
  rigid_inverse(ed.Z, Zi);
  mul4(Zi, A, E);
  double e[6];
  log_rigid(E, e);
  rigid_inverse(Tj, Tji);
  double J[6][6];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const double R = Tji[4 * r + c];
      J[r][c] = R;
      J[r][3 + c] = 0.0;
      J[3 + r][3 + c] = R;
    }
  const double tx = Tji[3], ty = Tji[7], tz = Tji[11];
  for (int c = 0; c < 3; ++c) {  // [t]_x R'
    const double r0 = Tji[c], r1 = Tji[4 + c], r2 = Tji[8 + c];
    J[3][c] = ty * r2 - tz * r1;
    J[4][c] = tz * r0 - tx * r2;
    J[5][c] = tx * r1 - ty * r0;
  }
  double LJ[6][6], Le[6];
  for (int r = 0; r < 6; ++r) {
    double s = 0.0;
    for (int c = 0; c < 6; ++c) {
      double a = 0.0;
      for (int m2 = 0; m2 < 6; ++m2) a += ed.L[6 * r + m2] * J[m2][c];
      LJ[r][c] = a;
      s += ed.L[6 * r + c] * e[c];
    }
    Le[r] = s;
  }
  double* out = terms + (int64_t)k * kTerms;
  double f = 0.0;
  for (int r = 0; r < 6; ++r) {
    for (int c = 0; c < 6; ++c) {
      double a = 0.0;
      for (int m2 = 0; m2 < 6; ++m2) a += J[m2][r] * LJ[m2][c];
      out[6 * r + c] = a;
    }
    double u = 0.0;
    for (int m2 = 0; m2 < 6; ++m2) u += J[m2][r] * Le[m2];
    out[36 + r] = u;
    f += e[r] * Le[r];
  }
  out[42] = f;
}

// H block (a, b): sum of sign * K over its contributions, in list order;
// the transposed block is written too.
__global__ __launch_bounds__(64) void pg_assemble_h_kernel(const PgBlock* __restrict__ blocks,
                                                           const int2* __restrict__ contrib,
                                                           const double* __restrict__ terms,
                                                           double* __restrict__ H, int n) {
  const PgBlock bl = blocks[blockIdx.x];
  const int t = threadIdx.x;
  if (t >= 36) return;
  const int r = t / 6, c = t % 6;
  double s = 0.0;
  for (int k = 0; k < bl.count; ++k) {
    const int2 ce = contrib[bl.start + k];
    const double v = terms[(int64_t)ce.x * kTerms + 6 * r + c];
    s += ce.y > 0 ? v : -v;
  }
  H[(int64_t)(6 * bl.a + r) * n + 6 * bl.b + c] = s;
  if (bl.a != bl.b) H[(int64_t)(6 * bl.b + c) * n + 6 * bl.a + r] = s;
}

// g over the free nodes: sum of sign * u over each node's incident edges.
__global__ void pg_assemble_g_kernel(const int2* __restrict__ node_range,
                                     const int2* __restrict__ contrib,
                                     const double* __restrict__ terms, double* __restrict__ g,
                                     int n_free) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 6 * n_free) return;
  const int a = q / 6, comp = q % 6;
  const int2 rg = node_range[a];
  double s = 0.0;
  for (int k = 0; k < rg.y; ++k) {
    const int2 ce = contrib[rg.x + k];
    const double v = terms[(int64_t)ce.x * kTerms + 36 + comp];
    s += ce.y > 0 ? v : -v;
  }
  g[q] = s;
}

// F = sum of the edges' f: per-thread sums over a fixed stride, then a fixed
// tree in LDS.
__global__ __launch_bounds__(256) void pg_objective_kernel(const double* __restrict__ terms, int m,
                                                           double* __restrict__ F) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < m; k += 256) s += terms[(int64_t)k * kTerms + 42];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *F = sh[0];
}

// A = H with the diagonal scaled by (1 + lambda), d = -g.
__global__ void pg_damp_kernel(const double* __restrict__ H, double* __restrict__ A,
                               const double* __restrict__ g, double* __restrict__ d, int n,
                               double lambda) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;  // n * n < 2^31 for n <= 6 * 255
  if (q >= n * n) return;
  const int r = q / n, c = q - r * n;
  A[q] = r == c ? H[q] * (1.0 + lambda) : H[q];
  if (q < n) d[q] = -g[q];
}

// Largest diagonal entry of the damped A (before the factorisation).
__global__ __launch_bounds__(256) void pg_diag_max_kernel(const double* __restrict__ A, int n,
                                                          double* __restrict__ dmax) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) m = fmax(m, A[(int64_t)r * n + r]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dmax = sh[0];
}

// Diagonal block [k0, k0 + nb) of the column-major lower factor, nb <= 64,
// by the four wavefronts of a workgroup: lane r keeps row r of the block and
// wavefront w the columns 4m + w, in registers.  Column by column: the
// wavefront holding it reads the pivot from its lane, forms its reciprocal
// square root, scales the column below it (within an ulp or two of dividing
// by the root) and publishes it in LDS; after one barrier every wavefront
// applies the rank-1 update to its own columns (entries right of the
// diagonal are updated too and never stored).  A non-positive pivot records
// its 1-based position in `info` (first one only), is replaced by 1 so that
// nothing becomes NaN, and the run is flagged degenerate by the pivot rule
// afterwards.
constexpr int kPgNb = 64;

// Value of lane `lane` (uniform) to the whole wavefront, read into scalar
// registers (no LDS round trip).
__device__ inline double lane_value(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <bool FULL>
__device__ __forceinline__ void diag_factor_t(double* __restrict__ A, int n, int k0, int nb_arg,
                                              int* __restrict__ info) {
  __shared__ __align__(16) double colbuf[2][4][16];  // column j: L_(4k+q),j at [j & 1][q][k]
  const int nb = FULL ? kPgNb : nb_arg;
  const int t = threadIdx.x, r = t & 63, w = t >> 6;  // row r; wave w holds columns 4k + w
  // every load is issued before any is used: addresses are clamped into the
  // block and the entries outside its lower triangle are zeroed afterwards
  // (a load under a per-lane branch would be waited for at the branch)
  double b[16];
  const int rc = min(r, nb - 1);
#pragma unroll
  for (int k = 0; k < 16; ++k) b[k] = A[(int64_t)(k0 + min(4 * k + w, nb - 1)) * n + (k0 + rc)];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int c = 4 * k + w;
    b[k] = c < nb && r < nb && c <= r ? b[k] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < kPgNb; ++j) {
    if (FULL || j < nb) {
      const int kj = j >> 2, wj = j & 3, par = j & 1;
      if (w == wj) {  // the wavefront that holds column j: pivot, scaling, publication
        const double d = lane_value(b[kj], j);
        const bool bad = !(d > 0.0);
        const double inv = rsqrt(bad ? 1.0 : d);  // the root itself is d / sqrt(d)
        const double piv = bad ? 1.0 : d * inv;
        if (bad && r == 0 && *info == 0) *info = k0 + j + 1;
        b[kj] = r == j ? piv : b[kj] * inv;
        colbuf[par][r & 3][r >> 2] = b[kj];
      }
      __syncthreads();
      const double lrj = colbuf[par][r & 3][r >> 2];
      const double* cj = &colbuf[par][w][0];
#pragma unroll
      for (int k = kj; k < 16; ++k) {
        const double nv = fma(-lrj, cj[k], b[k]);
        b[k] = k > kj || w > wj ? nv : b[k];  // columns 4k + w > j only
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int c = 4 * k + w;
    if (c < nb && r < nb && c <= r) A[(int64_t)(k0 + c) * n + (k0 + r)] = b[k];
  }
}

// All 256 threads of the workgroup take part.
__device__ __forceinline__ void diag_factor(double* __restrict__ A, int n, int k0, int nb, int* __restrict__ info) {
  if (nb == kPgNb)
    diag_factor_t<true>(A, n, k0, nb, info);
  else
    diag_factor_t<false>(A, n, k0, nb, info);
}

__global__ __launch_bounds__(256) void pg_chol_diag_kernel(double* __restrict__ A, int n, int k0, int nb,
                                                           int* __restrict__ info) {
  diag_factor(A, n, k0, nb, info);
}

// Value of lane Q of each group of four lanes, to all four (a DPP quad
// permutation of both halves of the double).
template <int Q>
__device__ inline double quad_bcast_q(double v) {
  constexpr int ctrl = Q | (Q << 2) | (Q << 4) | (Q << 6);
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), ctrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline double quad_bcast(double v, int q) {  // q folds to a constant in unrolled loops
  switch (q) {
    case 0: return quad_bcast_q<0>(v);
    case 1: return quad_bcast_q<1>(v);
    case 2: return quad_bcast_q<2>(v);
    default: return quad_bcast_q<3>(v);
  }
}

// Panel below a factorised diagonal block: row i of X = B L_kk^-T, four
// lanes per row, lane q holding columns 4k + q, right-looking in registers:
// at column c the lane that holds it forms x_c = b_c / L_cc and passes it to
// the other three (a DPP quad broadcast), and each lane applies
// b_m -= x_c L_mc to its columns m > c.  The critical path is nb steps of a
// quarter of the row's work.  L_kk sits in LDS as Lq[c][q][k] = L_(4k+q),c,
// each lane's values along k contiguous (rows padded against bank conflicts),
// with the reciprocals of its diagonal.  FULL: nb == 64 (every block but the
// last), which removes the per-entry bounds from the unrolled loops.
constexpr int kPgPanelRows = 64;  // rows per block of 256 threads
constexpr int kPgLqPad = 18;
template <bool FULL>
__global__ __launch_bounds__(256) void pg_chol_panel_kernel(double* __restrict__ A, int n, int k0, int nb_arg,
                                                            int rem) {
  const int nb = FULL ? kPgNb : nb_arg;
  __shared__ __align__(16) double Lq[kPgNb][4][kPgLqPad];
  __shared__ double rinv[kPgNb];
  const int t = threadIdx.x;
  {
    // all loads in flight at once (clamped addresses; entries above the
    // diagonal and past nb are stored but never read)
    const int m = t & 63, mc = min(m, nb - 1);
    double v[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int c = (t >> 6) + 4 * a;
      v[a] = A[(int64_t)(k0 + min(c, nb - 1)) * n + (k0 + mc)];
    }
#pragma unroll
    for (int a = 0; a < 16; ++a) Lq[(t >> 6) + 4 * a][m & 3][m >> 2] = v[a];
  }
  __syncthreads();
  if (t < nb) rinv[t] = 1.0 / Lq[t][t & 3][t >> 2];
  __syncthreads();
  const int q = t & 3;
  const int i = blockIdx.x * kPgPanelRows + (t >> 2);
  if (i >= rem) return;  // whole quads leave together
  double* row = A + (int64_t)k0 * n + (k0 + nb + i);  // element c at row[c * n]
  double b[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) b[k] = row[(int64_t)min(4 * k + q, nb - 1) * n];
#pragma unroll
  for (int c = 0; c < kPgNb; ++c) {
    if (c < nb) {
      const int kc = c >> 2, qc = c & 3;
      const double x = quad_bcast(b[kc] * rinv[c], qc);
      if (q == qc) b[kc] = x;
      const double* lrow = &Lq[c][q][0];
#pragma unroll
      for (int k = kc; k < 16; ++k) {
        const int m = 4 * k + q;
        const bool upd = (k > kc || q > qc) && (FULL || m < nb);
        const double nv = fma(-x, lrow[k], b[k]);
        b[k] = upd ? nv : b[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (FULL || 4 * k + q < nb) row[(int64_t)(4 * k + q) * n] = b[k];
}

// Forward substitution L y = g, step for the block column [k0, k0 + nb), by
// a whole workgroup of 256 threads: wavefront 0 solves the diagonal block
// (lane r holding row r of L_kk and g_r: y_j is taken from lane j, then
// g_r -= L_rj y_j in lanes r > j), then the workgroup subtracts L_ik y_k from
// rows k0 + nb + first + t, t + stride, ... (one thread per row, coalesced
// along the column).  y goes to its own vector, so no workgroup reads an
// entry of g that another one has already overwritten.
__device__ __forceinline__ void lower_solve_step(const double* __restrict__ L, int n, int k0, int nb,
                                                 double* __restrict__ g, double* __restrict__ y, bool write_y,
                                                 int first, int stride) {
  // (rows of L are read in halves of 32 columns: few registers, so that the
  // trailing-update kernel that also runs this keeps its occupancy)
  constexpr int H = kPgNb / 2;
  __shared__ double ys[kPgNb];
  const int t = threadIdx.x;
  if (t < kPgNb) {
    const int r = t, rc = min(r, nb - 1);
    const double rinv = 1.0 / L[(int64_t)(k0 + rc) * n + (k0 + rc)];
    double v = g[k0 + rc];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double l[H];
#pragma unroll
      for (int c = 0; c < H; ++c) l[c] = L[(int64_t)(k0 + min(h * H + c, nb - 1)) * n + (k0 + rc)];
#pragma unroll
      for (int jj = 0; jj < H; ++jj) {
        const int j = h * H + jj;
        if (j < nb) {
          const double yj = lane_value(v * rinv, j);
          v = r == j ? yj : (r > j ? fma(-l[jj], yj, v) : v);
        }
      }
    }
    ys[r] = v;
    if (write_y && r < nb) y[k0 + r] = v;
  }
  __syncthreads();
  for (int row = k0 + nb + first + t; row < n; row += stride) {
    double acc = g[row];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double lv[H];
#pragma unroll
      for (int c = 0; c < H; ++c) lv[c] = L[(int64_t)(k0 + min(h * H + c, nb - 1)) * n + row];
#pragma unroll
      for (int c = 0; c < H; ++c)
        if (h * H + c < nb) acc = fma(-lv[c], ys[h * H + c], acc);
    }
    g[row] = acc;
  }
}

// One forward-substitution step over a grid: every workgroup solves the
// diagonal block itself and takes its own 256 rows below.
__global__ __launch_bounds__(256) void pg_trsv_lower_kernel(const double* __restrict__ L, int n, int k0, int nb,
                                                            double* __restrict__ g, double* __restrict__ y) {
  lower_solve_step(L, n, k0, nb, g, y, blockIdx.x == 0, (int)blockIdx.x * 256, (int)gridDim.x * 256);
}

// Trailing update C -= P P^T (lower part) after a panel P (rem x nb, column
// k0 .. k0 + nb, rows below the block): block (bj, bi), bj <= bi, computes the
// 64 x 64 output tile (bi, bj) from the two 64-row slices of P in LDS; thread
// (tx, ty) owns rows tx + 16u and columns ty + 16v, so that for each (u, v)
// sixteen lanes update sixteen consecutive entries of one column.  Tile
// (0, 0) is the next diagonal block: once updated, its workgroup factorises
// it, which hides that sequential step behind the other tiles.  An extra row
// of workgroups (blockIdx.y == gridDim.x) carries, in its first workgroup,
// the forward-substitution step of this block column, whose diagonal block
// and panel are final by now.
__global__ __launch_bounds__(256) void pg_chol_update_kernel(double* __restrict__ A, int n, int k0, int nb,
                                                             int rem, int* __restrict__ info, double* __restrict__ g,
                                                             double* __restrict__ y) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi == (int)gridDim.x) {
    if (bj == 0) lower_solve_step(A, n, k0, nb, g, y, true, 0, 256);
    return;
  }
  if (bj > bi) return;  // upper tiles: nothing (uniform per block)
  __shared__ double Pi[kPgNb][kPgNb + 1];
  __shared__ double Pj[kPgNb][kPgNb + 1];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int64_t col0 = (int64_t)k0 * n, row0 = k0 + nb;
  {
    // all 32 loads in flight at once: clamped addresses, then zeroed where
    // out of range (columns past nb are never read)
    double vi[4][4], vj[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = min(ty + 16 * a, nb - 1), q = tx + 16 * e;
        vi[a][e] = A[col0 + (int64_t)c * n + row0 + min(bi * kPgNb + q, rem - 1)];
        vj[a][e] = A[col0 + (int64_t)c * n + row0 + min(bj * kPgNb + q, rem - 1)];
      }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = ty + 16 * a, q = tx + 16 * e;
        Pi[q][c] = bi * kPgNb + q < rem ? vi[a][e] : 0.0;
        Pj[q][c] = bj * kPgNb + q < rem ? vj[a][e] : 0.0;
      }
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int c = 0; c < nb; ++c) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Pi[tx + 16 * u][c];
      b[u] = Pj[ty + 16 * u][c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = bi * kPgNb + tx + 16 * u, q = bj * kPgNb + ty + 16 * v;
      if (r < rem && q <= r) {
        double* e = A + (int64_t)(row0 + q) * n + row0 + r;
        *e = *e - acc[u][v];
      }
    }
  if (bi == 0 && bj == 0) {
    __syncthreads();  // the tile's updated entries, written by all four waves
    diag_factor(A, n, (int)row0, min(kPgNb, rem), info);
  }
}

// Backward substitution L^T x = y for the block column [k0, k0 + nb), blocks
// taken last to first, one wavefront per workgroup: every workgroup solves
// the transposed diagonal block (lane r holding column r of L_kk and y_r: x_j
// from lane j, then y_r -= L_jr x_j in lanes r < j), then subtracts
// L_kj^T x_k from its 64 rows above, one lane per row.  Both the block and the
// rows are read along the factor's columns (coalesced) and transposed in LDS.
// x goes to its own vector.
__global__ __launch_bounds__(kPgNb) void pg_trsv_upper_kernel(const double* __restrict__ L, int n, int k0, int nb,
                                                              double* __restrict__ y, double* __restrict__ x) {
  __shared__ double T[kPgNb][kPgNb + 1];
  __shared__ double xs[kPgNb];
  const int r = threadIdx.x;
  const int rc = min(r, nb - 1);
  {
    double v[kPgNb];  // element (rc, c) of the block
#pragma unroll
    for (int c = 0; c < kPgNb; ++c) v[c] = L[(int64_t)(k0 + min(c, nb - 1)) * n + (k0 + rc)];
#pragma unroll
    for (int c = 0; c < kPgNb; ++c) T[r][c] = v[c];
  }
  __syncthreads();
  double u[kPgNb];  // column r of the block: u[j] = L_jr
#pragma unroll
  for (int j = 0; j < kPgNb; ++j) u[j] = T[min(j, nb - 1)][rc];
  const double rinv = 1.0 / T[rc][rc];
  double v = y[k0 + rc];
#pragma unroll
  for (int j = kPgNb - 1; j >= 0; --j) {
    if (j < nb) {
      const double xj = lane_value(v * rinv, j);
      v = r == j ? xj : (r < j ? fma(-u[j], xj, v) : v);
    }
  }
  xs[r] = v;
  if (blockIdx.x == 0 && r < nb) x[k0 + r] = v;
  const int row0 = (int)blockIdx.x * kPgNb;
  if (row0 >= k0) return;  // uniform: no rows above for this workgroup
  {
    double w[kPgNb];  // lane r: element (k0 + r, row0 + jj) of the factor
#pragma unroll
    for (int jj = 0; jj < kPgNb; ++jj) w[jj] = L[(int64_t)min(row0 + jj, k0 - 1) * n + (k0 + rc)];
    __syncthreads();  // every lane is done reading the diagonal block from T
#pragma unroll
    for (int jj = 0; jj < kPgNb; ++jj) T[jj][r] = w[jj];
  }
  __syncthreads();
  const int row = row0 + r;
  if (row < k0) {
    double acc = y[row];
#pragma unroll
    for (int c = 0; c < kPgNb; ++c)
      if (c < nb) acc = fma(-T[r][c], xs[c], acc);
    y[row] = acc;
  }
}

// Pivot rule on the factor: failed factorisation, or some L_kk^2 <= 1e-12 max diag.
__global__ __launch_bounds__(256) void pg_pivot_check_kernel(const double* __restrict__ L, int n,
                                                             const double* __restrict__ dmax,
                                                             const int* __restrict__ info,
                                                             int* __restrict__ flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = *info != 0 ? 1 : 0;
  __syncthreads();
  const double thr = 1e-12 * *dmax;
  int mine = 0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double l = L[(int64_t)r * n + r];
    if (!(l * l > thr)) mine = 1;
  }
  if (mine) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) *flag = bad;
}

__global__ void pg_update_kernel(const double* __restrict__ poses, const double* __restrict__ d,
                                 int n_nodes, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_nodes) return;
  if (k == 0) {
    for (int q = 0; q < 16; ++q) out[q] = poses[q];
    return;
  }
  exp_left(d + 6 * (k - 1), poses + 16 * k, out + 16 * k);
}

bool rigid_ok(const double* T) {
  for (int k = 0; k < 16; ++k)
    if (!std::isfinite(T[k])) return false;
  return T[12] == 0.0 && T[13] == 0.0 && T[14] == 0.0 && T[15] == 1.0;
}

}  // namespace

extern "C" {

int icp_pose_graph_optimize(icp_ctx_t* ctx, int32_t n_nodes, double* poses, int32_t n_edges,
                            const icp_pose_edge_t* edges, int32_t method, int32_t max_iter,
                            double rel_tol, icp_pose_graph_result_t* out) {
  if (n_nodes < 2 || n_nodes > kMaxPgNodes)
    return fail(ICP_E_INVALID_ARG, "n_nodes must be in [2, " + std::to_string(kMaxPgNodes) + "]");
  if (!poses || !edges || !out || n_edges < 1) return fail(ICP_E_INVALID_ARG, "NULL pointer or no edges");
  if (method != ICP_PG_GAUSS_NEWTON && method != ICP_PG_LEVENBERG_MARQUARDT)
    return fail(ICP_E_INVALID_ARG, "unknown method");
  if (max_iter < 0 || !(rel_tol >= 0.0) || !std::isfinite(rel_tol))
    return fail(ICP_E_INVALID_ARG, "max_iter must be >= 0 and rel_tol finite and >= 0");
  for (int k = 0; k < n_nodes; ++k)
    if (!rigid_ok(poses + 16 * k)) return fail(ICP_E_INVALID_ARG, "pose " + std::to_string(k) + " is not a finite rigid transform");
  for (int k = 0; k < n_edges; ++k) {
    const icp_pose_edge_t& e = edges[k];
    if (e.i < 0 || e.j < 0 || e.i >= n_nodes || e.j >= n_nodes || e.i == e.j)
      return fail(ICP_E_INVALID_ARG, "edge " + std::to_string(k) + " has a bad node index");
    if (!rigid_ok(e.Z)) return fail(ICP_E_INVALID_ARG, "edge " + std::to_string(k) + ": Z is not a finite rigid transform");
    for (int q = 0; q < 36; ++q)
      if (!std::isfinite(e.information[q])) return fail(ICP_E_INVALID_ARG, "edge " + std::to_string(k) + ": information not finite");
    // the factorisation reads one triangle of H: an asymmetric information
    // matrix would silently solve other normal equations than F's
    for (int a = 0; a < 6; ++a)
      for (int b = a + 1; b < 6; ++b)
        if (e.information[6 * a + b] != e.information[6 * b + a])
          return fail(ICP_E_INVALID_ARG, "edge " + std::to_string(k) + ": information matrix is not symmetric");
  }
  int rc;
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  hipStream_t s = c->stream;
  const int nf = n_nodes - 1, n = 6 * nf, m = n_edges;

  // incidence lists (host): H blocks (diagonal and one per connected pair of
  // free nodes) and per-node g contributions, each in edge order
  std::vector<PgBlock> blocks;
  std::vector<int2> hcontrib, gcontrib;
  std::vector<int2> node_range(nf);
  {
    std::vector<std::vector<int2>> inc(nf);
    for (int k = 0; k < m; ++k) {
      if (edges[k].i > 0) inc[edges[k].i - 1].push_back(make_int2(k, -1));
      if (edges[k].j > 0) inc[edges[k].j - 1].push_back(make_int2(k, +1));
    }
    for (int a = 0; a < nf; ++a) {
      node_range[a] = make_int2((int)gcontrib.size(), (int)inc[a].size());
      gcontrib.insert(gcontrib.end(), inc[a].begin(), inc[a].end());
      // diagonal block: sign * sign = +1 for every incident edge
      PgBlock b{a, a, (int)hcontrib.size(), (int)inc[a].size()};
      for (const int2& ce : inc[a]) hcontrib.push_back(make_int2(ce.x, +1));
      blocks.push_back(b);
    }
    std::vector<std::pair<std::pair<int, int>, int>> off;  // ((a, b), edge), a < b
    for (int k = 0; k < m; ++k) {
      const int a = edges[k].i - 1, b = edges[k].j - 1;
      if (a < 0 || b < 0) continue;
      off.push_back({{std::min(a, b), std::max(a, b)}, k});
    }
    std::stable_sort(off.begin(), off.end(),
                     [](const auto& x, const auto& y) { return x.first < y.first; });
    for (size_t q = 0; q < off.size();) {
      size_t r = q;
      PgBlock b{off[q].first.first, off[q].first.second, (int)hcontrib.size(), 0};
      while (r < off.size() && off[r].first == off[q].first) {
        hcontrib.push_back(make_int2(off[r].second, -1));  // J_i^T L J_j = -K
        ++r;
      }
      b.count = (int)(r - q);
      blocks.push_back(b);
      q = r;
    }
  }
  std::vector<PgEdge> hedges(m);
  for (int k = 0; k < m; ++k) {
    hedges[k].i = edges[k].i;
    hedges[k].j = edges[k].j;
    for (int q = 0; q < 16; ++q) hedges[k].Z[q] = edges[k].Z[q];
    for (int q = 0; q < 36; ++q) hedges[k].L[q] = edges[k].information[q];
  }

  // device layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align256(off);
    off = o + bytes;
    return o;
  };
  const size_t o_p = take(sizeof(double) * 16 * n_nodes), o_c = take(sizeof(double) * 16 * n_nodes);
  const size_t o_e = take(sizeof(PgEdge) * m);
  const size_t o_t = take(sizeof(double) * kTerms * m), o_tc = take(sizeof(double) * kTerms * m);
  const size_t o_h = take(sizeof(double) * (size_t)n * n), o_a = take(sizeof(double) * (size_t)n * n);
  const size_t o_g = take(sizeof(double) * n), o_d = take(sizeof(double) * n), o_y = take(sizeof(double) * n);
  const size_t o_b = take(sizeof(PgBlock) * blocks.size());
  const size_t o_hc = take(sizeof(int2) * std::max<size_t>(hcontrib.size(), 1));
  const size_t o_gc = take(sizeof(int2) * std::max<size_t>(gcontrib.size(), 1));
  const size_t o_nr = take(sizeof(int2) * nf);
  const size_t o_s = take(64);  // F (double), flag (int), max diag (double), info (int)
  const size_t total = align256(off);
  HIP_TRY(c->pg.ensure(total), "alloc");
  char* dd = c->pg.as<char>();
  if ((rc = ensure_host(c, 64)) != 0) return rc;
  char* hs = static_cast<char*>(c->host);
  HIP_TRY(hipMemcpyAsync(dd + o_p, poses, sizeof(double) * 16 * n_nodes, hipMemcpyHostToDevice, s), "upload");
  HIP_TRY(hipMemcpyAsync(dd + o_e, hedges.data(), sizeof(PgEdge) * m, hipMemcpyHostToDevice, s), "upload");
  HIP_TRY(hipMemcpyAsync(dd + o_b, blocks.data(), sizeof(PgBlock) * blocks.size(), hipMemcpyHostToDevice, s), "upload");
  if (!hcontrib.empty())
    HIP_TRY(hipMemcpyAsync(dd + o_hc, hcontrib.data(), sizeof(int2) * hcontrib.size(), hipMemcpyHostToDevice, s), "upload");
  if (!gcontrib.empty())
    HIP_TRY(hipMemcpyAsync(dd + o_gc, gcontrib.data(), sizeof(int2) * gcontrib.size(), hipMemcpyHostToDevice, s), "upload");
  HIP_TRY(hipMemcpyAsync(dd + o_nr, node_range.data(), sizeof(int2) * nf, hipMemcpyHostToDevice, s), "upload");

  double* P = reinterpret_cast<double*>(dd + o_p);
  double* Cn = reinterpret_cast<double*>(dd + o_c);
  double* TT = reinterpret_cast<double*>(dd + o_t);
  double* TC = reinterpret_cast<double*>(dd + o_tc);
  double* H = reinterpret_cast<double*>(dd + o_h);
  double* A = reinterpret_cast<double*>(dd + o_a);
  double* g = reinterpret_cast<double*>(dd + o_g);
  double* dv = reinterpret_cast<double*>(dd + o_d);
  double* Fd = reinterpret_cast<double*>(dd + o_s);
  int* flag = reinterpret_cast<int*>(dd + o_s + 8);
  double* dmax = reinterpret_cast<double*>(dd + o_s + 16);
  int* info = reinterpret_cast<int*>(dd + o_s + 24);
  double* yv = reinterpret_cast<double*>(dd + o_y);
  const PgEdge* E = reinterpret_cast<const PgEdge*>(dd + o_e);
  const PgBlock* B = reinterpret_cast<const PgBlock*>(dd + o_b);
  const int2* HC = reinterpret_cast<const int2*>(dd + o_hc);
  const int2* GC = reinterpret_cast<const int2*>(dd + o_gc);
  const int2* NR = reinterpret_cast<const int2*>(dd + o_nr);
  const unsigned eb = (unsigned)((m + 63) / 64);

  auto terms_and_F = [&](const double* poses_d, double* terms_d) -> int {
    hipLaunchKernelGGL(pg_edge_kernel, dim3(eb), dim3(64), 0, s, poses_d, E, m, terms_d);
    hipLaunchKernelGGL(pg_objective_kernel, dim3(1), dim3(256), 0, s, terms_d, m, Fd);
    HIP_TRY(hipGetLastError(), "pose graph terms");
    return ICP_SUCCESS;
  };
  auto assemble = [&](const double* terms_d) -> int {
    HIP_TRY(hipMemsetAsync(H, 0, sizeof(double) * (size_t)n * n, s), "memset");
    hipLaunchKernelGGL(pg_assemble_h_kernel, dim3((unsigned)blocks.size()), dim3(64), 0, s, B, HC, terms_d, H, n);
    hipLaunchKernelGGL(pg_assemble_g_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, NR, GC, terms_d, g, nf);
    HIP_TRY(hipGetLastError(), "pose graph assembly");
    return ICP_SUCCESS;
  };
  auto read_scalars = [&](double* F, int* fl) -> int {
    HIP_TRY(hipMemcpyAsync(hs, dd + o_s, 16, hipMemcpyDeviceToHost, s), "readback");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    *F = *reinterpret_cast<double*>(hs);
    *fl = *reinterpret_cast<int*>(hs + 8);
    return ICP_SUCCESS;
  };

  int fl = 0;
  double F = 0.0;
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s), "memset");
  if ((rc = terms_and_F(P, TT)) != 0) return rc;
  if ((rc = assemble(TT)) != 0) return rc;
  if ((rc = read_scalars(&F, &fl)) != 0) return rc;
  const double F0 = F;
  const bool lm = method == ICP_PG_LEVENBERG_MARQUARDT;
  double lambda = 1e-4;
  int steps = 0, refusals = 0, status = ICP_OK;
  while (steps < max_iter) {
    hipLaunchKernelGGL(pg_damp_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, H, A, g,
                       dv, n, lm ? lambda : 0.0);
    hipLaunchKernelGGL(pg_diag_max_kernel, dim3(1), dim3(256), 0, s, A, n, dmax);
    // A is symmetric: its row-major storage is also its column-major one.
    // Blocked right-looking Cholesky of its lower triangle.
    HIP_TRY(hipMemsetAsync(info, 0, sizeof(int), s), "memset");
    // the first diagonal block here, every later one by the update before it
    hipLaunchKernelGGL(pg_chol_diag_kernel, dim3(1), dim3(256), 0, s, A, n, 0, std::min(kPgNb, n), info);
    HIP_TRY(hipGetLastError(), "pose graph factorisation");
    for (int k0 = 0; k0 < n; k0 += kPgNb) {
      const int nb = std::min(kPgNb, n - k0), rem = n - k0 - nb;
      if (rem == 0) break;
      const dim3 pgrid((unsigned)((rem + kPgPanelRows - 1) / kPgPanelRows));
      if (nb == kPgNb)
        hipLaunchKernelGGL(pg_chol_panel_kernel<true>, pgrid, dim3(256), 0, s, A, n, k0, nb, rem);
      else
        hipLaunchKernelGGL(pg_chol_panel_kernel<false>, pgrid, dim3(256), 0, s, A, n, k0, nb, rem);
      HIP_TRY(hipGetLastError(), "pose graph factorisation");
      // the trailing update also carries this block column's forward-
      // substitution step (L y = rhs): dv is consumed, y collects
      const unsigned tiles = (unsigned)((rem + kPgNb - 1) / kPgNb);
      hipLaunchKernelGGL(pg_chol_update_kernel, dim3(tiles, tiles + 1), dim3(256), 0, s, A, n, k0, nb, rem, info, dv,
                         yv);
      HIP_TRY(hipGetLastError(), "pose graph factorisation");
    }
    hipLaunchKernelGGL(pg_pivot_check_kernel, dim3(1), dim3(256), 0, s, A, n, dmax, info, flag);
    // the last block column's forward step, then L^T x = y from the last
    // block back; dv receives x
    {
      const int k0 = ((n - 1) / kPgNb) * kPgNb;
      hipLaunchKernelGGL(pg_trsv_lower_kernel, dim3(1), dim3(256), 0, s, A, n, k0, n - k0, dv, yv);
    }
    for (int k0 = ((n - 1) / kPgNb) * kPgNb; k0 >= 0; k0 -= kPgNb) {
      const int nb = std::min(kPgNb, n - k0);
      hipLaunchKernelGGL(pg_trsv_upper_kernel, dim3((unsigned)std::max(1, (k0 + kPgNb - 1) / kPgNb)), dim3(kPgNb), 0,
                         s, A, n, k0, nb, yv, dv);
    }
    HIP_TRY(hipGetLastError(), "pose graph solve");
    hipLaunchKernelGGL(pg_update_kernel, dim3((unsigned)((n_nodes + 63) / 64)), dim3(64), 0, s, P, dv,
                       n_nodes, Cn);
    HIP_TRY(hipGetLastError(), "pose graph step");
    if ((rc = terms_and_F(Cn, TC)) != 0) return rc;
    double Fn = 0.0;
    if ((rc = read_scalars(&Fn, &fl)) != 0) return rc;
    if (fl) {
      status = ICP_DEGENERATE;
      break;
    }
    if (lm && !(Fn < F)) {
      lambda *= 10.0;
      if (++refusals >= 10) {
        status = ICP_CONVERGED;
        break;
      }
      continue;
    }
    refusals = 0;
    if (lm) lambda /= 10.0;
    ++steps;
    const bool done = fabs(F - Fn) <= rel_tol * F;
    std::swap(P, Cn);
    std::swap(TT, TC);
    F = Fn;
    if ((rc = assemble(TT)) != 0) return rc;
    if (done) {
      status = ICP_CONVERGED;
      break;
    }
  }
  HIP_TRY(hipMemcpyAsync(poses, P, sizeof(double) * 16 * n_nodes, hipMemcpyDeviceToHost, s), "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  out->F_initial = F0;
  out->F_final = F;
  out->steps = steps;
  out->status = status;
  return ICP_SUCCESS;
}

}  // extern "C"
