// ICP oracle: plain, slow, FP64 CPU implementation of the registration loop.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code,
// header, table or helper with the GPU library; the product path never calls
// it.
//
// What it computes (paper: Open3D, Sec. 3.3 "Registration" and Sec. 4
// "Optimization"):
//   * ICP refinement of a source cloud onto a target cloud given an initial
//     transform and a maximum correspondence distance (Sec. 3.3, the
//     registration_icp example), point-to-plane or point-to-point [2, 4].
//   * Each iteration is one Gauss-Newton step of the least-squares objective
//     L(x) = sum_i r_i(x)^2 (Sec. 4, eq. (1)): x <- x - (J^T J)^{-1} J^T r
//     (eq. (2)), with J^T J and J^T r formed as a reduction over per-record
//     contributions (Sec. 4, the OpenMP reduction over a per-record lambda).
//   * Nearest neighbours come from a k-d tree (the paper delegates NN search to
//     FLANN, Sec. 2) or brute force on small inputs.
//
// Readings where the paper is silent (all shared with the GPU path by
// definition, not by code):
//   - selection: PINNED_FP32 mode transforms s in FP64 without FMA
//     (((R00*sx + R01*sy) + R02*sz) + tx), rounds to FP32, and takes the FP32
//     squared distance ((dx*dx + dy*dy) + dz*dz) without FMA; FP64 mode uses the
//     unrounded FP64 distance.  Nearest = lexicographic minimum of
//     (distance, original target index); inlier iff distance <= r^2, with
//     r2_32 = (float)(r*r) in PINNED_FP32 mode.
//   - update: xi = (omega, v) rotation first, left perturbation
//     T <- Exp(xi) * T, xi solves A xi = -b (no damping, no line search).
//   - fitness = inliers / N_src, inlier_rmse = sqrt(sum |T s - p|^2 / inliers)
//     with the FP64 Euclidean distance, both at the returned T.
//   - convergence: relative change of both the inlier count and the rmse
//     between consecutive passes <= rel_tol.
//   - degeneracy: no inliers, or a Cholesky pivot <= 1e-12 * max(diag A).
//
// Robust variants (the paper mentions "other ICP variants" without naming
// them): iteratively reweighted least squares.  Each correspondence's terms
// are multiplied by w(s) = rho'(s) / s at its residual magnitude s (|n . d|
// point-to-plane, |d| point-to-point) at the current pose, for the Huber,
// Tukey (biweight) and Cauchy losses of scale k; fitness and rmse stay
// unweighted.
//
// Normal estimation (Sec. 3.2, Fig. 1, and the Sec. 3.3 workflow: a hybrid
// neighbourhood of at most max_nn points within a radius; the method of [16],
// the normal being the direction of least variance of the neighbourhood).
// Readings: the neighbourhood of point i is the max_nn lexicographically
// smallest (pinned FP32 squared distance, original index) among the points j
// (i included) with that distance <= (float)(radius^2); fewer than three
// neighbours give the zero vector; mean and covariance (divided by the count)
// in FP64; the normal is the unit eigenvector of the smallest eigenvalue,
// turned so that n . (viewpoint - p_i) >= 0.
//
// Build: g++ -std=c++17 -O2 -ffp-contract=off -fopenmp -shared -fPIC.
// Every function here is plain scalar code so it can be checked by eye.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include <omp.h>

namespace {

constexpr int kSelPinnedF32 = 0;
constexpr int kSelF64 = 1;
constexpr int kPointToPoint = 0;
constexpr int kPointToPlane = 1;
constexpr int kStatusOk = 0;
constexpr int kStatusConverged = 1;
constexpr int kStatusDegenerate = 2;
constexpr int kLeafSize = 16;
constexpr int64_t kChunk = 4096;  // fixed summation chunk: order independent of threads

// ---------------------------------------------------------------- transform
// q64 = R s + t, evaluated term by term in the pinned order, no FMA.
inline void transform64(const double T[16], const float s[3], double q[3]) {
  const double sx = s[0], sy = s[1], sz = s[2];
  for (int a = 0; a < 3; ++a) {
    double acc = T[4 * a + 0] * sx;
    acc = acc + T[4 * a + 1] * sy;
    acc = acc + T[4 * a + 2] * sz;
    q[a] = acc + T[4 * a + 3];
  }
}

// FP32 squared distance in the pinned order, no FMA.
inline float pinned_d2(const float q[3], const float p[3]) {
  const float dx = q[0] - p[0];
  const float dy = q[1] - p[1];
  const float dz = q[2] - p[2];
  float d2 = dx * dx + dy * dy;
  d2 = d2 + dz * dz;
  return d2;
}

inline double d2_64(const double q[3], const float p[3]) {
  const double dx = q[0] - (double)p[0];
  const double dy = q[1] - (double)p[1];
  const double dz = q[2] - (double)p[2];
  return (dx * dx + dy * dy) + dz * dz;
}

// ---------------------------------------------------------------- k-d tree
struct KdNode {
  int64_t lo, hi;      // range in idx[]
  int dim;             // split dimension (-1 = leaf)
  double split;
  int64_t left, right;
};

struct KdTree {
  const float* pts = nullptr;  // (n, 3) original target points
  int64_t n = 0;
  std::vector<int64_t> idx;
  std::vector<KdNode> nodes;

  void build(const float* p, int64_t count) {
    pts = p;
    n = count;
    idx.resize(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    nodes.clear();
    nodes.reserve(2 * (n / kLeafSize + 1) + 1);
    if (n > 0) make(0, n);
  }

  int64_t make(int64_t lo, int64_t hi) {
    const int64_t id = (int64_t)nodes.size();
    nodes.push_back(KdNode{lo, hi, -1, 0.0, -1, -1});
    if (hi - lo <= kLeafSize) return id;
    double mn[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL};
    double mx[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int64_t k = lo; k < hi; ++k)
      for (int a = 0; a < 3; ++a) {
        const double v = pts[3 * idx[k] + a];
        mn[a] = std::min(mn[a], v);
        mx[a] = std::max(mx[a], v);
      }
    int dim = 0;
    for (int a = 1; a < 3; ++a)
      if (mx[a] - mn[a] > mx[dim] - mn[dim]) dim = a;
    if (mx[dim] - mn[dim] <= 0.0) return id;  // all coincident: keep as a leaf
    const int64_t mid = lo + (hi - lo) / 2;
    std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi,
                     [&](int64_t a, int64_t b) { return pts[3 * a + dim] < pts[3 * b + dim]; });
    const double split = pts[3 * idx[mid] + dim];
    const int64_t l = make(lo, mid);
    const int64_t r = make(mid, hi);
    nodes[id].dim = dim;
    nodes[id].split = split;
    nodes[id].left = l;
    nodes[id].right = r;
    return id;
  }

  // Calls f(j) for every point j with squared distance to c possibly <= R2
  // (a superset: the caller applies the exact test).  Left subtrees hold
  // coordinates <= split, right subtrees >= split.
  template <class F>
  void range(const double c[3], double R2, F&& f) const {
    if (n == 0) return;
    int64_t stack[128];
    int top = 0;
    stack[top++] = 0;
    while (top > 0) {
      const KdNode& nd = nodes[stack[--top]];
      if (nd.dim < 0) {
        for (int64_t k = nd.lo; k < nd.hi; ++k) f(idx[k]);
        continue;
      }
      const double diff = c[nd.dim] - nd.split;
      const int64_t near_child = diff <= 0.0 ? nd.left : nd.right;
      const int64_t far_child = diff <= 0.0 ? nd.right : nd.left;
      if (diff * diff <= R2) stack[top++] = far_child;
      stack[top++] = near_child;
    }
  }
};

// ---------------------------------------------------------------- selection
struct Match {
  int64_t j;      // original target index, -1 if none
  float d2f;      // pinned FP32 squared distance (PINNED_FP32 mode)
  double d2d;     // FP64 squared distance |q64 - p|^2
};

struct Selector {
  const float* tgt;
  int64_t n_tgt;
  double r;
  int mode;
  bool use_tree;
  KdTree tree;

  Selector(const float* t, int64_t nt, double radius, int m, bool tree_search)
      : tgt(t), n_tgt(nt), r(radius), mode(m), use_tree(tree_search) {
    if (use_tree) tree.build(tgt, n_tgt);
  }

  Match select(const double q64[3]) const {
    Match best{-1, std::numeric_limits<float>::infinity(), std::numeric_limits<double>::infinity()};
    if (mode == kSelPinnedF32) {
      const float q32[3] = {(float)q64[0], (float)q64[1], (float)q64[2]};
      const float r2f = (float)(r * r);
      auto visit = [&](int64_t j) {
        const float d = pinned_d2(q32, tgt + 3 * j);
        if (!(d <= r2f)) return;
        if (d < best.d2f || (d == best.d2f && j < best.j)) {
          best.j = j;
          best.d2f = d;
        }
      };
      if (use_tree) {
        const double c[3] = {(double)q32[0], (double)q32[1], (double)q32[2]};
        tree.range(c, r * r * (1.0 + 1e-5), visit);
      } else {
        for (int64_t j = 0; j < n_tgt; ++j) visit(j);
      }
    } else {
      const double r2 = r * r;
      auto visit = [&](int64_t j) {
        const double d = d2_64(q64, tgt + 3 * j);
        if (!(d <= r2)) return;
        if (d < best.d2d || (d == best.d2d && j < best.j)) {
          best.j = j;
          best.d2d = d;
        }
      };
      if (use_tree) {
        tree.range(q64, r2 * (1.0 + 1e-9), visit);
      } else {
        for (int64_t j = 0; j < n_tgt; ++j) visit(j);
      }
    }
    if (best.j >= 0) best.d2d = d2_64(q64, tgt + 3 * best.j);
    return best;
  }
};

// ---------------------------------------------------------------- per record
// Residual(s) and Jacobian rows at q for target point p with normal n.
// Point-to-plane [4]: r = n . (q - p),  J = [ (q x n)^T , n^T ].
// Point-to-point [2]: r = q - p,        J = [ -[q]_x , I ].
// Returns the number of residual rows (1 or 3); J is row-major rows x 6.
int residual_jacobian(int variant, const double q[3], const double p[3], const double n[3],
                      double res[3], double J[18]) {
  const double d[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
  if (variant == kPointToPlane) {
    res[0] = (n[0] * d[0] + n[1] * d[1]) + n[2] * d[2];
    J[0] = q[1] * n[2] - q[2] * n[1];
    J[1] = q[2] * n[0] - q[0] * n[2];
    J[2] = q[0] * n[1] - q[1] * n[0];
    J[3] = n[0];
    J[4] = n[1];
    J[5] = n[2];
    return 1;
  }
  // -[q]_x rows
  const double mq[3][3] = {{0.0, q[2], -q[1]}, {-q[2], 0.0, q[0]}, {q[1], -q[0], 0.0}};
  for (int a = 0; a < 3; ++a) {
    res[a] = d[a];
    for (int c = 0; c < 3; ++c) {
      J[6 * a + c] = mq[a][c];
      J[6 * a + 3 + c] = (a == c) ? 1.0 : 0.0;
    }
  }
  return 3;
}

// Accumulator of one chunk: upper triangle of A (21), b (6), sum d2, count.
struct Sums {
  double A[36];
  double b[6];
  double sd2;
  int64_t n;
  void clear() {
    std::memset(A, 0, sizeof A);
    std::memset(b, 0, sizeof b);
    sd2 = 0.0;
    n = 0;
  }
  void add(const Sums& o) {
    for (int k = 0; k < 36; ++k) A[k] += o.A[k];
    for (int k = 0; k < 6; ++k) b[k] += o.b[k];
    sd2 += o.sd2;
    n += o.n;
  }
};

struct PassResult {
  Sums s;
};

// Robust loss: kind 0 none (w = 1), 1 Huber, 2 Tukey, 3 Cauchy, scale k > 0.
constexpr int kLossNone = 0, kLossHuber = 1, kLossTukey = 2, kLossCauchy = 3;
struct Loss {
  int kind = kLossNone;
  double k = 1.0;
};

// IRLS weight rho'(s) / s of the loss at residual magnitude s >= 0:
//   Huber  rho = s^2 / 2 (s <= k), k (s - k / 2) otherwise  -> w = 1 or k / s
//   Tukey  rho = k^2 / 6 (1 - (1 - (s/k)^2)^3) (s <= k), k^2 / 6 otherwise
//          -> w = (1 - (s/k)^2)^2 or 0
//   Cauchy rho = k^2 / 2 log(1 + (s/k)^2)  -> w = 1 / (1 + (s/k)^2)
double loss_weight(const Loss& L, double s) {
  switch (L.kind) {
    case kLossHuber:
      return s <= L.k ? 1.0 : L.k / s;
    case kLossTukey: {
      if (s > L.k) return 0.0;
      const double u = 1.0 - (s / L.k) * (s / L.k);
      return u * u;
    }
    case kLossCauchy:
      return 1.0 / (1.0 + (s / L.k) * (s / L.k));
    default:
      return 1.0;
  }
}

// One correspondence pass at T: fills per-source matches (optional) and the
// normal-equation sums.  Summation is in fixed chunks of kChunk source points,
// chunk partials are added in chunk order, so the result does not depend on
// the number of threads.
void pass(const Selector& sel, const float* src, int64_t n_src, const float* tgt_n,
          const double T[16], int variant, Sums* out, int64_t* idx_out, float* d2f_out,
          double* d2d_out, const Loss& loss = Loss()) {
  const int64_t n_chunks = (n_src + kChunk - 1) / kChunk;
  std::vector<Sums> part((size_t)n_chunks);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < n_chunks; ++c) {
    Sums& S = part[(size_t)c];
    S.clear();
    const int64_t i0 = c * kChunk, i1 = std::min(n_src, i0 + kChunk);
    for (int64_t i = i0; i < i1; ++i) {
      double q[3];
      transform64(T, src + 3 * i, q);
      const Match m = sel.select(q);
      if (idx_out) idx_out[i] = m.j;
      if (d2f_out) d2f_out[i] = m.d2f;
      if (d2d_out) d2d_out[i] = m.d2d;
      if (m.j < 0) continue;
      const float* pf = sel.tgt + 3 * m.j;
      const double p[3] = {pf[0], pf[1], pf[2]};
      double nrm[3] = {0.0, 0.0, 0.0};
      if (variant == kPointToPlane) {
        const float* nf = tgt_n + 3 * m.j;
        nrm[0] = nf[0]; nrm[1] = nf[1]; nrm[2] = nf[2];
      }
      double res[3], J[18];
      const int rows = residual_jacobian(variant, q, p, nrm, res, J);
      double w = 1.0;
      if (loss.kind != kLossNone) {
        double s2 = 0.0;
        for (int a = 0; a < rows; ++a) s2 += res[a] * res[a];
        w = loss_weight(loss, std::sqrt(s2));
      }
      for (int a = 0; a < rows; ++a) {
        const double* Ja = J + 6 * a;
        for (int u = 0; u < 6; ++u) {
          for (int v = u; v < 6; ++v) S.A[6 * u + v] += w * (Ja[u] * Ja[v]);
          S.b[u] += w * (Ja[u] * res[a]);
        }
      }
      S.sd2 += m.d2d;
      S.n += 1;
    }
  }
  out->clear();
  for (int64_t c = 0; c < n_chunks; ++c) out->add(part[(size_t)c]);
}

// ---------------------------------------------------------------- solve
// Cholesky of the symmetric 6x6 A (upper triangle given), then xi = -A^{-1} b.
// Returns false if a pivot is <= 1e-12 * max(diag A).
bool solve6(const double Aup[36], const double b[6], double xi[6]) {
  double A[6][6];
  for (int u = 0; u < 6; ++u)
    for (int v = u; v < 6; ++v) A[u][v] = A[v][u] = Aup[6 * u + v];
  double dmax = 0.0;
  for (int u = 0; u < 6; ++u) dmax = std::max(dmax, A[u][u]);
  const double tol = 1e-12 * dmax;
  double L[6][6] = {};
  for (int j = 0; j < 6; ++j) {
    double piv = A[j][j];
    for (int k = 0; k < j; ++k) piv -= L[j][k] * L[j][k];
    if (!(piv > tol)) return false;
    L[j][j] = std::sqrt(piv);
    for (int i = j + 1; i < 6; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s / L[j][j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = -b[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 6; ++k) s -= L[k][i] * xi[k];
    xi[i] = s / L[i][i];
  }
  return true;
}

// Exp of the twist xi = (omega, v) as a 4x4 row-major matrix:
//   R = I + A W + B W^2,  V = I + B W + C W^2,  t = V v,  W = [omega]_x,
//   A = sin(th)/th, B = (1 - cos th)/th^2 = 2 sin^2(th/2)/th^2 (half-angle form,
//   free of cancellation), C = (th - sin th)/th^3, with three-term Taylor
//   series below th = 1e-4.
void se3_exp(const double xi[6], double E[16]) {
  const double w[3] = {xi[0], xi[1], xi[2]};
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = std::sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    const double s = std::sin(th), sh = std::sin(0.5 * th);
    A = s / th;
    B = 2.0 * sh * sh / th2;
    C = (th - s) / (th2 * th);
  }
  const double W[3][3] = {{0.0, -w[2], w[1]}, {w[2], 0.0, -w[0]}, {-w[1], w[0], 0.0}};
  double W2[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += W[i][k] * W[k][j];
      W2[i][j] = s;
    }
  double R[3][3], V[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double I = (i == j) ? 1.0 : 0.0;
      R[i][j] = I + A * W[i][j] + B * W2[i][j];
      V[i][j] = I + B * W[i][j] + C * W2[i][j];
    }
  std::memset(E, 0, 16 * sizeof(double));
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) E[4 * i + j] = R[i][j];
    E[4 * i + 3] = V[i][0] * xi[3] + V[i][1] * xi[4] + V[i][2] * xi[5];
  }
  E[15] = 1.0;
}

void matmul4(const double X[16], const double Y[16], double Z[16]) {
  double tmp[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += X[4 * i + k] * Y[4 * k + j];
      tmp[4 * i + j] = s;
    }
  std::memcpy(Z, tmp, sizeof tmp);
}

void pack21(const Sums& S, double A21[21], double b6[6]) {
  int k = 0;
  for (int u = 0; u < 6; ++u)
    for (int v = u; v < 6; ++v) A21[k++] = S.A[6 * u + v];
  for (int u = 0; u < 6; ++u) b6[u] = S.b[u];
}

bool bad_args(const float* src, int64_t n_src, const float* tgt, int64_t n_tgt, double r) {
  return !src || !tgt || n_src < 1 || n_tgt < 1 || !(r > 0.0) || !std::isfinite(r);
}

// ---------------------------------------------------------------- normals
// Cyclic Jacobi eigenvalue iteration on a symmetric 3x3 matrix (Golub & Van
// Loan, Sec. 8.5): rotations zero each off-diagonal entry in turn until the
// off-diagonal mass is negligible.  On return A is (numerically) diagonal
// with the eigenvalues and the columns of V are the eigenvectors.
void jacobi3(double A[3][3], double V[3][3]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) V[r][c] = r == c ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-36 * diag || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        // rotation angle from tan(2 phi) = 2 a_pq / (a_qq - a_pp)
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0);
        const double sn = t * c;
        // A <- J^T A J, V <- V J with J the rotation in the (p, q) plane
        for (int k = 0; k < 3; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
}

// Normal of point i from its neighbourhood (original indices nb[0..m));
// evals (or null) receives the covariance eigenvalues, ascending.
void normal_of(const float* pts, const int64_t* nb, int m, const float pi[3], const double view[3],
               float out[3], double* evals) {
  if (m < 3) {
    out[0] = out[1] = out[2] = 0.0f;
    if (evals) evals[0] = evals[1] = evals[2] = 0.0;
    return;
  }
  double mu[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < m; ++k)
    for (int a = 0; a < 3; ++a) mu[a] += (double)pts[3 * nb[k] + a];
  for (int a = 0; a < 3; ++a) mu[a] /= (double)m;
  double C[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int k = 0; k < m; ++k) {
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = (double)pts[3 * nb[k] + a] - mu[a];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[r][c] += d[r] * d[c];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) C[r][c] /= (double)m;
  double V[3][3];
  jacobi3(C, V);
  int lo = 0;
  for (int a = 1; a < 3; ++a)
    if (C[a][a] < C[lo][lo]) lo = a;
  if (evals) {
    double e[3] = {C[0][0], C[1][1], C[2][2]};
    std::sort(e, e + 3);
    for (int a = 0; a < 3; ++a) evals[a] = e[a];
  }
  double n[3] = {V[0][lo], V[1][lo], V[2][lo]};
  const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int a = 0; a < 3; ++a) n[a] /= len;
  double dot = 0.0;
  for (int a = 0; a < 3; ++a) dot += n[a] * (view[a] - (double)pi[a]);
  if (dot < 0.0)
    for (int a = 0; a < 3; ++a) n[a] = -n[a];
  for (int a = 0; a < 3; ++a) out[a] = (float)n[a];
}

}  // namespace

extern "C" {

int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

// Pinned FP32 squared distances of n (s, p) pairs under T (test of the
// pinned expression itself).
void oracle_pinned_d2(const double T[16], const float* s, const float* p, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) {
    double q[3];
    transform64(T, s + 3 * i, q);
    const float q32[3] = {(float)q[0], (float)q[1], (float)q[2]};
    out[i] = pinned_d2(q32, p + 3 * i);
  }
}

void oracle_transform64(const double T[16], const float* s, int64_t n, double* q_out) {
  for (int64_t i = 0; i < n; ++i) transform64(T, s + 3 * i, q_out + 3 * i);
}

void oracle_se3_exp(const double xi[6], double E[16]) { se3_exp(xi, E); }

int oracle_residual_jacobian(int variant, const double q[3], const double p[3], const double n[3],
                             double res[3], double J[18]) {
  return residual_jacobian(variant, q, p, n, res, J);
}

int oracle_solve6(const double A21[21], const double b6[6], double xi[6]) {
  double Aup[36] = {};
  int k = 0;
  for (int u = 0; u < 6; ++u)
    for (int v = u; v < 6; ++v) Aup[6 * u + v] = A21[k++];
  return solve6(Aup, b6, xi) ? 0 : 1;
}

// Correspondences at T.  search: 0 = automatic (brute force when
// n_src * n_tgt <= 2e7), 1 = brute force, 2 = k-d tree.  idx = -1 when no
// target point lies within r.  d2f = pinned FP32 distance (PINNED_FP32 mode,
// +inf otherwise or when none), d2d = FP64 distance of the match.
int oracle_correspondences(const float* src, int64_t n_src, const double T[16], const float* tgt,
                           int64_t n_tgt, double r, int selection, int search, int64_t* idx_out,
                           float* d2f_out, double* d2d_out) {
  if (bad_args(src, n_src, tgt, n_tgt, r)) return -1;
  const bool tree = search == 2 || (search == 0 && (double)n_src * (double)n_tgt > 2e7);
  Selector sel(tgt, n_tgt, r, selection, tree);
  Sums S;
  pass(sel, src, n_src, nullptr, T, kPointToPoint, &S, idx_out, d2f_out, d2d_out);
  return 0;
}

// Normal equations at T: A (upper triangle, 21, row-major), b (6), sum of FP64
// squared distances and the inlier count.
int oracle_normal_equations_robust(const float* src, int64_t n_src, const double T[16],
                                   const float* tgt, const float* tgt_n, int64_t n_tgt, double r,
                                   int variant, int selection, int search, int loss_kind,
                                   double loss_k, double A21[21], double b6[6], double* sum_d2,
                                   int64_t* n_in) {
  if (bad_args(src, n_src, tgt, n_tgt, r)) return -1;
  if (variant == kPointToPlane && !tgt_n) return -1;
  if (loss_kind < kLossNone || loss_kind > kLossCauchy || !(loss_k > 0.0)) return -1;
  const bool tree = search == 2 || (search == 0 && (double)n_src * (double)n_tgt > 2e7);
  Selector sel(tgt, n_tgt, r, selection, tree);
  Sums S;
  Loss L;
  L.kind = loss_kind;
  L.k = loss_k;
  pass(sel, src, n_src, tgt_n, T, variant, &S, nullptr, nullptr, nullptr, L);
  pack21(S, A21, b6);
  *sum_d2 = S.sd2;
  *n_in = S.n;
  return 0;
}

int oracle_normal_equations(const float* src, int64_t n_src, const double T[16], const float* tgt,
                            const float* tgt_n, int64_t n_tgt, double r, int variant, int selection,
                            int search, double A21[21], double b6[6], double* sum_d2,
                            int64_t* n_in) {
  return oracle_normal_equations_robust(src, n_src, T, tgt, tgt_n, n_tgt, r, variant, selection,
                                        search, kLossNone, 1.0, A21, b6, sum_d2, n_in);
}

// IRLS weight of a loss at residual magnitude s (exposed for its pins).
double oracle_loss_weight(int loss_kind, double loss_k, double s) {
  Loss L;
  L.kind = loss_kind;
  L.k = loss_k;
  return loss_weight(L, s);
}

// The ICP loop.  Pass k = 0..max_iter computes correspondences at T_k and the
// metrics (n_k, fitness_k, rmse_k); it stops at no inliers (DEGENERATE), at
// k == max_iter (OK), or when both relative changes are <= rel_tol (CONVERGED);
// otherwise it solves the normal equations (DEGENERATE on a failed pivot) and
// sets T_{k+1} = Exp(xi) T_k.  Optional trajectory outputs hold T_k, n_k and
// rmse_k for every executed pass (capacity max_iter + 1).
int oracle_icp_register_robust(const float* src, int64_t n_src, const float* tgt, const float* tgt_n,
                               int64_t n_tgt, const double T_init[16], double r, int32_t max_iter,
                               double rel_tol, int variant, int selection, int search,
                               int loss_kind, double loss_k, double T_out[16], double* fitness,
                               double* rmse, int64_t* n_inliers, int32_t* n_iter, int32_t* status,
                               double* traj_T, int64_t* traj_n, double* traj_rmse) {
  if (bad_args(src, n_src, tgt, n_tgt, r) || max_iter < 0 || !(rel_tol >= 0.0)) return -1;
  if (variant == kPointToPlane && !tgt_n) return -1;
  if (loss_kind < kLossNone || loss_kind > kLossCauchy || !(loss_k > 0.0)) return -1;
  Loss L;
  L.kind = loss_kind;
  L.k = loss_k;
  const bool tree = search == 2 || (search == 0 && (double)n_src * (double)n_tgt > 2e7);
  Selector sel(tgt, n_tgt, r, selection, tree);
  double T[16];
  std::memcpy(T, T_init, sizeof T);
  int64_t n_prev = 0;
  double e_prev = 0.0;
  for (int32_t k = 0;; ++k) {
    Sums S;
    pass(sel, src, n_src, tgt_n, T, variant, &S, nullptr, nullptr, nullptr, L);
    const int64_t nk = S.n;
    const double fk = (double)nk / (double)n_src;
    const double ek = nk > 0 ? std::sqrt(S.sd2 / (double)nk) : 0.0;
    if (traj_T) std::memcpy(traj_T + 16 * k, T, 16 * sizeof(double));
    if (traj_n) traj_n[k] = nk;
    if (traj_rmse) traj_rmse[k] = ek;
    int st = -1;
    if (nk == 0) {
      st = kStatusDegenerate;
    } else if (k == max_iter) {
      st = kStatusOk;
    } else if (k >= 1 && std::fabs((double)(nk - n_prev)) <= rel_tol * (double)n_prev &&
               std::fabs(ek - e_prev) <= rel_tol * e_prev) {
      st = kStatusConverged;
    } else {
      double xi[6];
      if (!solve6(S.A, S.b, xi)) {
        st = kStatusDegenerate;
      } else {
        double E[16];
        se3_exp(xi, E);
        matmul4(E, T, T);
      }
    }
    if (st >= 0) {
      std::memcpy(T_out, T, sizeof T);
      *fitness = fk;
      *rmse = ek;
      *n_inliers = nk;
      *n_iter = k;
      *status = st;
      return 0;
    }
    n_prev = nk;
    e_prev = ek;
  }
}

int oracle_icp_register(const float* src, int64_t n_src, const float* tgt, const float* tgt_n,
                        int64_t n_tgt, const double T_init[16], double r, int32_t max_iter,
                        double rel_tol, int variant, int selection, int search, double T_out[16],
                        double* fitness, double* rmse, int64_t* n_inliers, int32_t* n_iter,
                        int32_t* status, double* traj_T, int64_t* traj_n, double* traj_rmse) {
  return oracle_icp_register_robust(src, n_src, tgt, tgt_n, n_tgt, T_init, r, max_iter, rel_tol,
                                    variant, selection, search, kLossNone, 1.0, T_out, fitness, rmse,
                                    n_inliers, n_iter, status, traj_T, traj_n, traj_rmse);
}

// Voxel downsampling (Sec. 3.3, voxel_down_sample): voxel indices
// floor(((double)p - o) * (1 / voxel)) per axis with o the box minimum and
// dims = floor((max - o) / voxel) + 1, key = (cz * dy + cy) * dx + cx; output
// one point per occupied voxel in increasing key order: the float64 mean of
// its points summed in original-index order (rounded to float32) and, with
// normals, the normalised float64 sum of its normals (the first point's
// normal when that sum is shorter than 1e-12).  Returns the voxel count.
int64_t oracle_voxel_downsample(const float* pts, const float* nrm, int64_t n, double voxel,
                                float* out_pts, float* out_nrm) {
  if (!pts || n < 1 || !(voxel > 0.0)) return -1;
  double mn[3], mx[3];
  for (int a = 0; a < 3; ++a) mn[a] = mx[a] = pts[a];
  for (int64_t i = 1; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      mn[a] = std::min(mn[a], (double)pts[3 * i + a]);
      mx[a] = std::max(mx[a], (double)pts[3 * i + a]);
    }
  const double inv = 1.0 / voxel;
  int64_t dims[3];
  for (int a = 0; a < 3; ++a) dims[a] = (int64_t)std::floor((mx[a] - mn[a]) * inv) + 1;
  std::vector<uint64_t> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t c[3];
    for (int a = 0; a < 3; ++a) {
      c[a] = (int64_t)std::floor(((double)pts[3 * i + a] - mn[a]) * inv);
      c[a] = std::min(std::max(c[a], (int64_t)0), dims[a] - 1);
    }
    key[(size_t)i] = (uint64_t)((c[2] * dims[1] + c[1]) * dims[0] + c[0]);
  }
  std::vector<int64_t> order((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return key[(size_t)a] < key[(size_t)b]; });
  int64_t v = 0;
  for (int64_t s = 0; s < n;) {
    int64_t e = s;
    while (e < n && key[(size_t)order[(size_t)e]] == key[(size_t)order[(size_t)s]]) ++e;
    double sum[3] = {0.0, 0.0, 0.0}, ns[3] = {0.0, 0.0, 0.0};
    for (int64_t k = s; k < e; ++k) {
      const int64_t i = order[(size_t)k];
      for (int a = 0; a < 3; ++a) {
        sum[a] += (double)pts[3 * i + a];
        if (nrm) ns[a] += (double)nrm[3 * i + a];
      }
    }
    for (int a = 0; a < 3; ++a) out_pts[3 * v + a] = (float)(sum[a] / (double)(e - s));
    if (nrm && out_nrm) {
      const double len = std::sqrt((ns[0] * ns[0] + ns[1] * ns[1]) + ns[2] * ns[2]);
      for (int a = 0; a < 3; ++a)
        out_nrm[3 * v + a] = len < 1e-12 ? nrm[3 * order[(size_t)s] + a] : (float)(ns[a] / len);
    }
    ++v;
    s = e;
  }
  return v;
}

// Normals of the points of a cloud with the hybrid neighbourhood (radius,
// max_nn): of all n points, or of the nq points listed in queries (original
// indices) when queries is not null; output k belongs to query k.  counts
// receives each neighbourhood size, evals (or null) the covariance
// eigenvalues (3 per query, ascending).  search: 0 automatic, 1 brute force,
// 2 k-d tree.  Returns 0, or -1 on invalid arguments.
int oracle_estimate_normals(const float* pts, int64_t n, double radius, int max_nn,
                            const double view[3], int search, const int64_t* queries, int64_t nq,
                            float* normals, int32_t* counts, double* evals) {
  if (!pts || n < 1 || !(radius > 0.0) || max_nn < 1 || !view || !normals || !counts) return -1;
  if (!queries) nq = n;
  if (nq < 0) return -1;
  const bool use_tree = search == 2 || (search == 0 && n * nq > 20000000);
  KdTree tree;
  if (use_tree) tree.build(pts, n);
  const float r2f = (float)(radius * radius);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t q = 0; q < nq; ++q) {
    const int64_t i = queries ? queries[q] : q;
    const float* pi = pts + 3 * i;
    std::vector<std::pair<float, int64_t>> cand;
    auto visit = [&](int64_t j) {
      const float d = pinned_d2(pi, pts + 3 * j);
      if (d <= r2f) cand.push_back({d, j});
    };
    if (use_tree) {
      const double c[3] = {(double)pi[0], (double)pi[1], (double)pi[2]};
      tree.range(c, radius * radius * (1.0 + 1e-5), visit);
    } else {
      for (int64_t j = 0; j < n; ++j) visit(j);
    }
    std::sort(cand.begin(), cand.end());  // by (distance, original index)
    const int m = (int)std::min<size_t>(cand.size(), (size_t)max_nn);
    std::vector<int64_t> nb((size_t)m);
    for (int k = 0; k < m; ++k) nb[(size_t)k] = cand[(size_t)k].second;
    counts[q] = m;
    normal_of(pts, nb.data(), m, pi, view, normals + 3 * q, evals ? evals + 3 * q : nullptr);
  }
  return 0;
}

// Hybrid neighbourhoods (the selection of oracle_estimate_normals) of all n
// points: row i of idx (n x max_nn, original indices, -1 padded) lists the
// max_nn smallest (pinned float32 squared distance, index) within radius,
// the point itself included, in that order; counts[i] its length.
int oracle_hybrid_neighbors(const float* pts, int64_t n, double radius, int max_nn, int search,
                            int64_t* idx, int32_t* counts) {
  if (!pts || n < 1 || !(radius > 0.0) || max_nn < 1 || !idx || !counts) return -1;
  const bool use_tree = search == 2 || (search == 0 && n * n > 20000000);
  KdTree tree;
  if (use_tree) tree.build(pts, n);
  const float r2f = (float)(radius * radius);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    const float* pi = pts + 3 * i;
    std::vector<std::pair<float, int64_t>> cand;
    auto visit = [&](int64_t j) {
      const float d = pinned_d2(pi, pts + 3 * j);
      if (d <= r2f) cand.push_back({d, j});
    };
    if (use_tree) {
      const double c[3] = {(double)pi[0], (double)pi[1], (double)pi[2]};
      tree.range(c, radius * radius * (1.0 + 1e-5), visit);
    } else {
      for (int64_t j = 0; j < n; ++j) visit(j);
    }
    std::sort(cand.begin(), cand.end());
    const int m = (int)std::min<size_t>(cand.size(), (size_t)max_nn);
    for (int k = 0; k < max_nn; ++k) idx[i * max_nn + k] = k < m ? cand[(size_t)k].second : -1;
    counts[i] = m;
  }
  return 0;
}

// Eigen-decomposition used by the normals (exposed for its pins): A6 is the
// upper triangle (a00, a01, a02, a11, a12, a22); evals ascending, evecs
// their eigenvectors as columns of a row-major 3x3.
void oracle_sym_eig3(const double A6[6], double evals[3], double evecs[9]) {
  double A[3][3] = {{A6[0], A6[1], A6[2]}, {A6[1], A6[3], A6[4]}, {A6[2], A6[4], A6[5]}};
  double V[3][3];
  jacobi3(A, V);
  int ord[3] = {0, 1, 2};
  std::sort(ord, ord + 3, [&](int a, int b) { return A[a][a] < A[b][b]; });
  for (int k = 0; k < 3; ++k) {
    evals[k] = A[ord[k]][ord[k]];
    for (int r = 0; r < 3; ++r) evecs[3 * r + k] = V[r][ord[k]];
  }
}

}  // extern "C"
