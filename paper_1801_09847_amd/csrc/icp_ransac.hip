// Global registration on feature matches (paper Sec. 3.3, the RANSAC step of
// the pairwise workflow [17]): nearest-feature matching, hypothesis
// generation with the edge-length and distance checkers, validation of the
// surviving hypotheses, and the choice of the best one; the C ABI behind
// icp_feature_match, icp_ransac_validate and icp_ransac_register.
//
// The sequential loop (draw a sample, check it, fit, check again, validate,
// stop at the max_validation-th validated hypothesis) is run as data-parallel
// chunks: hypothesis h depends only on (seed, h) through a counter-based
// generator, so a chunk of hypotheses is checked by one thread each, an
// exclusive scan of the pass flags puts the survivors in iteration order,
// and the first max_validation of them are validated together, one block per
// (source tile, hypothesis).  The result equals the sequential loop's.

#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "icp_runtime.h"

using namespace icp;

namespace {

constexpr int kHypBlock = 256;
constexpr int kMinRansacN = 3, kMaxRansacN = 8;
constexpr int64_t kMaxChunk = int64_t(1) << 21;   // hypotheses per check launch (96 B of fit each)
constexpr int64_t kFirstChunk = int64_t(1) << 16;
constexpr int kFmBlock = 256;  // threads per feature-match block
constexpr int kFmQ = 2;        // queries per thread
constexpr int kFmTile = 64;    // target features staged in LDS at a time
constexpr int kMaxFeatureDim = 64;
constexpr int64_t kMaxRansacSrc = int64_t(1) << 23;  // keeps sumq below 2^63

// ---------------------------------------------------------------- Philox4x64-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten
// rounds of two 64x64->128-bit multiplies and a key schedule bumped by Weyl
// constants.  Block b of hypothesis h: counter (h, b, 0, 0), key (seed, 0).
__device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1,
                                     uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

struct HypArgs {
  const float* src;      // (n_src, 3) original order
  const float* tgt;      // (n_tgt, 3)
  const int32_t* corr;   // (n_src) target index per source point
  int64_t n_src, n_tgt;
  uint64_t seed;
  double sig2;           // sigma^2 of the edge-length checker (<= 0: off)
  double d2;             // d^2 of the distance checker (<= 0: off)
  int64_t h0;            // first hypothesis of the chunk
  int64_t count;         // hypotheses in the chunk
  uint32_t* flags;       // count + 1 words: 1 = passed; scanned in place
  double* Tc;            // [count][12]: the fit of each passing hypothesis
  // emission of the survivors (second launch)
  int64_t base;          // survivors before this chunk
  int32_t max_valid;
  double* T_list;        // [max_valid][16]
  int64_t* h_list;       // [max_valid]
};

template <int N>
struct Sample {  // float32 inputs; every use converts to float64
  float s[N][3];
  float t[N][3];
};

// Draw, match lookup and edge-length check of hypothesis h.
template <int N>
__device__ bool draw_sample(const HypArgs& a, int64_t h, Sample<N>& sm) {
  uint32_t id[N];
#pragma unroll
  for (int b = 0; b < (N + 3) / 4; ++b) {
    uint64_t z[4];
    philox4x64_10((uint64_t)h, (uint64_t)b, a.seed, 0ull, z);
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (4 * b + w < N) id[4 * b + w] = (uint32_t)(((z[w] >> 32) * (uint64_t)a.n_src) >> 32);
  }
  bool ok = true;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i + 1; j < N; ++j) ok = ok && id[i] != id[j];
  if (!ok) return false;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int32_t c = a.corr[id[k]];
    if (c < 0 || (int64_t)c >= a.n_tgt) return false;
    const float* ps = a.src + 3 * (size_t)id[k];
    const float* pt = a.tgt + 3 * (size_t)c;
    sm.s[k][0] = ps[0]; sm.s[k][1] = ps[1]; sm.s[k][2] = ps[2];
    sm.t[k][0] = pt[0]; sm.t[k][1] = pt[1]; sm.t[k][2] = pt[2];
  }
  if (a.sig2 > 0.0) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i + 1; j < N; ++j) {
        const double sx = (double)sm.s[i][0] - (double)sm.s[j][0];
        const double sy = (double)sm.s[i][1] - (double)sm.s[j][1];
        const double sz = (double)sm.s[i][2] - (double)sm.s[j][2];
        const double tx = (double)sm.t[i][0] - (double)sm.t[j][0];
        const double ty = (double)sm.t[i][1] - (double)sm.t[j][1];
        const double tz = (double)sm.t[i][2] - (double)sm.t[j][2];
        const double ds2 = (sx * sx + sy * sy) + sz * sz;
        const double dt2 = (tx * tx + ty * ty) + tz * tz;
        ok = ok && ds2 >= a.sig2 * dt2 && dt2 >= a.sig2 * ds2;
      }
  }
  return ok;
}

// One Jacobi rotation of the symmetric 4x4 A in the (P, Q) plane (Golub and
// Van Loan, the symmetric Schur step), accumulated into V.
template <int P, int Q>
__device__ inline void jacobi4(double (&A)[4][4], double (&V)[4][4]) {
  const double apq = A[P][Q];
  if (apq == 0.0) return;
  const double tau = (A[Q][Q] - A[P][P]) / (2.0 * apq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double akp = A[k][P], akq = A[k][Q];
    A[k][P] = c * akp - s * akq;
    A[k][Q] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double apk = A[P][k], aqk = A[Q][k];
    A[P][k] = c * apk - s * aqk;
    A[Q][k] = s * apk + c * aqk;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double vkp = V[k][P], vkq = V[k][Q];
    V[k][P] = c * vkp - s * vkq;
    V[k][Q] = s * vkp + c * vkq;
  }
}

// Rigid transform (no scale) minimising sum |R s + t - p|^2 over the sample:
// Horn's closed form, the rotation being the unit quaternion of the largest
// eigenvalue of the 4x4 matrix built from the cross-covariance of the
// centred points.  T: 3x4 row-major.
template <int N>
__device__ void rigid_fit(const Sample<N>& sm, double T[12]) {
  double cs[3] = {0.0, 0.0, 0.0}, ct[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cs[a] = cs[a] + (double)sm.s[k][a];
      ct[a] = ct[a] + (double)sm.t[k][a];
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cs[a] = cs[a] / N;
    ct[a] = ct[a] / N;
  }
  double M[3][3] = {};
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double u[3] = {(double)sm.s[k][0] - cs[0], (double)sm.s[k][1] - cs[1], (double)sm.s[k][2] - cs[2]};
    const double v[3] = {(double)sm.t[k][0] - ct[0], (double)sm.t[k][1] - ct[1], (double)sm.t[k][2] - ct[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) M[a][b] = M[a][b] + u[a] * v[b];
  }
  const double xx = M[0][0], xy = M[0][1], xz = M[0][2];
  const double yx = M[1][0], yy = M[1][1], yz = M[1][2];
  const double zx = M[2][0], zy = M[2][1], zz = M[2][2];
  double A[4][4] = {{xx + yy + zz, yz - zy, zx - xz, xy - yx},
                    {yz - zy, xx - yy - zz, xy + yx, zx + xz},
                    {zx - xz, xy + yx, -xx + yy - zz, yz + zy},
                    {xy - yx, zx + xz, yz + zy, -xx - yy + zz}};
  double V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
  for (int sweep = 0; sweep < 24; ++sweep) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      dia = dia + A[p][p] * A[p][p];
#pragma unroll
      for (int q = p + 1; q < 4; ++q) off = off + A[p][q] * A[p][q];
    }
    if (off <= 1e-32 * dia || off == 0.0) break;
    jacobi4<0, 1>(A, V);
    jacobi4<0, 2>(A, V);
    jacobi4<0, 3>(A, V);
    jacobi4<1, 2>(A, V);
    jacobi4<1, 3>(A, V);
    jacobi4<2, 3>(A, V);
  }
  // eigenvector of the largest diagonal entry (first of equals), selected
  // without a dynamic index so that A and V stay in registers
  double lam = A[0][0], q0 = V[0][0], qx = V[1][0], qy = V[2][0], qz = V[3][0];
#pragma unroll
  for (int p = 1; p < 4; ++p)
    if (A[p][p] > lam) {
      lam = A[p][p];
      q0 = V[0][p];
      qx = V[1][p];
      qy = V[2][p];
      qz = V[3][p];
    }
  const double nq = sqrt((q0 * q0 + qx * qx) + (qy * qy + qz * qz));
  q0 /= nq; qx /= nq; qy /= nq; qz /= nq;
  const double R[3][3] = {{q0 * q0 + qx * qx - qy * qy - qz * qz, 2.0 * (qx * qy - q0 * qz), 2.0 * (qx * qz + q0 * qy)},
                          {2.0 * (qx * qy + q0 * qz), q0 * q0 - qx * qx + qy * qy - qz * qz, 2.0 * (qy * qz - q0 * qx)},
                          {2.0 * (qx * qz - q0 * qy), 2.0 * (qy * qz + q0 * qx), q0 * q0 - qx * qx - qy * qy + qz * qz}};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    T[4 * r + 0] = R[r][0];
    T[4 * r + 1] = R[r][1];
    T[4 * r + 2] = R[r][2];
    T[4 * r + 3] = ct[r] - ((R[r][0] * cs[0] + R[r][1] * cs[1]) + R[r][2] * cs[2]);
  }
}

// Distance checker: every sampled pair within d after the fit.
template <int N>
__device__ bool distance_ok(const HypArgs& a, const Sample<N>& sm, const double T[12]) {
  if (!(a.d2 > 0.0)) return true;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double e[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double t = T[4 * r] * (double)sm.s[k][0];
      t = t + T[4 * r + 1] * (double)sm.s[k][1];
      t = t + T[4 * r + 2] * (double)sm.s[k][2];
      e[r] = (t + T[4 * r + 3]) - (double)sm.t[k][r];
    }
    ok = ok && ((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]) <= a.d2;
  }
  return ok;
}

template <int N>
__device__ bool hypothesis(const HypArgs& a, int64_t h, double T[12]) {
  Sample<N> sm;
  if (!draw_sample<N>(a, h, sm)) return false;
  rigid_fit<N>(sm, T);
  return distance_ok<N>(a, sm, T);
}

// Pass flags of a chunk (flags[count] = 0 so the in-place exclusive scan of
// count + 1 words ends with the chunk's total).
template <int N>
__global__ __launch_bounds__(kHypBlock) void hyp_check_kernel(HypArgs a) {
  const int64_t g = (int64_t)blockIdx.x * kHypBlock + threadIdx.x;
  if (g > a.count) return;
  uint32_t f = 0;
  if (g < a.count) {
    double T[12];
    if (hypothesis<N>(a, a.h0 + g, T)) {
      f = 1u;
#pragma unroll
      for (int k = 0; k < 12; ++k) a.Tc[12 * g + k] = T[k];
    }
  }
  a.flags[g] = f;
}

// After the scan: each survivor whose rank is below max_valid moves its fit
// to its rank.
__global__ __launch_bounds__(kHypBlock) void hyp_emit_kernel(HypArgs a) {
  const int64_t g = (int64_t)blockIdx.x * kHypBlock + threadIdx.x;
  if (g >= a.count) return;
  const uint32_t p = a.flags[g], p1 = a.flags[g + 1];
  if (p1 == p) return;
  const int64_t v = a.base + p;
  if (v >= a.max_valid) return;
  double* o = a.T_list + 16 * v;
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k] = a.Tc[12 * g + k];
  o[12] = 0.0; o[13] = 0.0; o[14] = 0.0; o[15] = 1.0;
  a.h_list[v] = a.h0 + g;
}

struct RansacOut {
  double T[16];
  int64_t count;
  uint64_t sumq;
  int64_t h;       // hypothesis index of the best
  int64_t v;       // its rank among the validated
  int64_t h_last;  // hypothesis index of the last validated one
};

__device__ inline bool better(int64_t c0, uint64_t q0, int64_t v0, int64_t c1, uint64_t q1, int64_t v1) {
  if (c0 != c1) return c0 > c1;
  if (q0 != q1) return q0 < q1;
  return v0 < v1;
}

// The lexicographic best (count desc, sumq asc, rank asc) of n validated
// hypotheses, with its transform, in one block.
__global__ __launch_bounds__(1024) void ransac_select_kernel(const int64_t* cnt, const uint64_t* sq, int64_t n,
                                                             const double* T_list, const int64_t* h_list,
                                                             RansacOut* out) {
  __shared__ int64_t sc[1024];
  __shared__ uint64_t sqs[1024];
  __shared__ int64_t sv[1024];
  int64_t bc = -1, bv = -1;
  uint64_t bq = ~0ull;
  for (int64_t v = threadIdx.x; v < n; v += 1024)
    if (bv < 0 || better(cnt[v], sq[v], v, bc, bq, bv)) {
      bc = cnt[v];
      bq = sq[v];
      bv = v;
    }
  sc[threadIdx.x] = bc;
  sqs[threadIdx.x] = bq;
  sv[threadIdx.x] = bv;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const int o = threadIdx.x + w;
      if (sv[o] >= 0 && (sv[threadIdx.x] < 0 || better(sc[o], sqs[o], sv[o], sc[threadIdx.x], sqs[threadIdx.x], sv[threadIdx.x]))) {
        sc[threadIdx.x] = sc[o];
        sqs[threadIdx.x] = sqs[o];
        sv[threadIdx.x] = sv[o];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 16) {
    const int64_t v = sv[0];
    out->T[threadIdx.x] = v >= 0 ? T_list[16 * v + threadIdx.x] : (threadIdx.x % 5 == 0 ? 1.0 : 0.0);
  }
  if (threadIdx.x == 0) {
    const int64_t v = sv[0];
    out->count = v >= 0 ? sc[0] : 0;
    out->sumq = v >= 0 ? sqs[0] : 0;
    out->v = v;
    out->h = v >= 0 ? h_list[v] : -1;
    out->h_last = n > 0 ? h_list[n - 1] : -1;
  }
}

// ---------------------------------------------------------------- feature matching
// Block (x, y): kFmBlock * kFmQ queries against target split y.  Each thread
// holds kFmQ queries (zero-padded to 4 * D4 dimensions: zeros add exact zeros
// to a float32 sum) and walks the split's targets staged in LDS, kFmTile at a
// time, so one LDS read of a target feeds kFmQ distances; each distance is
// accumulated dimension by dimension in float32 without FMA, and strict <
// over increasing j keeps the smallest index of equal distances.  Splits
// merge through a 64-bit atomic minimum of (distance bits, index): the order
// of non-negative float bit patterns is the numeric order.
template <int D4>
__global__ __launch_bounds__(kFmBlock) void feature_match_kernel(const float* __restrict__ fs, int64_t n_src,
                                                                 const float* __restrict__ ft, int64_t n_tgt,
                                                                 int dim, int64_t per_split,
                                                                 unsigned long long* __restrict__ keys) {
  __shared__ float4 tile[kFmTile][D4];
  float4 q[kFmQ][D4];
  int64_t qi[kFmQ];
#pragma unroll
  for (int u = 0; u < kFmQ; ++u) {
    qi[u] = ((int64_t)blockIdx.x * kFmQ + u) * kFmBlock + threadIdx.x;
#pragma unroll
    for (int k4 = 0; k4 < D4; ++k4) {
      float e[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = 4 * k4 + c;
        e[c] = (qi[u] < n_src && k < dim) ? fs[qi[u] * dim + k] : 0.f;
      }
      q[u][k4] = make_float4(e[0], e[1], e[2], e[3]);
    }
  }
  const int64_t j0 = (int64_t)blockIdx.y * per_split;
  const int64_t j1 = min(n_tgt, j0 + per_split);
  float best[kFmQ];
  int64_t bj[kFmQ];
#pragma unroll
  for (int u = 0; u < kFmQ; ++u) {
    best[u] = INFINITY;
    bj[u] = -1;
  }
  float* tf = reinterpret_cast<float*>(&tile[0][0]);
  for (int64_t jt = j0; jt < j1; jt += kFmTile) {
    __syncthreads();
    for (int e = threadIdx.x; e < kFmTile * D4 * 4; e += kFmBlock) {
      const int t = e / (D4 * 4), k = e % (D4 * 4);
      const int64_t j = jt + t;
      tf[e] = (j < j1 && k < dim) ? ft[j * dim + k] : 0.f;
    }
    __syncthreads();
    const int nt = (int)min<int64_t>(kFmTile, j1 - jt);
    for (int t = 0; t < nt; ++t) {
      float acc[kFmQ];
#pragma unroll
      for (int u = 0; u < kFmQ; ++u) acc[u] = 0.f;
#pragma unroll
      for (int k4 = 0; k4 < D4; ++k4) {
        const float4 b = tile[t][k4];
#pragma unroll
        for (int u = 0; u < kFmQ; ++u) {
          float d;
          d = q[u][k4].x - b.x; acc[u] = acc[u] + d * d;
          d = q[u][k4].y - b.y; acc[u] = acc[u] + d * d;
          d = q[u][k4].z - b.z; acc[u] = acc[u] + d * d;
          d = q[u][k4].w - b.w; acc[u] = acc[u] + d * d;
        }
      }
#pragma unroll
      for (int u = 0; u < kFmQ; ++u)
        if (acc[u] < best[u]) {
          best[u] = acc[u];
          bj[u] = jt + t;
        }
    }
  }
#pragma unroll
  for (int u = 0; u < kFmQ; ++u)
    if (qi[u] < n_src && bj[u] >= 0)
      atomicMin(&keys[qi[u]], ((unsigned long long)__float_as_uint(best[u]) << 32) | (unsigned long long)bj[u]);
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void feature_match_final_kernel(const unsigned long long* keys, int64_t n, int32_t* match,
                                           float* dist) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const unsigned long long k = keys[i];
  match[i] = k == ~0ull ? -1 : (int32_t)(uint32_t)k;
  if (dist) dist[i] = k == ~0ull ? INFINITY : __uint_as_float((uint32_t)(k >> 32));
}

template <int D4>
void launch_fm(dim3 grid, hipStream_t s, const float* fs, int64_t n_src, const float* ft, int64_t n_tgt,
               int dim, int64_t per, unsigned long long* keys) {
  hipLaunchKernelGGL(feature_match_kernel<D4>, grid, dim3(kFmBlock), 0, s, fs, n_src, ft, n_tgt, dim, per, keys);
}

hipError_t launch_feature_match(const float* fs, int64_t n_src, const float* ft, int64_t n_tgt, int dim,
                                unsigned long long* keys, int32_t* match, float* dist, hipStream_t s) {
  const int64_t nb = (n_src + 255) / 256;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)nb), dim3(256), 0, s, keys, n_src, ~0ull);
  if (n_tgt > 0) {
    const int64_t qb = (n_src + kFmBlock * kFmQ - 1) / (kFmBlock * kFmQ);
    const int64_t max_splits = (n_tgt + kFmTile - 1) / kFmTile;
    const int64_t splits = std::max<int64_t>(1, std::min<int64_t>(max_splits, (2048 + qb - 1) / qb));
    int64_t per = (n_tgt + splits - 1) / splits;
    per = (per + kFmTile - 1) / kFmTile * kFmTile;
    const int64_t ns = (n_tgt + per - 1) / per;
    const dim3 grid((unsigned)qb, (unsigned)ns);
    switch ((dim + 3) / 4) {
#define ICP_FM_CASE(D) \
  case D: launch_fm<D>(grid, s, fs, n_src, ft, n_tgt, dim, per, keys); break;
      ICP_FM_CASE(1) ICP_FM_CASE(2) ICP_FM_CASE(3) ICP_FM_CASE(4) ICP_FM_CASE(5) ICP_FM_CASE(6)
      ICP_FM_CASE(7) ICP_FM_CASE(8) ICP_FM_CASE(9) ICP_FM_CASE(10) ICP_FM_CASE(11) ICP_FM_CASE(12)
      ICP_FM_CASE(13) ICP_FM_CASE(14) ICP_FM_CASE(15) ICP_FM_CASE(16)
#undef ICP_FM_CASE
      default: return hipErrorInvalidValue;
    }
  }
  hipLaunchKernelGGL(feature_match_final_kernel, dim3((unsigned)nb), dim3(256), 0, s, keys, n_src, match, dist);
  return hipGetLastError();
}

hipError_t launch_hyp(const HypArgs& a, int n, bool emit, hipStream_t s) {
  const dim3 grid((unsigned)((a.count + 1 + kHypBlock - 1) / kHypBlock));
  if (emit) {
    hipLaunchKernelGGL(hyp_emit_kernel, grid, dim3(kHypBlock), 0, s, a);
    return hipGetLastError();
  }
  switch (n) {
    case 3: hipLaunchKernelGGL(hyp_check_kernel<3>, grid, dim3(kHypBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL(hyp_check_kernel<4>, grid, dim3(kHypBlock), 0, s, a); break;
    case 5: hipLaunchKernelGGL(hyp_check_kernel<5>, grid, dim3(kHypBlock), 0, s, a); break;
    case 6: hipLaunchKernelGGL(hyp_check_kernel<6>, grid, dim3(kHypBlock), 0, s, a); break;
    case 7: hipLaunchKernelGGL(hyp_check_kernel<7>, grid, dim3(kHypBlock), 0, s, a); break;
    case 8: hipLaunchKernelGGL(hyp_check_kernel<8>, grid, dim3(kHypBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

namespace icp_rt {

namespace {

int check_features(const float* f, int64_t n, const char* name) {
  if (n < 0) return fail(ICP_E_INVALID_ARG, std::string(name) + ": count must be >= 0");
  if (n > (int64_t)INT32_MAX) return fail(ICP_E_TOO_LARGE, std::string(name) + ": more than 2^31-1 rows");
  if (n > 0 && !f) return fail(ICP_E_INVALID_ARG, std::string(name) + " is NULL");
  if ((reinterpret_cast<uintptr_t>(f) & 3u) != 0)
    return fail(ICP_E_INVALID_ARG, std::string(name) + " is not 4-byte aligned");
  return ICP_SUCCESS;
}

// ---- no-allocation feature match -----------------------------------------
// The scratch of icp_feature_match_noalloc: one 64-bit (distance, index) key
// per source feature, in a file-scope device array that every call on a
// device shares (each device holds its own copy).  Host code never names the
// array as a device address: its address on each device is looked up once,
// with that device current, and kept in g_noalloc_ptr.
constexpr int64_t kNoAllocMaxSrc = int64_t(1) << 20;  // 8 MiB of keys
static __device__ __align__(256) unsigned long long scratch[kNoAllocMaxSrc];
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned long long* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// The scratch address on the current device (looked up on its first use).
int noalloc_scratch(unsigned long long** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(ICP_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return fail(ICP_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_noalloc_ptr[dev] = static_cast<unsigned long long*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return ICP_SUCCESS;
}

int check_radius(double r) {
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite((float)(r * r)) || !((float)(r * r) > 0.0f))
    return fail(ICP_E_INVALID_ARG, "max_corr_dist must be > 0 with a finite, non-zero float32 square");
  return ICP_SUCCESS;
}

// 2^S with fl32(r^2) = m 2^e, m in [0.5, 1), S = 40 - e: every inlier's
// floor(d2 * 2^S) is below 2^40.
int score_shift(double r) {
  int e = 0;
  (void)frexp((double)(float)(r * r), &e);
  return 40 - e;
}

// Device workspace of one RANSAC / validation call, carved from ctx->rs.
struct RsLayout {
  size_t flags, Tc, sums, T_list, h_list, cnt, sq, part_cnt, part_sq, Tdev, out, total;
};

RsLayout rs_layout(int64_t chunk, int64_t max_valid, int64_t part_entries) {
  RsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align256(off);
    off = o + bytes;
    return o;
  };
  L.flags = take(sizeof(uint32_t) * (size_t)(chunk + 4));
  L.Tc = take(sizeof(double) * 12 * (size_t)chunk);
  L.sums = take(sizeof(uint32_t) * (size_t)scan_block_sums_needed(chunk + 1));
  L.T_list = take(sizeof(double) * 16 * (size_t)max_valid);
  L.h_list = take(sizeof(int64_t) * (size_t)max_valid);
  L.cnt = take(sizeof(int64_t) * (size_t)max_valid);
  L.sq = take(sizeof(uint64_t) * (size_t)max_valid);
  L.part_cnt = take(sizeof(uint32_t) * (size_t)part_entries);
  L.part_sq = take(sizeof(uint64_t) * (size_t)part_entries);
  L.Tdev = take(sizeof(double) * 12 * (size_t)max_valid);
  L.out = take(sizeof(RansacOut));
  L.total = align256(off);
  return L;
}

// Hypotheses validated per launch so that the per-tile partials stay below
// 64 MiB.
int64_t validate_batch(int64_t n_tiles) {
  return std::max<int64_t>(1, std::min<int64_t>(kMaxValidateHyp, (int64_t(64) << 20) / (12 * n_tiles)));
}

// Scores hypotheses [0, n) whose 3x4 transforms are at Tdev (12 doubles each)
// into cnt / sq, in batches; times the validation launches when profiling.
int validate_all(icp_ctx* c, const Prep& P, double r, const double* Tdev, int64_t n, char* base,
                 const RsLayout& L, int64_t* cnt, uint64_t* sq) {
  hipStream_t s = c->stream;
  const int64_t n_tiles = tiles_of(P.src_off[1]);
  const int64_t batch = validate_batch(n_tiles);
  const int S = score_shift(r);
  const bool prof = c->profiling;
  if (prof) {
    const size_t need = 2 + 2 * (size_t)((n + batch - 1) / batch);
    while (c->ev.size() < need) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e), "hipEventCreate");
      c->ev.push_back(e);
    }
  }
  int launches = 0;
  for (int64_t v0 = 0; v0 < n; v0 += batch) {
    ValidateArgs a;
    memset(&a, 0, sizeof a);
    PassArgs& p = a.p;
    p.sx = c->sx.as<float>();
    p.sy = c->sy.as<float>();
    p.sz = c->sz.as<float>();
    p.sperm = c->perm.as<uint32_t>();
    p.n_src = (int32_t)P.src_off[1];
    p.tp = c->tp.as<float4>();
    p.cs = c->cs.as<uint32_t>();
    p.g = P.g[0];
    p.r2f = (float)(r * r);
    p.inv_h2 = (float)(P.g[0].inv_h * P.g[0].inv_h);
    p.n_tgt = (int32_t)P.tgt_off[1];
    a.T = Tdev + 12 * v0;
    a.n_hyp = (int32_t)std::min<int64_t>(batch, n - v0);
    a.n_tiles = (int32_t)n_tiles;
    a.scale = ldexp(1.0, S);
    a.part_cnt = reinterpret_cast<uint32_t*>(base + L.part_cnt);
    a.part_sq = reinterpret_cast<uint64_t*>(base + L.part_sq);
    a.cnt_out = cnt + v0;
    a.sq_out = sq + v0;
    if (prof) HIP_TRY(hipEventRecord(c->ev[2 + 2 * launches], s), "hipEventRecord");
    HIP_TRY(launch_validate(a, P.g[0].sub, s), "validate");
    if (prof) HIP_TRY(hipEventRecord(c->ev[3 + 2 * launches], s), "hipEventRecord");
    ++launches;
  }
  if (prof && launches) {
    HIP_TRY(hipStreamSynchronize(s), "sync");
    for (int k = 0; k < launches; ++k) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, c->ev[2 + 2 * k], c->ev[3 + 2 * k]), "hipEventElapsedTime");
      c->prof.validate_ms += ms;
      c->prof.validate_launches += 1;
    }
    c->prof.validate_evals += n * P.src_off[1];
  }
  return ICP_SUCCESS;
}

// 3x4 rows of n host 4x4 transforms, staged for upload.
__global__ void pack_rows_kernel(const double* T16, int64_t n, double* T12) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= 12 * n) return;
  T12[i] = T16[16 * (i / 12) + i % 12];
}

}  // namespace

}  // namespace icp_rt

using namespace icp_rt;

extern "C" {

int icp_feature_match(icp_ctx_t* ctx, const float* src_feat, int64_t n_src, const float* tgt_feat,
                      int64_t n_tgt, int32_t dim, int32_t* match_out, float* dist_out) {
  int rc;
  if ((rc = check_features(src_feat, n_src, "src_feat")) != 0) return rc;
  if ((rc = check_features(tgt_feat, n_tgt, "tgt_feat")) != 0) return rc;
  if (dim < 1 || dim > kMaxFeatureDim)
    return fail(ICP_E_INVALID_ARG, "dim must be in [1, " + std::to_string(kMaxFeatureDim) + "]");
  if (n_src > 0 && !match_out) return fail(ICP_E_INVALID_ARG, "match_out is NULL");
  if ((reinterpret_cast<uintptr_t>(match_out) & 3u) || (reinterpret_cast<uintptr_t>(dist_out) & 3u))
    return fail(ICP_E_INVALID_ARG, "output pointer is not 4-byte aligned");
  if ((double)n_tgt * dim > 9.2e18 || (double)n_src * dim > 9.2e18)
    return fail(ICP_E_TOO_LARGE, "feature array too large");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  if (n_src == 0) return ICP_SUCCESS;
  DeviceGuard dg(c->device);
  HIP_TRY(c->rs.ensure(sizeof(unsigned long long) * (size_t)n_src), "hipMalloc");
  HIP_TRY(launch_feature_match(src_feat, n_src, tgt_feat, n_tgt, dim, c->rs.as<unsigned long long>(), match_out,
                               dist_out, c->stream),
          "feature match");
  HIP_TRY(hipStreamSynchronize(c->stream), "sync");
  return ICP_SUCCESS;
}

int icp_feature_match_noalloc(const float* src_feat, int64_t n_src, const float* tgt_feat, int64_t n_tgt,
                              int32_t dim, int32_t* match_out, float* dist_out, void* hip_stream) {
  int rc;
  if ((rc = check_features(src_feat, n_src, "src_feat")) != 0) return rc;
  if ((rc = check_features(tgt_feat, n_tgt, "tgt_feat")) != 0) return rc;
  if (dim < 1 || dim > kMaxFeatureDim)
    return fail(ICP_E_INVALID_ARG, "dim must be in [1, " + std::to_string(kMaxFeatureDim) + "]");
  if (n_src > 0 && !match_out) return fail(ICP_E_INVALID_ARG, "match_out is NULL");
  if ((reinterpret_cast<uintptr_t>(match_out) & 3u) || (reinterpret_cast<uintptr_t>(dist_out) & 3u))
    return fail(ICP_E_INVALID_ARG, "output pointer is not 4-byte aligned");
  if (n_src > kNoAllocMaxSrc)
    return fail(ICP_E_TOO_LARGE, "icp_feature_match_noalloc: n_src exceeds " + std::to_string(kNoAllocMaxSrc) +
                                     " (the size of its static scratch)");
  if ((double)n_tgt * dim > 9.2e18) return fail(ICP_E_TOO_LARGE, "feature array too large");
  unsigned long long* keys = nullptr;
  if ((rc = noalloc_scratch(&keys)) != 0) return rc;
  if (n_src == 0) return ICP_SUCCESS;
  // the keys are initialised by a fill kernel (not a memset) inside the launch
  HIP_TRY(launch_feature_match(src_feat, n_src, tgt_feat, n_tgt, dim, keys, match_out, dist_out,
                               static_cast<hipStream_t>(hip_stream)),
          "feature match");
  return ICP_SUCCESS;
}

int icp_compute_fpfh(icp_ctx_t* ctx, const float* pts, const float* normals, int64_t n, double radius,
                     int32_t max_nn, float* features_out, int32_t* nn_out) {
  int rc;
  if ((rc = check_cloud(pts, n, "pts")) != 0) return rc;
  if (!normals || (reinterpret_cast<uintptr_t>(normals) & 3u))
    return fail(ICP_E_INVALID_ARG, "normals is NULL or not 4-byte aligned");
  if (!(radius > 0.0) || !std::isfinite(radius) || !std::isfinite((float)(radius * radius)))
    return fail(ICP_E_INVALID_ARG, "radius must be > 0 with a finite float32 square");
  if (max_nn < 1 || max_nn > kMaxFpfhNN)
    return fail(ICP_E_INVALID_ARG, "max_nn must be in [1, " + std::to_string(kMaxFpfhNN) + "]");
  if (!features_out) return fail(ICP_E_INVALID_ARG, "features_out is NULL");
  if ((reinterpret_cast<uintptr_t>(features_out) & 3u) || (reinterpret_cast<uintptr_t>(nn_out) & 3u))
    return fail(ICP_E_INVALID_ARG, "output pointer is not 4-byte aligned");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const PairIn in{pts, n, pts, nullptr, n, radius};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align256(off);
    off = o + bytes;
    return o;
  };
  const size_t o_counts = take((size_t)kFpfhCountBytes * (size_t)n);
  const size_t o_k = take(sizeof(int32_t) * (size_t)n);
  const size_t o_nbr = take(sizeof(int32_t) * (size_t)max_nn * (size_t)n);
  const size_t o_nn = take(sizeof(int32_t) * (size_t)n);
  HIP_TRY(c->rs.ensure(align256(off)), "hipMalloc");
  char* base = c->rs.as<char>();
  FpfhArgs a;
  memset(&a, 0, sizeof a);
  a.sx = c->sx.as<float>();
  a.sy = c->sy.as<float>();
  a.sz = c->sz.as<float>();
  a.sperm = c->perm.as<uint32_t>();
  a.n = (int32_t)n;
  a.tp = c->tp.as<float4>();
  a.cs = c->cs.as<uint32_t>();
  a.g = P.g[0];
  a.r2f = (float)(radius * radius);
  a.inv_h2 = (float)(P.g[0].inv_h * P.g[0].inv_h);
  a.max_nn = max_nn;
  a.pts = pts;
  a.nrm = normals;
  a.counts = reinterpret_cast<uint8_t*>(base + o_counts);
  a.k = reinterpret_cast<int32_t*>(base + o_k);
  a.nbr = reinterpret_cast<int32_t*>(base + o_nbr);
  a.nn = nn_out ? nn_out : reinterpret_cast<int32_t*>(base + o_nn);
  a.out = features_out;
  HIP_TRY(launch_fpfh(a, P.g[0].sub, c->stream), "fpfh");
  HIP_TRY(hipStreamSynchronize(c->stream), "sync");
  return ICP_SUCCESS;
}

int icp_ransac_validate(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const float* tgt_xyz,
                        int64_t n_tgt, double max_corr_dist, int32_t n_hyp, const double* T,
                        int64_t* count_out, uint64_t* sumq_out) {
  int rc;
  if ((rc = check_cloud(src_xyz, n_src, "src")) != 0) return rc;
  if ((rc = check_cloud(tgt_xyz, n_tgt, "tgt")) != 0) return rc;
  if (n_src > kMaxRansacSrc) return fail(ICP_E_TOO_LARGE, "src: more than 2^23 points");
  if ((rc = check_radius(max_corr_dist)) != 0) return rc;
  if (n_hyp < 1 || n_hyp > kMaxValidateHyp)
    return fail(ICP_E_INVALID_ARG, "n_hyp must be in [1, " + std::to_string(kMaxValidateHyp) + "]");
  if (!T || !count_out || !sumq_out) return fail(ICP_E_INVALID_ARG, "T / count_out / sumq_out is NULL");
  for (int32_t v = 0; v < n_hyp; ++v)
    if ((rc = check_pose(T + 16 * (size_t)v, "T")) != 0) {
      g_last_error += " (hypothesis " + std::to_string(v) + ")";
      return rc;
    }
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const PairIn in{src_xyz, n_src, tgt_xyz, nullptr, n_tgt, max_corr_dist};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  const int64_t n_tiles = tiles_of(n_src);
  const RsLayout L = rs_layout(0, n_hyp, validate_batch(n_tiles) * n_tiles);
  const size_t tbytes = sizeof(double) * 16 * (size_t)n_hyp;
  HIP_TRY(c->rs.ensure(L.total + tbytes), "hipMalloc");
  const size_t io = sizeof(int64_t) * 2 * (size_t)n_hyp;
  if ((rc = ensure_host(c, std::max(tbytes, io))) != 0) return rc;
  char* base = c->rs.as<char>();
  double* T16 = reinterpret_cast<double*>(base + L.total);
  hipStream_t s = c->stream;
  memcpy(c->host, T, tbytes);
  HIP_TRY(hipMemcpyAsync(T16, c->host, tbytes, hipMemcpyHostToDevice, s), "upload");
  double* T12 = reinterpret_cast<double*>(base + L.Tdev);
  hipLaunchKernelGGL(pack_rows_kernel, dim3((unsigned)((12 * n_hyp + 255) / 256)), dim3(256), 0, s, T16,
                     (int64_t)n_hyp, T12);
  HIP_TRY(hipGetLastError(), "pack");
  int64_t* cnt = reinterpret_cast<int64_t*>(base + L.cnt);
  uint64_t* sq = reinterpret_cast<uint64_t*>(base + L.sq);
  if ((rc = validate_all(c, P, max_corr_dist, T12, n_hyp, base, L, cnt, sq)) != 0) return rc;
  char* h = static_cast<char*>(c->host);
  HIP_TRY(hipMemcpyAsync(h, cnt, sizeof(int64_t) * n_hyp, hipMemcpyDeviceToHost, s), "readback");
  HIP_TRY(hipMemcpyAsync(h + sizeof(int64_t) * n_hyp, sq, sizeof(uint64_t) * n_hyp, hipMemcpyDeviceToHost, s),
          "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  memcpy(count_out, h, sizeof(int64_t) * n_hyp);
  memcpy(sumq_out, h + sizeof(int64_t) * n_hyp, sizeof(uint64_t) * n_hyp);
  return ICP_SUCCESS;
}

int icp_ransac_register(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const float* tgt_xyz, int64_t n_tgt,
                        const int32_t* corr, const icp_ransac_params_t* prm, icp_ransac_result_t* out,
                        const icp_ransac_trace_t* trace) {
  int rc;
  if ((rc = check_cloud(src_xyz, n_src, "src")) != 0) return rc;
  if ((rc = check_cloud(tgt_xyz, n_tgt, "tgt")) != 0) return rc;
  if (n_src > kMaxRansacSrc) return fail(ICP_E_TOO_LARGE, "src: more than 2^23 points");
  if (!corr || (reinterpret_cast<uintptr_t>(corr) & 3u))
    return fail(ICP_E_INVALID_ARG, "corr is NULL or not 4-byte aligned");
  if (!prm || !out) return fail(ICP_E_INVALID_ARG, "params / out is NULL");
  if ((rc = check_radius(prm->max_corr_dist)) != 0) return rc;
  if (prm->ransac_n < kMinRansacN || prm->ransac_n > kMaxRansacN)
    return fail(ICP_E_INVALID_ARG, "ransac_n must be in [3, 8]");
  if (!std::isfinite(prm->edge_length) || !std::isfinite(prm->distance))
    return fail(ICP_E_INVALID_ARG, "edge_length / distance must be finite (<= 0: checker off)");
  if (prm->max_iteration < 1) return fail(ICP_E_INVALID_ARG, "max_iteration must be >= 1");
  if (prm->max_validation < 1 || prm->max_validation > kMaxValidateHyp)
    return fail(ICP_E_INVALID_ARG, "max_validation must be in [1, " + std::to_string(kMaxValidateHyp) + "]");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const double r = prm->max_corr_dist;
  const PairIn in{src_xyz, n_src, tgt_xyz, nullptr, n_tgt, r};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  hipStream_t s = c->stream;
  const int64_t max_valid = prm->max_validation;
  const int64_t chunk_cap = std::min<int64_t>(kMaxChunk, prm->max_iteration);
  const int64_t n_tiles = tiles_of(n_src);
  const RsLayout L = rs_layout(chunk_cap, max_valid, validate_batch(n_tiles) * n_tiles);
  HIP_TRY(c->rs.ensure(L.total), "hipMalloc");
  if ((rc = ensure_host(c, sizeof(RansacOut) + 64)) != 0) return rc;
  char* base = c->rs.as<char>();
  HypArgs a;
  memset(&a, 0, sizeof a);
  a.src = src_xyz;
  a.tgt = tgt_xyz;
  a.corr = corr;
  a.n_src = n_src;
  a.n_tgt = n_tgt;
  a.seed = prm->seed;
  a.sig2 = prm->edge_length > 0.0 ? prm->edge_length * prm->edge_length : 0.0;
  a.d2 = prm->distance > 0.0 ? prm->distance * prm->distance : 0.0;
  a.flags = reinterpret_cast<uint32_t*>(base + L.flags);
  a.Tc = reinterpret_cast<double*>(base + L.Tc);
  a.max_valid = (int32_t)max_valid;
  a.T_list = reinterpret_cast<double*>(base + L.T_list);
  a.h_list = reinterpret_cast<int64_t*>(base + L.h_list);
  uint32_t* sums = reinterpret_cast<uint32_t*>(base + L.sums);
  uint32_t* hflag = static_cast<uint32_t*>(c->host);

  // hypothesis chunks until max_validation survivors: after the first, each
  // chunk is sized from the survivor rate so far to finish in one more
  // (at most kMaxChunk); the result does not depend on the chunking
  int64_t valid = 0, h0 = 0, chunk = std::min<int64_t>(kFirstChunk, chunk_cap);
  while (h0 < prm->max_iteration && valid < max_valid) {
    const int64_t cnt = std::min<int64_t>(chunk, prm->max_iteration - h0);
    a.h0 = h0;
    a.count = cnt;
    a.base = valid;
    HIP_TRY(launch_hyp(a, prm->ransac_n, false, s), "hypothesis check");
    HIP_TRY(launch_scan_exclusive(a.flags, cnt + 1, sums, scan_block_sums_needed(chunk_cap + 1), s), "scan");
    HIP_TRY(launch_hyp(a, prm->ransac_n, true, s), "hypothesis emit");
    HIP_TRY(hipMemcpyAsync(hflag, a.flags + cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "readback");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    valid += *hflag;
    h0 += cnt;
    if (valid < max_valid) {
      const double rate = (double)valid / (double)h0;
      const double want = rate > 0.0 ? 1.25 * (double)(max_valid - valid) / rate + 1024.0 : (double)chunk_cap;
      chunk = std::min<int64_t>(chunk_cap, std::max<int64_t>(kFirstChunk, (int64_t)std::min(want, 1e18)));
    }
  }
  const int64_t n_val = std::min<int64_t>(valid, max_valid);

  // validation of the first max_validation survivors, then the best
  int64_t* cnt = reinterpret_cast<int64_t*>(base + L.cnt);
  uint64_t* sq = reinterpret_cast<uint64_t*>(base + L.sq);
  double* T12 = reinterpret_cast<double*>(base + L.Tdev);
  if (n_val > 0) {
    hipLaunchKernelGGL(pack_rows_kernel, dim3((unsigned)((12 * n_val + 255) / 256)), dim3(256), 0, s, a.T_list,
                       n_val, T12);
    HIP_TRY(hipGetLastError(), "pack");
    if ((rc = validate_all(c, P, r, T12, n_val, base, L, cnt, sq)) != 0) return rc;
  }
  RansacOut* dout = reinterpret_cast<RansacOut*>(base + L.out);
  hipLaunchKernelGGL(ransac_select_kernel, dim3(1), dim3(1024), 0, s, cnt, sq, n_val, a.T_list, a.h_list, dout);
  HIP_TRY(hipGetLastError(), "select");
  if (trace) {
    if (trace->h) HIP_TRY(hipMemcpyAsync(trace->h, a.h_list, sizeof(int64_t) * n_val, hipMemcpyDeviceToDevice, s), "trace");
    if (trace->T) HIP_TRY(hipMemcpyAsync(trace->T, a.T_list, sizeof(double) * 16 * n_val, hipMemcpyDeviceToDevice, s), "trace");
    if (trace->count) HIP_TRY(hipMemcpyAsync(trace->count, cnt, sizeof(int64_t) * n_val, hipMemcpyDeviceToDevice, s), "trace");
    if (trace->sumq) HIP_TRY(hipMemcpyAsync(trace->sumq, sq, sizeof(uint64_t) * n_val, hipMemcpyDeviceToDevice, s), "trace");
  }
  RansacOut* hout = static_cast<RansacOut*>(c->host);
  HIP_TRY(hipMemcpyAsync(hout, dout, sizeof(RansacOut), hipMemcpyDeviceToHost, s), "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  const int S = score_shift(r);
  icp_ransac_result_t res{};
  memcpy(res.T, hout->T, sizeof res.T);
  res.n_inliers = hout->count;
  res.sumq = hout->sumq;
  res.shift = S;
  res.fitness = (double)hout->count / (double)n_src;
  res.inlier_rmse = hout->count > 0 ? sqrt(ldexp((double)hout->sumq, -S) / (double)hout->count) : 0.0;
  res.best_hypothesis = hout->h;
  res.n_validated = n_val;
  res.n_iterations = valid >= max_valid ? hout->h_last + 1 : prm->max_iteration;
  res.status = n_val > 0 ? ICP_OK : ICP_RANSAC_NO_HYPOTHESIS;
  *out = res;
  return ICP_SUCCESS;
}

}  // extern "C"
