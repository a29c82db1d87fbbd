// HIP kernels of the ICP registration loop for CDNA4 (gfx950, wave64): the
// per-iteration pass (correspondence + normal equations) and the solve /
// pose update.  The grid and source ordering they consume are built by the
// kernels in icp_build.hip.
//
// Method: Open3D paper Sec. 3.3 (ICP refinement with a maximum
// correspondence distance, point-to-plane / point-to-point) and Sec. 4
// (Gauss-Newton step of eq. (2) with J^T J and J^T r built by a parallel
// reduction over per-correspondence terms).  The paper's nearest-neighbour
// search is a CPU k-d tree; here it is a dense uniform grid over the target
// (cell edge >= max_corr_dist, 27-cell neighbourhood) built by a counting
// sort of cell keys, and the source is ordered along a Morton curve so that a
// wavefront's queries touch the same cells.
//
// Every kernel is compiled with floating-point contraction disabled: the
// correspondence distance must be the exact float32 expression the interface
// specifies, and the transform the exact float64 one.

#include <float.h>
#include <math.h>

#include <algorithm>
#include <utility>

#include "icp_internal.h"

#pragma clang fp contract(off)

namespace icp {

namespace {

constexpr int kWave = 64;
constexpr int kRounds = kTile / kBlock;  // queries per thread in one pass launch
static_assert(kRounds * kBlock == kTile, "tile size");

__device__ inline int lane_id() { return __lane_id(); }

// Global-address-space view of a pointer.  Arguments that arrive through a
// struct in memory (batched and served launches) are otherwise generic
// pointers, which compile to FLAT accesses; FLAT loads share the LDS wait
// counter and serialise this kernel's LDS and memory waits.
#define ICP_G __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ ICP_G T* glb(T* p) {
  return (ICP_G T*)(p);
}
// float4 has a user-declared copy constructor on a generic reference, so a
// global-space element is read as a clang vector and repacked.
typedef float icp_f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4(const float4* p, int64_t i) {
  const icp_f4v v = ((const ICP_G icp_f4v*)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}

// Cell-start table entry: the table holds fewer than 2^30 entries, so the
// byte offset fits 32 bits and the load takes the scalar-base + 32-bit
// vector-offset form.
__device__ __forceinline__ uint32_t ld_cell(const uint32_t* cs, uint32_t idx) {
  const ICP_G char* b = (const ICP_G char*)(cs);
  return *(const ICP_G uint32_t*)(b + (uint32_t)(idx << 2));
}

// ------------------------------------------------------------------ small helpers
template <class T>
__device__ inline T wave_sum_xor(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = v + __shfl_xor(v, off, kWave);
  return v;
}

// Exact error-free sum: s + e == a + b exactly (Knuth TwoSum).
__device__ inline void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  const float aa = s - bb;
  e = (a - aa) + (b - bb);
}

struct Mat16 {
  double v[16];
};

// ------------------------------------------------------------------ loop state
__global__ void state_init_kernel(IterState* st, Mat16 T) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < 16; ++k) st->T[k] = T.v[k];
    st->fitness = 0.0;
    st->rmse = 0.0;
    st->e_prev = 0.0;
    st->n_in = 0;
    st->n_prev = 0;
    st->k = 0;
    st->done = 0;
    st->status = 0;
    st->pad = 0;
  }
}

// ------------------------------------------------------------------ correspondence + normal equations
// Per-correspondence terms: 21 entries of J^T J (upper, row-major), 6 of J^T r,
// the squared distance.  Point-to-plane: one row J = [q x n, n], r = n . d.
// Point-to-point: three rows J_a = [-[q]_x row a, e_a], r = d, summed in
// closed form: J^T J = [[|q|^2 I - q q^T, [q]_x], [[q]_x^T, I]],
// J^T r = [q x d, d].
template <int VAR, class F>
__device__ inline void record_terms(F qx, F qy, F qz, F rx, F ry, F rz, F nx, F ny, F nz, F* v) {
  if (VAR == 1) {
    const F res = (nx * rx + ny * ry) + nz * rz;
    const F J[6] = {qy * nz - qz * ny, qz * nx - qx * nz, qx * ny - qy * nx, nx, ny, nz};
    int k = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u)
#pragma unroll
      for (int w = u; w < 6; ++w) v[k++] = J[u] * J[w];
#pragma unroll
    for (int u = 0; u < 6; ++u) v[21 + u] = J[u] * res;
  } else {
    const F xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const F one = F(1), zero = F(0);
    // row 0: (yy+zz, -xy, -xz, 0, -z, y)
    v[0] = yy + zz; v[1] = -(qx * qy); v[2] = -(qx * qz); v[3] = zero; v[4] = -qz; v[5] = qy;
    // row 1: (xx+zz, -yz, z, 0, -x)
    v[6] = xx + zz; v[7] = -(qy * qz); v[8] = qz; v[9] = zero; v[10] = -qx;
    // row 2: (xx+yy, -y, x, 0)
    v[11] = xx + yy; v[12] = -qy; v[13] = qx; v[14] = zero;
    // rows 3..5: identity
    v[15] = one; v[16] = zero; v[17] = zero; v[18] = one; v[19] = zero; v[20] = one;
    v[21] = qy * rz - qz * ry;
    v[22] = qz * rx - qx * rz;
    v[23] = qx * ry - qy * rx;
    v[24] = rx; v[25] = ry; v[26] = rz;
  }
}

// IRLS weight rho'(s) / s of the robust loss at residual magnitude s >= 0:
// Huber 1 (s <= k) or k / s; Tukey (1 - (s/k)^2)^2 (s <= k) or 0; Cauchy
// 1 / (1 + (s/k)^2).  A query without a correspondence has s = 0 and w = 1.
template <class F>
__device__ inline F loss_weight(int kind, F k, F s) {
  if (kind == 1) return s <= k ? F(1) : k / s;
  if (kind == 2) {
    if (s > k) return F(0);
    const F u = F(1) - (s / k) * (s / k);
    return u * u;
  }
  if (kind == 3) return F(1) / (F(1) + (s / k) * (s / k));
  return F(1);
}

// Correspondence search of one query on the dense grid (cells of edge
// h >= r (1 + 2^-10) / R, neighbourhood of (2R+1)^3 cells).  Cells are pruned
// when their box lies farther from the query than the best distance known so
// far (the previous pass's match when a warm start is available, else r); the
// bound is conservative (relative margin 1e-4 on the squared distance, 1e-5
// cell on each gap) so no candidate that could win under the float32 pinned
// distance is dropped.  Candidates of one (dy, dz) row are contiguous in the
// cell-ordered target, so each surviving row is one index range; the ranges of
// a lane are staged in LDS and scanned as a single flattened loop so that the
// wavefront runs max(candidates) iterations instead of a sum over rows of the
// per-row maximum.
// Cell of a query (clamped to R + 1 cells around the grid) and its position
// inside the cell, from the float32 query in float64.
struct QueryCell {
  int cx, cy, cz;
  float fx, fy, fz;
};

template <int R>
__device__ inline QueryCell query_cell(const GridDesc& g, float q32x, float q32y, float q32z) {
  const double lo = -(double)R - 1.0;
  double ux = ((double)q32x - g.ox) * g.inv_h;
  double uy = ((double)q32y - g.oy) * g.inv_h;
  double uz = ((double)q32z - g.oz) * g.inv_h;
  ux = fmin(fmax(ux, lo), (double)g.dx + R);
  uy = fmin(fmax(uy, lo), (double)g.dy + R);
  uz = fmin(fmax(uz, lo), (double)g.dz + R);
  const double flx = floor(ux), fly = floor(uy), flz = floor(uz);
  QueryCell c;
  c.cx = (int)flx; c.cy = (int)fly; c.cz = (int)flz;
  c.fx = (float)(ux - flx); c.fy = (float)(uy - fly); c.fz = (float)(uz - flz);
  return c;
}

// The dilated-occupancy-bitmap word and bit of a query's cell: the bit is set
// when any target lies in the 27 cells around it.  The cell is clamped into
// the grid first: along each axis the clamped cell's neighbours include every
// in-grid neighbour of the query's own cell, so a clear bit proves that the
// query has no candidate (with R = 1; for R = 2 the bitmap is not used).
// Returns false (no word to read, no candidate) for a cell more than one cell
// outside the grid, which has no neighbour in it.
__device__ inline bool occupancy_word(const PassArgs& a, const QueryCell& c, uint32_t* word, uint32_t* bit) {
  const GridDesc& g = a.g;
  if (c.cx < -1 || c.cx > g.dx || c.cy < -1 || c.cy > g.dy || c.cz < -1 || c.cz > g.dz) return false;
  const uint32_t x = (uint32_t)min(max(c.cx, 0), g.dx - 1);
  const uint32_t y = (uint32_t)min(max(c.cy, 0), g.dy - 1);
  const uint32_t z = (uint32_t)min(max(c.cz, 0), g.dz - 1);
  if (g.hashed) {
    const uint32_t slot = hashed_slot(g, (int32_t)x, (int32_t)y, (int32_t)z);
    *word = slot >> 5;
    *bit = 1u << (slot & 31u);
    return true;
  }
  *word = (z * (uint32_t)g.dy + y) * occ_row_words(g.dx) + (x >> 5);
  *bit = 1u << (x & 31u);
  return true;
}

// Whether the x cells [cx - R, cx + R] (clamped to the grid) of a query span
// two runs of a hashed grid.
template <int R>
__device__ inline bool hashed_straddle(const GridDesc& g, int cx) {
  const int lo = max(cx - R, 0), hi = min(cx + R, g.dx - 1);
  return lo <= hi && (hi & ~(kHashRun - 1)) > lo;
}

// Dense grid: one range per surviving row.  Hashed grid: a row segment lies
// in one run of kHashRun cells or straddles two; part 0 stages each row's
// range in its first run, part 1 the rest of the straddling rows (the caller
// scans part 0 before it stages part 1 into the same slots).
template <int R>
__device__ inline uint32_t stage_rows(const PassArgs& a, const QueryCell& qc, uint2* lane_ranges,
                                      uint64_t best, int part = 0) {
  constexpr int W = 2 * R + 1;
  const GridDesc& g = a.g;
  const int cx = qc.cx, cy = qc.cy, cz = qc.cz;
  const float fx = qc.fx, fy = qc.fy, fz = qc.fz;

  // squared gaps (in cells) from the query to the slab of offset d, lowered by
  // a safety margin; slabs outside the grid get an infinite gap
  float g2x[W], g2y[W], g2z[W];
#pragma unroll
  for (int d = -R; d <= R; ++d) {
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (d < 0) {
      gx = fx + (float)(-d - 1); gy = fy + (float)(-d - 1); gz = fz + (float)(-d - 1);
    } else if (d > 0) {
      gx = (float)d - fx; gy = (float)d - fy; gz = (float)d - fz;
    }
    gx = fmaxf(gx - 1e-5f, 0.f); gy = fmaxf(gy - 1e-5f, 0.f); gz = fmaxf(gz - 1e-5f, 0.f);
    g2x[d + R] = gx * gx;
    g2y[d + R] = (unsigned)(cy + d) < (unsigned)g.dy ? gy * gy : INFINITY;
    g2z[d + R] = (unsigned)(cz + d) < (unsigned)g.dz ? gz * gz : INFINITY;
  }
  float B = a.r2f;
  if (best != ~0ull) B = fminf(B, __uint_as_float((uint32_t)(best >> 32)));
  const float thr = B * a.inv_h2 * (1.0f + 1e-4f) + 1e-6f;
  // a row of (y, z) gap gyz spans x offsets -d..d' where gyz + g2x <= thr;
  // the thresholds and the clamped x bounds are shared by all rows
  float tlo[R + 1], thi[R + 1];
  int xlo_c[R + 1], xhi_c[R + 1];
#pragma unroll
  for (int d = 0; d <= R; ++d) {
    tlo[d] = thr - g2x[R - d];
    thi[d] = thr - g2x[R + d];
    xlo_c[d] = max(cx - d, 0);
    xhi_c[d] = min(cx + d, g.dx - 1);
  }
  // hashed grids: first x of the run holding the neighbourhood's last cell
  const int xsplit = xhi_c[R] & ~(kHashRun - 1);
  const uint32_t sdx = (uint32_t)g.dx, sdxdy = (uint32_t)g.dx * (uint32_t)g.dy;
  // row index of (cy, cz); rows of out-of-grid slabs wrap but are never loaded
  uint32_t base = ((uint32_t)cz * (uint32_t)g.dy + (uint32_t)cy) * sdx;
  // keep the rows as base + constant: without this the compiler refactors each
  // row index into its own (quarter-rate) integer multiply
  asm volatile("" : "+v"(base));

  // every surviving row's two table entries are loaded before any is used,
  // so the rows cost one memory round trip instead of one each
  constexpr int NR = W * W;
  uint32_t beg[NR], end_[NR];
  bool ok[NR];
#pragma unroll
  for (int dz = -R; dz <= R; ++dz) {
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
      const int k = (dz + R) * W + (dy + R);
      const float gyz = g2z[dz + R] + g2y[dy + R];
      int xlo = xlo_c[0], xhi = xhi_c[0];
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        if (gyz <= tlo[d]) xlo = xlo_c[d];
        if (gyz <= thi[d]) xhi = xhi_c[d];
      }
      ok[k] = gyz <= thr && xlo <= xhi;
      if (!g.hashed) {
        if (part != 0) ok[k] = false;
        if (ok[k]) {
          const uint32_t row = base + (uint32_t)dz * sdxdy + (uint32_t)dy * sdx;
          beg[k] = ld_cell(a.cs, row + (uint32_t)xlo);
          end_[k] = ld_cell(a.cs, row + (uint32_t)xhi + 1u);
        }
      } else {
        // the split is fixed per query (the first x of the run that holds
        // the neighbourhood's last cell), not per bound: part 1 runs with the
        // bound that part 0 has tightened, which may narrow [xlo, xhi], and
        // must still cover every cell that part 0 did not
        int x0 = xlo, x1 = xhi;
        if (part == 0) {
          if (xsplit > xlo_c[R]) x1 = min(xhi, xsplit - 1);
        } else {
          ok[k] = ok[k] && xsplit > xlo_c[R];
          x0 = max(xlo, xsplit);
        }
        ok[k] = ok[k] && x0 <= x1;
        if (ok[k]) {
          const uint32_t slot = hashed_slot(g, x0, cy + dy, cz + dz);
          beg[k] = ld_cell(a.cs, slot);
          end_[k] = ld_cell(a.cs, slot + (uint32_t)(x1 - x0) + 1u);
        }
      }
    }
  }
  int m = 0;
  uint32_t total = 0;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (ok[k] && beg[k] < end_[k]) {
      lane_ranges[m * kWave] = make_uint2(beg[k], end_[k]);
      ++m;
      total += end_[k] - beg[k];
    }
  }
  return total;
}

template <int R>
__device__ inline uint32_t stage_rows(const PassArgs& a, float q32x, float q32y, float q32z,
                                      uint2* lane_ranges, uint64_t best) {
  return stage_rows<R>(a, query_cell<R>(a.g, q32x, q32y, q32z), lane_ranges, best);
}

// Scans the `total` candidates of the lane's staged ranges in order, keeping
// the smallest (d^2, original index) key.
__device__ inline void scan_ranges(const PassArgs& a, float q32x, float q32y, float q32z,
                                   const uint2* lane_ranges, uint32_t total, uint64_t& best,
                                   uint32_t& bj) {
  if (total == 0) return;
  uint2 e = lane_ranges[0];
  uint32_t pos = e.x, end = e.y;
  int slot = 0;
  for (uint32_t k = 0; k < total; ++k) {
    if (pos == end) {
      ++slot;
      e = lane_ranges[slot * kWave];
      pos = e.x;
      end = e.y;
    }
    const float4 p = ld4(a.tp, pos);
    const float dx = q32x - p.x, dy = q32y - p.y, dz = q32z - p.z;
    float d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint64_t)__float_as_uint(p.w);
    if (key < best) {
      best = key;
      bj = pos;
    }
    ++pos;
  }
}

// Per-wave LDS region: during the search it holds the lanes' candidate ranges
// ([slot][lane] uint2), during the reduction half of the transposed terms
// ([value][lane], 14 float or 14 double values).
template <int R, int PREC = 0>
struct WaveScratch {
  static constexpr int kRangeWords = (2 * R + 1) * (2 * R + 1) * kWave * 2;
  static constexpr int kTermWords = 14 * kWave * (PREC == 0 ? 1 : 2);
  static constexpr int kWords = kRangeWords > kTermWords ? kRangeWords : kTermWords;
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One pass over a tile of kRounds * kBlock queries per block (one query per
// thread and round): correspondence, per-correspondence J^T J / J^T r terms,
// and their sum.
//
// Latency: with several rounds, each round's source point, warm-start index
// and warm-start target point are loaded one round ahead.  A query whose
// 27-cell neighbourhood holds no target (dilated occupancy bitmap) skips the
// row search, and a wave without any correspondence skips the terms and the
// reduction.
//
// Reduction (float32 Kahan mode): each lane adds its own queries' 28 terms
// over the rounds in float32; after the last round the lanes write them to
// the wave's LDS region transposed ([term][lane], 14 terms at a time) and
// lane L (< 56) adds 16 entries of term L >> 2 with Kahan compensation, the
// four quarters merging by TwoSum.  Float64 mode does the transposed sum
// every round, in float64.  The block's waves are then merged in a fixed
// order and one float64 partial per term is written, so results do not
// depend on timing.
template <int VAR, int PREC, bool WRITE, int R, bool ROBUST>
__device__ void pass_tile(const PassArgs& a, uint32_t tile_index) {
  // float32 mode merges (sum, compensation) pairs, float64 mode plain sums
  constexpr int kRedS = PREC == 0 ? kNumSums : 1;
  constexpr int kRedD = PREC == 0 ? 1 : kNumSums;
  __shared__ __align__(16) uint32_t scratch[kBlock / kWave][WaveScratch<R, PREC>::kWords];
  __shared__ float red_s[kBlock / kWave][kRedS];
  __shared__ float red_c[kBlock / kWave][kRedS];
  __shared__ double red_d[kBlock / kWave][kRedD];
  __shared__ uint32_t red_n[kBlock / kWave];
  double T[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) T[k] = glb(a.st)->T[k];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint32_t* ws = scratch[w];
  uint2* lane_ranges = reinterpret_cast<uint2*>(ws) + lane;
  float* xf = reinterpret_cast<float*>(ws);
  double* xd = reinterpret_cast<double*>(ws);

  float lacc[28];                    // float32 mode: this lane's terms summed over its rounds
#pragma unroll
  for (int k = 0; k < 28; ++k) lacc[k] = 0.0f;
  double acc_d0 = 0.0, acc_d1 = 0.0; // float64 mode: terms lane>>2 and 14 + (lane>>2), quarter lane&3
  uint32_t cnt = 0;
  bool wave_any = false;  // some query of this wave had a correspondence (wave-uniform)

  // Phase 1, for all kRounds queries of the thread at once (their loads in
  // flight together): source point and warm-start index, then the query's
  // cell and its bit in the dilated occupancy bitmap.  Phase 2 searches, one
  // query at a time, only the queries whose neighbourhood holds a target; a
  // wave none of whose lanes has one for a round skips that round entirely.
  constexpr int Q = kRounds;
  const int64_t base = (int64_t)tile_index * kTile + threadIdx.x;
  float ssx[Q], ssy[Q], ssz[Q];
  uint32_t jpq[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = base + (int64_t)q * kBlock;
    const int64_t ic = min(i, (int64_t)a.n_src - 1);
    ssx[q] = glb(a.sx)[ic]; ssy[q] = glb(a.sy)[ic]; ssz[q] = glb(a.sz)[ic];
    jpq[q] = (a.jprev && i < a.n_src) ? glb(a.jprev)[ic] : 0xffffffffu;
  }
  uint32_t nbmask = 0;  // bit q: query q lies in the source and has a target in its 27 cells
  {
    uint32_t word[Q], bit[Q];
    bool inside[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      word[q] = 0u;
      bit[q] = 0u;
      inside[q] = base + (int64_t)q * kBlock < (int64_t)a.n_src;
      if (R == 1 && a.occ) {
        const double sx = ssx[q], sy = ssy[q], sz = ssz[q];
        double t;
        t = T[0] * sx; t = t + T[1] * sy; t = t + T[2] * sz; const float qx = (float)(t + T[3]);
        t = T[4] * sx; t = t + T[5] * sy; t = t + T[6] * sz; const float qy = (float)(t + T[7]);
        t = T[8] * sx; t = t + T[9] * sy; t = t + T[10] * sz; const float qz = (float)(t + T[11]);
        const QueryCell qc = query_cell<R>(a.g, qx, qy, qz);
        uint32_t w = 0u;
        if (occupancy_word(a, qc, &w, &bit[q])) word[q] = ld_cell(a.occ, w);
      } else {
        word[q] = bit[q] = 1u;
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (inside[q] && (word[q] & bit[q]) != 0u) nbmask |= 1u << q;
  }

#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = base + (int64_t)q * kBlock;
    const bool nb = (nbmask >> q) & 1u;
    if (__ballot(nb) == 0) {
      // no query of this round has a candidate: no correspondence
      if (WRITE && i < a.n_src) {
        const uint32_t oi = glb(a.sperm)[i];
        glb(a.idx_out)[oi] = -1;
        glb(a.d2_out)[oi] = INFINITY;
      }
      continue;
    }
    const uint32_t jp = jpq[q];
    // The warm-start point load is unconditional so that no branch forces an
    // early wait on it: a lane without a warm start (or past the end of the
    // source) reads target entry 0, which is never used.
    const float4 pw = ld4(a.tp, jp != 0xffffffffu ? jp : 0u);

    bool inl = false;
    uint32_t bj = 0xffffffffu;
    double q64x = 0.0, q64y = 0.0, q64z = 0.0;
    float q32x = 0.f, q32y = 0.f, q32z = 0.f;
    uint64_t best = ~0ull;
    uint32_t total = 0;
    if (i < a.n_src) {
      const double sx = ssx[q], sy = ssy[q], sz = ssz[q];
      double t;
      t = T[0] * sx; t = t + T[1] * sy; t = t + T[2] * sz; q64x = t + T[3];
      t = T[4] * sx; t = t + T[5] * sy; t = t + T[6] * sz; q64y = t + T[7];
      t = T[8] * sx; t = t + T[9] * sy; t = t + T[10] * sz; q64z = t + T[11];
      q32x = (float)q64x; q32y = (float)q64y; q32z = (float)q64z;
      if (jp != 0xffffffffu) {
        // warm start: a target point (the previous pass's match) bounds this
        // pass's distance; any target would do, so an index left over from an
        // earlier pass is as valid as a fresh one
        const float dx = q32x - pw.x, dy = q32y - pw.y, dz = q32z - pw.z;
        float d2 = dx * dx + dy * dy;
        d2 = d2 + dz * dz;
        if (d2 <= a.r2f) {
          best = ((uint64_t)__float_as_uint(d2) << 32) | (uint64_t)__float_as_uint(pw.w);
          bj = jp;
        }
      }
      if (nb) total = stage_rows<R>(a, query_cell<R>(a.g, q32x, q32y, q32z), lane_ranges, best);
    }
    scan_ranges(a, q32x, q32y, q32z, lane_ranges, total, best, bj);
    if (a.g.hashed) {
      // the second runs of straddling row segments (waves whose queries all
      // lie inside single runs skip this)
      const QueryCell qc = query_cell<R>(a.g, q32x, q32y, q32z);
      const bool straddle = i < a.n_src && nb && hashed_straddle<R>(a.g, qc.cx);
      if (__ballot(straddle) != 0) {
        const uint32_t total1 = straddle ? stage_rows<R>(a, qc, lane_ranges, best, 1) : 0u;
        scan_ranges(a, q32x, q32y, q32z, lane_ranges, total1, best, bj);
      }
    }
    if (i < a.n_src) {
      const float bd = __uint_as_float((uint32_t)(best >> 32));
      const uint32_t bo = (uint32_t)best;
      inl = best != ~0ull && bd <= a.r2f;
      // the warm-start index is written back only where a match is found at
      // another position (a query that loses its match keeps the old index)
      if (a.jprev && inl && bj != jp) glb(a.jprev)[i] = bj;
      if (WRITE) {
        const uint32_t oi = glb(a.sperm)[i];
        glb(a.idx_out)[oi] = inl ? (int32_t)bo : -1;
        glb(a.d2_out)[oi] = inl ? bd : INFINITY;
      }
    }
    const uint64_t inl_mask = __ballot(inl);
    cnt += (uint32_t)__popcll(inl_mask);
    wave_any = wave_any || inl_mask != 0;

    // a wave without any correspondence adds nothing (every term is zero);
    // the matched point and normal are loaded only by waves that use them
    float4 bp = make_float4(0.f, 0.f, 0.f, 0.f), bn = make_float4(0.f, 0.f, 0.f, 0.f);
    if (inl_mask != 0) {
      const uint32_t bjc = inl ? bj : 0u;
      bp = ld4(a.tp, bjc);
      if (VAR == 1) bn = ld4(a.tn, bjc);
    }
    if (inl_mask == 0) {
    } else if constexpr (PREC == 0) {
      // a query without a correspondence adds exact zeros: point-to-plane
      // terms vanish with a zero residual and normal, point-to-point terms
      // (which hold constants) are selected away
      float v[28];
      const double rx = q64x - (double)bp.x, ry = q64y - (double)bp.y, rz = q64z - (double)bp.z;
      const float fx = inl ? (float)rx : 0.f, fy = inl ? (float)ry : 0.f, fz = inl ? (float)rz : 0.f;
      const float nx = inl ? bn.x : 0.f, ny = inl ? bn.y : 0.f, nz = inl ? bn.z : 0.f;
      record_terms<VAR, float>(q32x, q32y, q32z, fx, fy, fz, nx, ny, nz, v);
      const float d2 = fx * fx + fy * fy;
      v[27] = d2 + fz * fz;
      if (ROBUST) {  // robust variant (IRLS weight of the loss)
        const float sr = VAR == 1 ? fabsf((nx * fx + ny * fy) + nz * fz) : sqrtf(v[27]);
        const float wr = loss_weight<float>(a.loss, a.loss_k32, sr);
#pragma unroll
        for (int k = 0; k < 27; ++k) v[k] = v[k] * wr;
      }
      if (VAR != 1) {
#pragma unroll
        for (int k = 0; k < 27; ++k) v[k] = inl ? v[k] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < 28; ++k) lacc[k] = lacc[k] + v[k];
    } else {
      wave_sync();  // the search's LDS ranges are dead from here on
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        double v[28];
        if (inl) {
          const double px = bp.x, py = bp.y, pz = bp.z;
          const double rx = q64x - px, ry = q64y - py, rz = q64z - pz;
          double nx = 0.0, ny = 0.0, nz = 0.0;
          if (VAR == 1) {
            nx = bn.x; ny = bn.y; nz = bn.z;
          }
          record_terms<VAR, double>(q64x, q64y, q64z, rx, ry, rz, nx, ny, nz, v);
          v[27] = (rx * rx + ry * ry) + rz * rz;
          if (ROBUST) {
            const double sr = VAR == 1 ? fabs((nx * rx + ny * ry) + nz * rz) : sqrt(v[27]);
            const double wr = loss_weight<double>(a.loss, a.loss_k, sr);
#pragma unroll
            for (int k = 0; k < 27; ++k) v[k] = v[k] * wr;
          }
        } else {
#pragma unroll
          for (int k = 0; k < 28; ++k) v[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 14; ++k) xd[k * kWave + lane] = v[14 * half + k];
        wave_sync();
        if (lane < 56) {
          const double2* src = reinterpret_cast<const double2*>(xd + (lane >> 2) * kWave + (lane & 3) * 16);
          double sacc = 0.0;
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            const double2 x2 = src[m];
            sacc = sacc + x2.x;
            sacc = sacc + x2.y;
          }
          if (half == 0) acc_d0 = acc_d0 + sacc; else acc_d1 = acc_d1 + sacc;
        }
        wave_sync();
      }
    }
  }

  // merge within the wave, then across the block's waves, in a fixed order
  if constexpr (PREC == 0) {
    // Kahan over the wave's lanes, 14 terms at a time through LDS: in half h
    // lane L < 56 sums the 16 entries (L & 3) * 16.. of term 14 h + (L >> 2)
    // with compensation; the four quarters merge by TwoSum (quarters 0+1 and
    // 2+3, then the two pairs).  A wave that saw no correspondence holds
    // only zeros and skips the sums.
    float s_h[2] = {0.f, 0.f}, c_h[2] = {0.f, 0.f};
    if (wave_any) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        wave_sync();  // the last search's ranges (or the previous half) are dead from here on
#pragma unroll
        for (int k = 0; k < 14; ++k) xf[k * kWave + lane] = lacc[14 * half + k];
        wave_sync();
        float acc_s = 0.f, acc_c = 0.f;
        if (lane < 56) {
          const float4* src = reinterpret_cast<const float4*>(xf + (lane >> 2) * kWave + (lane & 3) * 16);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const float4 x4 = src[m];
            const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float y = xs[e] - acc_c;
              const float t = acc_s + y;
              acc_c = (t - acc_s) - y;
              acc_s = t;
            }
          }
        }
#pragma unroll
        for (int off = 1; off <= 2; off <<= 1) {
          const float so = __shfl_xor(acc_s, off, kWave);
          const float co = __shfl_xor(acc_c, off, kWave);
          float s2, e;
          // the lower quarter is the first operand, so both lanes of a pair
          // form the same (s2, c2)
          if (lane & off) two_sum(so, acc_s, s2, e); else two_sum(acc_s, so, s2, e);
          acc_c = ((lane & off) ? (co + acc_c) : (acc_c + co)) + e;
          acc_s = s2;
        }
        s_h[half] = acc_s;
        c_h[half] = acc_c;
      }
    }
    if (lane < 56 && (lane & 3) == 0) {
      red_s[w][lane >> 2] = s_h[0];
      red_c[w][lane >> 2] = c_h[0];
      red_s[w][14 + (lane >> 2)] = s_h[1];
      red_c[w][14 + (lane >> 2)] = c_h[1];
    }
  } else {
    double d0 = acc_d0 + __shfl_xor(acc_d0, 1, kWave);
    double d1 = acc_d1 + __shfl_xor(acc_d1, 1, kWave);
    d0 = d0 + __shfl_xor(d0, 2, kWave);
    d1 = d1 + __shfl_xor(d1, 2, kWave);
    if (lane < 56 && (lane & 3) == 0) {
      red_d[w][lane >> 2] = d0;
      red_d[w][14 + (lane >> 2)] = d1;
    }
  }
  if (lane == 0) red_n[w] = cnt;
  __syncthreads();
  if (threadIdx.x < 28) {
    const int k = threadIdx.x;
    double out;
    if constexpr (PREC == 0) {
      float S = red_s[0][k], C = red_c[0][k];
      for (int ww = 1; ww < kBlock / kWave; ++ww) {
        float t2, e;
        two_sum(S, red_s[ww][k], t2, e);
        S = t2;
        C = (C + red_c[ww][k]) + e;
      }
      out = (double)S + (double)C;
    } else {
      out = red_d[0][k];
      for (int ww = 1; ww < kBlock / kWave; ++ww) out = out + red_d[ww][k];
    }
    glb(a.part)[(int64_t)k * a.n_blocks + tile_index] = out;
  } else if (threadIdx.x == 28) {
    uint32_t nn = 0;
    for (int ww = 0; ww < kBlock / kWave; ++ww) nn += red_n[ww];
    glb(a.part)[(int64_t)28 * a.n_blocks + tile_index] = (double)nn;
  }
}

// Block -> tile order.  Blocks are handed to the eight XCDs in turn (block b
// to XCD b mod 8), each with its own L2; consecutive Morton-ordered tiles
// share target cells, so each XCD takes runs of kXcdRun consecutive tiles:
// within a group of 8 kXcdRun blocks, block r works on tile
// (r mod 8) kXcdRun + r div 8.  Groups rotate over the XCDs, which keeps the
// work balanced when the busy tiles are clustered.  A bijection on the
// tiles; the last partial group keeps the identity.
#ifndef ICP_XCD_RUN
#define ICP_XCD_RUN 16
#endif
constexpr uint32_t kXcdRun = ICP_XCD_RUN;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  constexpr uint32_t G = 8 * kXcdRun;
  if (kXcdRun <= 1 || b >= (n / G) * G) return b;
  const uint32_t r = b % G;
  return (b - r) + (r % 8) * kXcdRun + r / 8;
}

template <int VAR, int PREC, bool WRITE, int R, bool ROBUST>
__global__ __launch_bounds__(kBlock) void pass_kernel(PassArgs a) {
  if (glb(a.st)->done) return;
  pass_tile<VAR, PREC, WRITE, R, ROBUST>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Batched form: block b handles tile items[b].y of pair items[b].x.  Tiles and
// their partial slots are the same as when the pair is registered alone, so a
// pair's result does not depend on the rest of the batch.
// ---- RANSAC validation --------------------------------------------------
// Block (tile, v) scores hypothesis v over kTile Morton-ordered source points:
// the same transform, candidate rows and selection as the pass (no warm
// start: every hypothesis is a new pose; instead the query's own cell is
// scanned first and its nearest point bounds the row pruning), then the
// block's inlier count and
// fixed-point squared-distance sum.  floor(d2 * 2^shift) of a float32 d2 is
// exact in float64 (a power-of-two scale) and below 2^40, so the sums are
// exact integers whatever the order.
template <int R>
__global__ __launch_bounds__(kBlock) void validate_kernel(ValidateArgs v) {
  __shared__ __align__(16) uint32_t scratch[kBlock / kWave][WaveScratch<R>::kRangeWords];
  __shared__ uint32_t red_n[kBlock / kWave];
  __shared__ uint64_t red_q[kBlock / kWave];
  const PassArgs& a = v.p;
  const uint32_t tile = blockIdx.x, hyp = blockIdx.y;
  const ICP_G double* Th = glb(v.T) + (size_t)hyp * 12;
  double T[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) T[k] = Th[k];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint2* lane_ranges = reinterpret_cast<uint2*>(scratch[w]) + lane;
  uint32_t cnt = 0;
  uint64_t sq = 0;
  const int64_t base = (int64_t)tile * kTile;
  for (int round = 0; round < kRounds; ++round) {
    const int64_t i = base + round * kBlock + threadIdx.x;
    bool inl = false;
    float bd = 0.f;
    if (i < a.n_src) {
      const double sx = glb(a.sx)[i], sy = glb(a.sy)[i], sz = glb(a.sz)[i];
      double t;
      t = T[0] * sx; t = t + T[1] * sy; t = t + T[2] * sz; const double qx = t + T[3];
      t = T[4] * sx; t = t + T[5] * sy; t = t + T[6] * sz; const double qy = t + T[7];
      t = T[8] * sx; t = t + T[9] * sy; t = t + T[10] * sz; const double qz = t + T[11];
      const float q32x = (float)qx, q32y = (float)qy, q32z = (float)qz;
      uint64_t best = ~0ull;
      uint32_t bj = 0xffffffffu;
      {
        // the query's own cell first: its nearest point bounds the search and
        // prunes the other rows (the bound is conservative, the result exact)
        const GridDesc& g = a.g;
        const double ux = ((double)q32x - g.ox) * g.inv_h, uy = ((double)q32y - g.oy) * g.inv_h,
                     uz = ((double)q32z - g.oz) * g.inv_h;
        if (ux >= 0.0 && uy >= 0.0 && uz >= 0.0 && ux < (double)g.dx && uy < (double)g.dy && uz < (double)g.dz) {
          const uint32_t cell = ((uint32_t)uz * (uint32_t)g.dy + (uint32_t)uy) * (uint32_t)g.dx + (uint32_t)ux;
          const uint32_t b0 = ld_cell(a.cs, cell), b1 = ld_cell(a.cs, cell + 1u);
          for (uint32_t pos = b0; pos < b1; ++pos) {
            const float4 p = ld4(a.tp, pos);
            const float dx = q32x - p.x, dy = q32y - p.y, dz = q32z - p.z;
            float d2 = dx * dx + dy * dy;
            d2 = d2 + dz * dz;
            const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint64_t)__float_as_uint(p.w);
            if (d2 <= a.r2f && key < best) best = key;
          }
        }
      }
      const uint32_t total = stage_rows<R>(a, q32x, q32y, q32z, lane_ranges, best);
      scan_ranges(a, q32x, q32y, q32z, lane_ranges, total, best, bj);
      bd = __uint_as_float((uint32_t)(best >> 32));
      inl = best != ~0ull && bd <= a.r2f;
    }
    cnt += (uint32_t)__popcll(__ballot(inl));
    if (inl) sq += (uint64_t)((double)bd * v.scale);
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) sq += __shfl_xor(sq, off, kWave);
  if (lane == 0) {
    red_n[w] = cnt;
    red_q[w] = sq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t n = 0;
    uint64_t q = 0;
    for (int ww = 0; ww < kBlock / kWave; ++ww) {
      n += red_n[ww];
      q += red_q[ww];
    }
    glb(v.part_cnt)[(size_t)hyp * v.n_tiles + tile] = n;
    glb(v.part_sq)[(size_t)hyp * v.n_tiles + tile] = q;
  }
}

// One block per hypothesis: integer sums of its tiles' partials.
__global__ __launch_bounds__(256) void validate_reduce_kernel(ValidateArgs v) {
  __shared__ uint64_t sn[256 / kWave], sq_s[256 / kWave];
  const uint32_t hyp = blockIdx.x;
  uint64_t n = 0, q = 0;
  for (int t = threadIdx.x; t < v.n_tiles; t += 256) {
    n += glb(v.part_cnt)[(size_t)hyp * v.n_tiles + t];
    q += glb(v.part_sq)[(size_t)hyp * v.n_tiles + t];
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    n += __shfl_xor(n, off, kWave);
    q += __shfl_xor(q, off, kWave);
  }
  if (lane_id() == 0) {
    sn[threadIdx.x / kWave] = n;
    sq_s[threadIdx.x / kWave] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t N = 0, Q = 0;
    for (int ww = 0; ww < 256 / kWave; ++ww) {
      N += sn[ww];
      Q += sq_s[ww];
    }
    glb(v.cnt_out)[hyp] = (int64_t)N;
    glb(v.sq_out)[hyp] = Q;
  }
}

template <int VAR, int PREC, int R, bool ROBUST = false>
__global__ __launch_bounds__(kBlock) void batch_pass_kernel(const PassArgs* __restrict__ pairs,
                                                            const uint2* __restrict__ items) {
  const uint2 it = items[xcd_tile(blockIdx.x, gridDim.x)];
  const PassArgs a = pairs[it.x];  // by value: uniform, kept in scalar registers
  if (glb(a.st)->done) return;
  pass_tile<VAR, PREC, false, R, ROBUST>(a, it.y);
}

// ------------------------------------------------------------------ solve + pose update
// 6x6 Cholesky of A (given by its upper triangle), x = -A^{-1} b.  Fails when
// a pivot is <= 1e-12 * max(diag A).
__device__ bool cholesky_solve6(const double* up21, const double* b, double* x) {
  double A[6][6];
  int k = 0;
  for (int r = 0; r < 6; ++r)
    for (int c = r; c < 6; ++c) {
      A[r][c] = up21[k];
      A[c][r] = up21[k];
      ++k;
    }
  double dmax = A[0][0];
  for (int r = 1; r < 6; ++r) dmax = fmax(dmax, A[r][r]);
  const double tol = 1e-12 * dmax;
  // one reciprocal per pivot instead of a division per entry: the solve
  // runs on a single thread between passes, and float64 divisions dominate
  // its latency
  double L[6][6];
  double inv[6];
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) L[r][c] = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double d = A[c][c];
#pragma unroll
    for (int m = 0; m < c; ++m) d -= L[c][m] * L[c][m];
    if (!(d > tol)) return false;
    L[c][c] = sqrt(d);
    inv[c] = 1.0 / L[c][c];
#pragma unroll
    for (int r = c + 1; r < 6; ++r) {
      double s = A[r][c];
#pragma unroll
      for (int m = 0; m < c; ++m) s -= L[r][m] * L[c][m];
      L[r][c] = s * inv[c];
    }
  }
  double y[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double s = -b[r];
#pragma unroll
    for (int m = 0; m < r; ++m) s -= L[r][m] * y[m];
    y[r] = s * inv[r];
  }
#pragma unroll
  for (int r = 5; r >= 0; --r) {
    double s = y[r];
#pragma unroll
    for (int m = r + 1; m < 6; ++m) s -= L[m][r] * x[m];
    x[r] = s * inv[r];
  }
  return true;
}

// T <- Exp(xi) T with xi = (omega, v): R = I + A W + B W^2, V = I + B W + C W^2.
__device__ void apply_exp(const double* xi, double* T) {
  const double wx = xi[0], wy = xi[1], wz = xi[2];
  const double th2 = (wx * wx + wy * wy) + wz * wz;
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    // one sincos of th / 2 (sin th = 2 sin(th/2) cos(th/2); 1 - cos th =
    // 2 sin^2(th/2) without cancellation) and one reciprocal
    double sh, ch;
    sincos(0.5 * th, &sh, &ch);
    const double s = 2.0 * sh * ch;
    const double it = 1.0 / th, it2 = it * it;
    A = s * it;
    B = 2.0 * sh * sh * it2;
    C = (th - s) * (it2 * it);
  }
  const double W[3][3] = {{0.0, -wz, wy}, {wz, 0.0, -wx}, {-wy, wx, 0.0}};
  double W2[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += W[r][m] * W[m][c];
      W2[r][c] = s;
    }
  double E[3][4];
  for (int r = 0; r < 3; ++r) {
    double Vr[3];
    for (int c = 0; c < 3; ++c) {
      const double I = (r == c) ? 1.0 : 0.0;
      E[r][c] = I + A * W[r][c] + B * W2[r][c];
      Vr[c] = I + B * W[r][c] + C * W2[r][c];
    }
    E[r][3] = Vr[0] * xi[3] + Vr[1] * xi[4] + Vr[2] * xi[5];
  }
  double N[12];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += E[r][m] * T[4 * m + c];
      if (c == 3) s += E[r][3];
      N[4 * r + c] = s;
    }
  for (int k = 0; k < 12; ++k) T[k] = N[k];
}

// Two-level partial sum, for pairs of more than kTwoLevel pass blocks: the
// blocks are cut into S = segs_of(n) segments of ceil(n / S) consecutive
// blocks; a segment's sum is taken by 8 lanes (lane j adds blocks j, j + 8,
// ... of the segment in order, then a fixed xor-shuffle tree), and the solve
// then adds the S segment sums.  A single pair's segment sums come from a
// separate many-block kernel (one block's bandwidth would bound the solve);
// the batched solve computes them in-block with the same function, so a pair
// gets the same bits in both forms.
constexpr int kTwoLevel = 512;

__device__ double segment_sum(const ICP_G double* row, int n_blocks, int s, int j) {
  const int segs = segs_of(n_blocks);
  const int len = (n_blocks + segs - 1) / segs;
  const int b1 = min(n_blocks, (s + 1) * len);
  double acc = 0.0;
  for (int b = s * len + j; b < b1; b += 8) acc = acc + row[b];
  acc = acc + __shfl_xor(acc, 1, 8);
  acc = acc + __shfl_xor(acc, 2, 8);
  acc = acc + __shfl_xor(acc, 4, 8);
  return acc;
}

// One thread's share of term v: entries g, g + 32, ... of a row of n values,
// 32 loads in flight per step, added into 8 accumulators in a fixed order.
template <class Ptr>
__device__ double row_share(Ptr p, int n, int g) {
  double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b0 = g; b0 < n; b0 += 32 * 32) {
    double x[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int b = b0 + 32 * u;
      x[u] = b < n ? p[b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) s8[u & 7] = s8[u & 7] + x[u];
  }
  return ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
}

// Reduces a pair's block partials (or, two-level, its segment sums: from
// `red` when given, else computed here) and updates its loop state.
__device__ void solve_body(const SolveArgs& a, const double* red) {
  ICP_G IterState* st = glb(a.st);
  // the converged flag and thread 0's loop state are loaded together with the
  // partials (one memory round trip); the partials read after convergence
  // are discarded
  const int done = st->done;
  int k = 0;
  int64_t n_prev = 0;
  double e_prev = 0.0, T[12];
  if (threadIdx.x == 0) {
    k = st->k;
    n_prev = st->n_prev;
    e_prev = st->e_prev;
    for (int m = 0; m < 12; ++m) T[m] = st->T[m];
  }
  __shared__ double sums[kNumSums];
  __shared__ double sred[kNumSums * kSegs];
  // term v = t / 32 is summed by 32 threads (half a wave), each over its
  // share of the row, then by a fixed shuffle tree
  const int t = threadIdx.x, v = t >> 5, g = t & 31;
  double acc = 0.0;
  if (a.n_blocks <= kTwoLevel) {
    if (v < kNumSums) acc = row_share(glb(a.part) + (int64_t)v * a.n_blocks, a.n_blocks, g);
    if (done) return;
  } else if (red) {
    if (v < kNumSums) acc = row_share(glb(red) + v * kSegs, segs_of(a.n_blocks), g);
    if (done) return;
  } else {
    if (done) return;
    const int segs = segs_of(a.n_blocks);
    for (int idx = t >> 3; idx < kNumSums * segs; idx += (int)(blockDim.x >> 3)) {
      const int vv = idx / segs, sg = idx % segs;
      const double x = segment_sum(glb(a.part) + (int64_t)vv * a.n_blocks, a.n_blocks, sg, t & 7);
      if ((t & 7) == 0) sred[vv * kSegs + sg] = x;
    }
    __syncthreads();
    if (v < kNumSums) acc = row_share(static_cast<const double*>(sred) + v * kSegs, segs, g);
  }
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) acc = acc + __shfl_xor(acc, off, kWave);
  if (v < kNumSums && g == 0) sums[v] = acc;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double n = sums[kSumCount];
  const int64_t nk = (int64_t)n;
  const double fk = n / (double)a.n_src;
  const double ek = nk > 0 ? sqrt(sums[kSumD2] / n) : 0.0;
  if (a.reduce_only) {
    for (int v = 0; v < kNumSums; ++v) st->sums[v] = sums[v];
    st->n_in = nk;
    st->fitness = fk;
    st->rmse = ek;
    return;
  }
  int status = -1;
  if (nk == 0) {
    status = 2;
  } else if (k == a.max_iter) {
    status = 0;
  } else if (k >= 1 && fabs((double)(nk - n_prev)) <= a.rel_tol * (double)n_prev &&
             fabs(ek - e_prev) <= a.rel_tol * e_prev) {
    status = 1;
  } else {
    double xi[6];
    if (!cholesky_solve6(sums, sums + 21, xi)) {
      status = 2;
    } else {
      apply_exp(xi, T);
      for (int m = 0; m < 12; ++m) st->T[m] = T[m];
    }
  }
  st->fitness = fk;
  st->rmse = ek;
  st->n_in = nk;
  if (status >= 0) {
    st->status = status;
    st->done = 1;
  } else {
    st->n_prev = nk;
    st->e_prev = ek;
    st->k = k + 1;
  }
}

__global__ __launch_bounds__(1024) void solve_kernel(SolveArgs a, const double* red) { solve_body(a, red); }

// Segment sums of a single pair's block partials (two-level form): block s
// computes segment s of every term.
__global__ __launch_bounds__(256) void reduce_partials_kernel(SolveArgs a, double* red) {
  const int done = glb(a.st)->done;  // loaded with the partials; checked before the store
  const int t = threadIdx.x, v = t >> 3;
  if (v < kNumSums) {
    const double x = segment_sum(glb(a.part) + (int64_t)v * a.n_blocks, a.n_blocks, blockIdx.x, t & 7);
    if ((t & 7) == 0 && !done) glb(red)[v * kSegs + blockIdx.x] = x;
  }
}

// Batched form: block p reduces, solves and updates pair p.
__global__ __launch_bounds__(1024) void batch_solve_kernel(const SolveArgs* __restrict__ arr) {
  const SolveArgs a = arr[blockIdx.x];
  solve_body(a, nullptr);
}

// Copies the loop states of a batch's pairs into one array (one readback).
__global__ void gather_states_kernel(const SolveArgs* __restrict__ arr, int n, IterState* __restrict__ out) {
  const int b = blockIdx.x;
  if (b >= n) return;
  const double* src = reinterpret_cast<const double*>(arr[b].st);
  double* dst = reinterpret_cast<double*>(out + b);
  for (int k = threadIdx.x; k < (int)(sizeof(IterState) / sizeof(double)); k += blockDim.x) dst[k] = src[k];
}

// ------------------------------------------------------------------ normal estimation
// Normal estimation with the hybrid neighbourhood of Sec. 3.2 / Sec. 3.3
// (radius and max_nn) and the least-variance direction of [16]: the
// neighbourhood of a point is the max_nn smallest (pinned float32 squared
// distance, original index) keys among the points within the radius, the
// point itself included; the normal is the eigenvector of the smallest
// eigenvalue of their float64 covariance, turned towards the viewpoint; fewer
// than three neighbours give the zero vector.
//
// A query's candidates are staged as row ranges exactly as in the pass.  Up to
// three scans follow, each with eight candidate loads in flight per lane:
// count the points within the radius; only when that exceeds max_nn, a
// max-heap of the max_nn smallest squared distances (32-bit, this lane's
// column of the block's heap array in LDS) finds the max_nn-th smallest
// distance t; then the covariance sums over the points with d^2 <= t.  The
// neighbourhood is the max_nn smallest (d^2, index) keys: the heap's entries
// below t are all the points closer than t, and its entries equal to t are
// how many of the points at exactly t belong to it.  The third scan counts
// the points at t; in the rare case that there are more than that, the
// belonging ones are the smallest indices among them, found by one more heap
// pass over indices, and the sums are taken again with that rule.  (A 64-bit
// key heap halves the blocks that fit in a CU's LDS and took 3.06 against
// 2.26 ms on 2M points; a single scan that pushes every point within the
// radius through a heap of (key, position) entries and gathers the
// neighbourhood from it measured slower still: the heap traffic, not the
// candidate loads, is the cost.)

// Visits the `total` candidates of the lane's staged ranges in order, loading
// kChunk of them before using any.
constexpr int kChunk = 8;
template <class F>
__device__ inline void for_each_candidate(const float4* tp, const uint2* lane_ranges, uint32_t total,
                                          F&& f) {
  if (total == 0) return;
  uint2 e = lane_ranges[0];
  uint32_t pos = e.x, end = e.y;
  int slot = 0;
  for (uint32_t k0 = 0; k0 < total; k0 += kChunk) {
    // positions first, then unconditional loads (a slot past the end rereads
    // the chunk's first candidate and is not used): a load under a branch
    // would be waited for before the branch joins
    uint32_t at[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      at[u] = at[0];
      if (k0 + u < total) {
        if (pos == end) {
          ++slot;
          e = lane_ranges[slot * kWave];
          pos = e.x;
          end = e.y;
        }
        at[u] = pos;
        ++pos;
      }
    }
    float4 p[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) p[u] = ld4(tp, at[u]);
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      if (k0 + u < total) f(p[u], at[u]);
  }
}

// One Jacobi rotation of the symmetric 3x3 (a, upper entries used) in the
// (p, q) plane that zeroes a_pq, accumulated into the eigenvector matrix v
// (classic symmetric update: a_pp -= t a_pq, a_qq += t a_pq, a_rp / a_rq
// rotated for the third index r).
template <int P, int Q>
__device__ inline void jacobi_rotate(double (&a)[3][3], double (&v)[3][3]) {
  constexpr int Rr = 3 - P - Q;
  const double apq = a[P][Q];
  if (apq == 0.0) return;
  const double theta = (a[Q][Q] - a[P][P]) / (2.0 * apq);
  const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0);
  const double sn = t * c;
  a[P][P] = a[P][P] - t * apq;
  a[Q][Q] = a[Q][Q] + t * apq;
  a[P][Q] = 0.0;
  a[Q][P] = 0.0;
  const double arp = a[Rr][P], arq = a[Rr][Q];
  a[Rr][P] = c * arp - sn * arq;
  a[Rr][Q] = sn * arp + c * arq;
  a[P][Rr] = a[Rr][P];
  a[Q][Rr] = a[Rr][Q];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vkp = v[k][P], vkq = v[k][Q];
    v[k][P] = c * vkp - sn * vkq;
    v[k][Q] = sn * vkp + c * vkq;
  }
}

// Unit eigenvector of the smallest eigenvalue of a symmetric 3x3 (cyclic
// Jacobi sweeps until the off-diagonal mass is negligible).
__device__ inline void least_eigvec3(double (&a)[3][3], double out[3]) {
  double v[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = (a[0][1] * a[0][1] + a[0][2] * a[0][2]) + a[1][2] * a[1][2];
    const double dg = (a[0][0] * a[0][0] + a[1][1] * a[1][1]) + a[2][2] * a[2][2];
    if (off == 0.0 || off <= 1e-36 * dg) break;
    jacobi_rotate<0, 1>(a, v);
    jacobi_rotate<0, 2>(a, v);
    jacobi_rotate<1, 2>(a, v);
  }
  int lo = 0;
  if (a[1][1] < a[lo][lo]) lo = 1;
  if (a[2][2] < a[lo][lo]) lo = 2;
  const double x = lo == 0 ? v[0][0] : (lo == 1 ? v[0][1] : v[0][2]);
  const double y = lo == 0 ? v[1][0] : (lo == 1 ? v[1][1] : v[1][2]);
  const double z = lo == 0 ? v[2][0] : (lo == 1 ? v[2][1] : v[2][2]);
  const double len = sqrt((x * x + y * y) + z * z);
  out[0] = x / len;
  out[1] = y / len;
  out[2] = z / len;
}

template <int R>
__global__ __launch_bounds__(kNormBlock) void normals_kernel(NormalArgs na) {
  extern __shared__ uint32_t nheap[];  // [max_nn][kNormBlock]: each lane's heap is a column
  __shared__ __align__(16) uint32_t nscratch[kNormBlock / kWave][WaveScratch<R>::kRangeWords];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint2* lane_ranges = reinterpret_cast<uint2*>(nscratch[w]) + lane;
  const int64_t i = (int64_t)blockIdx.x * kNormBlock + threadIdx.x;
  if (i >= na.n) return;  // no block-wide synchronisation below
  const float qx = glb(na.sx)[i], qy = glb(na.sy)[i], qz = glb(na.sz)[i];
  PassArgs pa{};
  pa.g = na.g;
  pa.r2f = na.r2f;
  pa.inv_h2 = na.inv_h2;
  pa.cs = na.cs;
  const uint32_t total = stage_rows<R>(pa, qx, qy, qz, lane_ranges, ~0ull);
  const float r2f = na.r2f;
  auto dist2 = [&](const float4& p) {
    const float dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
    float d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    return d2;
  };

  uint32_t within = 0;
  for_each_candidate(na.tp, lane_ranges, total, [&](const float4& p, uint32_t) {
    within += dist2(p) <= r2f ? 1u : 0u;
  });
  const uint32_t K = (uint32_t)na.max_nn;
  uint32_t* H = nheap + threadIdx.x;  // H[k * kNormBlock]
  // Max-heap of the K smallest of a stream of 32-bit values (squared
  // distance bits, or indices); non-negative float bits order as integers.
  auto heap_push = [&](uint32_t& size, uint32_t cap, uint32_t key) {
    if (size < cap) {
      uint32_t at = size++;
      while (at > 0) {  // sift up
        const uint32_t up = (at - 1) >> 1;
        const uint32_t hu = H[up * kNormBlock];
        if (hu >= key) break;
        H[at * kNormBlock] = hu;
        at = up;
      }
      H[at * kNormBlock] = key;
    } else if (key < H[0]) {
      uint32_t at = 0;
      for (;;) {  // sift down from the root
        const uint32_t l = 2 * at + 1;
        if (l >= cap) break;
        uint32_t c = l;
        uint32_t hc = H[l * kNormBlock];
        if (l + 1 < cap) {
          const uint32_t hr = H[(l + 1) * kNormBlock];
          if (hr > hc) {
            c = l + 1;
            hc = hr;
          }
        }
        if (hc <= key) break;
        H[at * kNormBlock] = hc;
        at = c;
      }
      H[at * kNormBlock] = key;
    }
  };
  // selection: d^2 bits below t, or equal to t with index at most tidx
  uint32_t t = 0xffffffffu, tidx = 0xffffffffu, need = 0;
  if (within > K) {
    uint32_t size = 0;
    for_each_candidate(na.tp, lane_ranges, total, [&](const float4& p, uint32_t) {
      const float d2 = dist2(p);
      if (d2 <= r2f) heap_push(size, K, __float_as_uint(d2));
    });
    t = H[0];
    for (uint32_t k = 0; k < K; ++k) need += H[k * kNormBlock] == t ? 1u : 0u;
  }

  // float64 sums of the selected points, relative to the query point
  double s1x = 0.0, s1y = 0.0, s1z = 0.0;
  double sxx = 0.0, sxy = 0.0, sxz = 0.0, syy = 0.0, syz = 0.0, szz = 0.0;
  uint32_t m = 0, at_t = 0;
  auto sums = [&](bool count_ties) {
    s1x = s1y = s1z = 0.0;
    sxx = sxy = sxz = syy = syz = szz = 0.0;
    m = 0;
    for_each_candidate(na.tp, lane_ranges, total, [&](const float4& p, uint32_t) {
      const float d2 = dist2(p);
      if (!(d2 <= r2f)) return;
      const uint32_t db = __float_as_uint(d2);
      if (db > t) return;
      if (db == t) {
        if (count_ties) ++at_t;
        if (__float_as_uint(p.w) > tidx) return;
      }
      const double dx = (double)p.x - (double)qx, dy = (double)p.y - (double)qy,
                   dz = (double)p.z - (double)qz;
      s1x += dx; s1y += dy; s1z += dz;
      sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
      syy += dy * dy; syz += dy * dz; szz += dz * dz;
      ++m;
    });
  };
  sums(within > K);
  if (within > K && at_t > need) {
    // more points at exactly t than belong: the `need` smallest indices
    // among them, the largest of which is the root of a heap of that size
    uint32_t size = 0;
    for_each_candidate(na.tp, lane_ranges, total, [&](const float4& p, uint32_t) {
      const float d2 = dist2(p);
      if (d2 <= r2f && __float_as_uint(d2) == t) heap_push(size, need, __float_as_uint(p.w));
    });
    tidx = H[0];
    sums(false);
  }
  double nrm[3] = {0.0, 0.0, 0.0};
  if (m >= 3) {
    const double inv = 1.0 / (double)m;
    const double mx = s1x * inv, my = s1y * inv, mz = s1z * inv;
    double a[3][3];
    a[0][0] = sxx * inv - mx * mx;
    a[0][1] = sxy * inv - mx * my;
    a[0][2] = sxz * inv - mx * mz;
    a[1][1] = syy * inv - my * my;
    a[1][2] = syz * inv - my * mz;
    a[2][2] = szz * inv - mz * mz;
    a[1][0] = a[0][1];
    a[2][0] = a[0][2];
    a[2][1] = a[1][2];
    least_eigvec3(a, nrm);
    const double dot = (nrm[0] * (na.vx - (double)qx) + nrm[1] * (na.vy - (double)qy)) +
                       nrm[2] * (na.vz - (double)qz);
    if (dot < 0.0) {
      nrm[0] = -nrm[0];
      nrm[1] = -nrm[1];
      nrm[2] = -nrm[2];
    }
  }
  const int64_t oi = glb(na.sperm)[i];
  glb(na.normals)[3 * oi + 0] = (float)nrm[0];
  glb(na.normals)[3 * oi + 1] = (float)nrm[1];
  glb(na.normals)[3 * oi + 2] = (float)nrm[2];
  if (na.counts) glb(na.counts)[oi] = (int32_t)m;
}

// ---- FPFH ---------------------------------------------------------------
// Pair features of (p_i, n_i) and (p_j, n_j), in float64 from the float32
// inputs with every dot and cross product evaluated left to right: the
// source is the end whose normal makes the smaller angle with the line to
// the other end; Darboux frame u = n_s, v = unit(u x e), w = u x v; features
// alpha = v . n_t, phi = u . e, theta = atan2(w . n_t, u . n_t), binned into
// 11 bins each.  False for a pair at zero distance or with u parallel to e.
__device__ inline double dot3(const double a[3], const double b[3]) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}
__device__ inline void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline int fpfh_bin(double x) {
  const double f = floor(x);
  return f < 0.0 ? 0 : (f > 10.0 ? 10 : (int)f);
}
__device__ inline bool pair_bins(const double pi[3], const double ni[3], const double pj[3], const double nj[3],
                                 int bins[3]) {
  double delta[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
  const double d = sqrt(dot3(delta, delta));
  const bool fwd = dot3(ni, delta) >= -dot3(nj, delta);
  const double* u = fwd ? ni : nj;
  const double* nt = fwd ? nj : ni;
  double e[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) e[a] = (fwd ? delta[a] : -delta[a]) / d;
  double c[3];
  cross3(u, e, c);
  const double cn = sqrt(dot3(c, c));
  if (!(d > 0.0) || !(cn > 0.0)) return false;
  const double v[3] = {c[0] / cn, c[1] / cn, c[2] / cn};
  double w[3];
  cross3(u, v, w);
  const double alpha = dot3(v, nt), phi = dot3(u, e);
  const double theta = atan2(dot3(w, nt), dot3(u, nt));
  constexpr double kThetaScale = 11.0 / (2.0 * M_PI);
  bins[0] = fpfh_bin((alpha + 1.0) * 5.5);
  bins[1] = 11 + fpfh_bin((phi + 1.0) * 5.5);
  bins[2] = 22 + fpfh_bin((theta + M_PI) * kThetaScale);
  return true;
}

// FPFH runs one wave per point in three launches (a thread per point would
// leave most SIMDs idle at the point counts of a downsampled cloud).
//
// Selection: every lane stages the point's candidate rows (the same rows, so
// the table loads are broadcasts) and the wave walks the flattened candidate
// list 64 at a time, lane L taking candidate base + L.  The in-radius count
// is a ballot sum; when it exceeds max_nn the max_nn-th smallest (pinned
// float32 squared distance, index) key is found by a radix select over its
// eight bytes, most significant first (per pass a 256-bin LDS histogram of
// the candidates that share the digits found so far; only for such points);
// the selected candidates are then written in candidate order by
// ballot-prefix compaction.
template <int R>
__global__ __launch_bounds__(kFpfhBlock) void fpfh_select_kernel(FpfhArgs fa) {
  __shared__ __align__(16) uint32_t fscratch[kFpfhBlock / kWave][WaveScratch<R>::kRangeWords];
  __shared__ uint32_t fhist[kFpfhBlock / kWave][256];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint2* ranges = reinterpret_cast<uint2*>(fscratch[w]) + lane;  // this lane's copy: ranges[slot * kWave]
  const int64_t i = (int64_t)blockIdx.x * (kFpfhBlock / kWave) + w;
  if (i >= fa.n) return;  // whole waves; no block-wide synchronisation below
  const float qx = glb(fa.sx)[i], qy = glb(fa.sy)[i], qz = glb(fa.sz)[i];
  PassArgs pa{};
  pa.g = fa.g;
  pa.r2f = fa.r2f;
  pa.inv_h2 = fa.inv_h2;
  pa.cs = fa.cs;
  const uint32_t total = stage_rows<R>(pa, qx, qy, qz, ranges, ~0ull);
  const float r2f = fa.r2f;
  // candidate base + lane: the lane's (slot, position) advance monotonically
  struct Walker {
    const uint2* ranges;
    int slot;
    uint32_t before;  // candidates in slots before `slot`
    uint2 e;
    __device__ uint32_t at(uint32_t k) {
      while (k >= before + (e.y - e.x)) {
        before += e.y - e.x;
        ++slot;
        e = ranges[slot * kWave];
      }
      return e.x + (k - before);
    }
  };
  auto key_at = [&](uint32_t pos) {
    const float4 p = ld4(fa.tp, pos);
    const float dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
    float d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    return d2 <= r2f ? ((uint64_t)__float_as_uint(d2) << 32) | (uint64_t)__float_as_uint(p.w) : ~0ull;
  };
  auto count_le = [&](uint64_t bound) {
    uint32_t c = 0;
    if (total == 0) return c;
    Walker wk{ranges, 0, 0u, ranges[0]};
    for (uint32_t base = 0; base < total; base += kWave) {
      const uint32_t k = base + (uint32_t)lane;
      bool hit = false;
      if (k < total) hit = key_at(wk.at(k)) <= bound;
      c += (uint32_t)__popcll(__ballot(hit));
    }
    return c;
  };
  const uint32_t K = (uint32_t)fa.max_nn;
  const uint32_t within = count_le(~0ull - 1);
  uint64_t kth = ~0ull - 1;
  if (within > K) {
    uint32_t* hist = fhist[w];
    uint64_t prefix = 0, mask = 0;
    uint32_t rem = K;  // rank of the wanted key among those matching `prefix` (1-based)
    for (int dg = 7; dg >= 0; --dg) {
      const int sh = 8 * dg;
#pragma unroll
      for (int q = 0; q < 4; ++q) hist[4 * lane + q] = 0u;
      wave_sync();
      Walker wk{ranges, 0, 0u, ranges[0]};
      for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t k = base + (uint32_t)lane;
        if (k < total) {
          const uint64_t key = key_at(wk.at(k));
          if (key != ~0ull && (key & mask) == prefix) atomicAdd(&hist[(key >> sh) & 255u], 1u);
        }
      }
      wave_sync();
      uint32_t c[4], own = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = hist[4 * lane + q];
        own += c[q];
      }
      uint32_t incl = own;  // inclusive scan of the lanes' four-bin sums
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += t;
      }
      const uint32_t before = incl - own;
      const bool mine = before < rem && rem <= incl;
      uint32_t digit = 0, below = before;
      if (mine) {
        uint32_t run = before;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (run + c[q] >= rem) {
            digit = 4 * lane + q;
            below = run;
            break;
          }
          run += c[q];
        }
      }
      const int src = __ffsll((unsigned long long)__ballot(mine)) - 1;
      digit = __shfl(digit, src, kWave);
      below = __shfl(below, src, kWave);
      rem -= below;
      prefix |= (uint64_t)digit << sh;
      mask |= 255ull << sh;
      wave_sync();
    }
    kth = prefix;
  }
  const int64_t oi = glb(fa.sperm)[i];
  ICP_G int32_t* list = glb(fa.nbr) + oi * (int64_t)fa.max_nn;
  uint32_t m = 0;
  if (total > 0) {
    Walker wk{ranges, 0, 0u, ranges[0]};
    for (uint32_t base = 0; base < total; base += kWave) {
      const uint32_t k = base + (uint32_t)lane;
      bool sel = false;
      int32_t j = 0;
      if (k < total) {
        const uint32_t pos = wk.at(k);
        sel = key_at(pos) <= kth;
        j = (int32_t)__float_as_uint(ld4(fa.tp, pos).w);
      }
      const uint64_t b = __ballot(sel);
      if (sel) list[m + (uint32_t)__popcll(b & ((1ull << lane) - 1ull))] = j;
      m += (uint32_t)__popcll(b);
    }
  }
  if (lane == 0) glb(fa.nn)[oi] = (int32_t)m;
}

// Pair bins: lane s takes neighbour s (two rounds for max_nn > 64); the
// point's 33 counts are ballot sums, written by lanes 0..32.
__global__ __launch_bounds__(kFpfhBlock) void fpfh_pairs_kernel(FpfhArgs fa) {
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * (kFpfhBlock / kWave) + w;
  if (i >= fa.n) return;
  const int64_t oi = glb(fa.sperm)[i];
  const int32_t m = glb(fa.nn)[oi];
  const ICP_G int32_t* list = glb(fa.nbr) + oi * (int64_t)fa.max_nn;
  const double pi[3] = {(double)glb(fa.sx)[i], (double)glb(fa.sy)[i], (double)glb(fa.sz)[i]};
  const double ni[3] = {(double)glb(fa.nrm)[3 * oi], (double)glb(fa.nrm)[3 * oi + 1], (double)glb(fa.nrm)[3 * oi + 2]};
  uint32_t mine = 0, pairs = 0;
  for (int32_t base = 0; base < m; base += kWave) {
    const int32_t s = base + lane;
    int bins[3] = {-1, -1, -1};
    bool ok = false;
    if (s < m) {
      const int64_t j = list[s];
      if (j != oi) {
        const double pj[3] = {(double)glb(fa.pts)[3 * j], (double)glb(fa.pts)[3 * j + 1], (double)glb(fa.pts)[3 * j + 2]};
        const double nj[3] = {(double)glb(fa.nrm)[3 * j], (double)glb(fa.nrm)[3 * j + 1], (double)glb(fa.nrm)[3 * j + 2]};
        ok = pair_bins(pi, ni, pj, nj, bins);
      }
    }
    if (!ok) bins[0] = bins[1] = bins[2] = -1;
    pairs += (uint32_t)__popcll(__ballot(ok));
#pragma unroll
    for (int b = 0; b < kFpfhBins; ++b) {
      const int f = b / 11;
      const uint32_t c = (uint32_t)__popcll(__ballot(bins[f] == b));
      if (lane == b) mine += c;
    }
  }
  if (lane < kFpfhBins) glb(fa.counts)[oi * kFpfhCountBytes + lane] = (uint8_t)mine;
  if (lane == 0) glb(fa.k)[oi] = (int32_t)pairs;
}

// FPFH(i) = SPFH(i) + (1 / k') sum over the neighbours j != i at non-zero
// distance w of SPFH(j) / w, SPFH = counts * (100 / k) (zero without pairs),
// in float64 in neighbour-list order, rounded to float32.  Per round of 64
// neighbours, lane s fetches neighbour s (its distance, 100 / k and count
// row, the row into LDS); then lane b adds bin b's terms of the round's
// neighbours in list order.
__global__ __launch_bounds__(kFpfhBlock) void fpfh_final_kernel(FpfhArgs fa) {
  __shared__ uint32_t crow[kFpfhBlock / kWave][kWave][kFpfhCountBytes / 4];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * (kFpfhBlock / kWave) + w;
  if (i >= fa.n) return;
  const int64_t oi = glb(fa.sperm)[i];
  const int b = lane < kFpfhBins ? lane : 0;
  const double pi[3] = {(double)glb(fa.sx)[i], (double)glb(fa.sy)[i], (double)glb(fa.sz)[i]};
  const int32_t m = glb(fa.nn)[oi];
  const ICP_G int32_t* list = glb(fa.nbr) + oi * (int64_t)fa.max_nn;
  const ICP_G uint32_t* cw = reinterpret_cast<const ICP_G uint32_t*>(glb(fa.counts));
  double acc = 0.0;
  int32_t kp = 0;
  for (int32_t base = 0; base < m; base += kWave) {
    const int32_t s = base + lane;
    bool ok = false;
    double wgt = 1.0, qj = 0.0;
    if (s < m) {
      const int64_t j = list[s];
      if (j != oi) {
        const double d[3] = {(double)glb(fa.pts)[3 * j] - pi[0], (double)glb(fa.pts)[3 * j + 1] - pi[1],
                             (double)glb(fa.pts)[3 * j + 2] - pi[2]};
        wgt = sqrt(dot3(d, d));
        ok = wgt > 0.0;
        if (ok) {
          const int32_t kj = glb(fa.k)[j];
          qj = kj > 0 ? 100.0 / (double)kj : 0.0;
#pragma unroll
          for (int wd = 0; wd < kFpfhCountBytes / 4; ++wd) crow[w][lane][wd] = cw[j * (kFpfhCountBytes / 4) + wd];
        }
      }
    }
    uint64_t okm = __ballot(ok);
    kp += __popcll(okm);
    wave_sync();
    while (okm) {
      const int src = __ffsll((unsigned long long)okm) - 1;
      okm &= okm - 1;
      const double ww = __shfl(wgt, src, kWave), qq = __shfl(qj, src, kWave);
      const uint32_t c = (crow[w][src][b >> 2] >> (8 * (b & 3))) & 0xffu;
      acc = acc + ((double)c * qq) / ww;
    }
    wave_sync();
  }
  const int32_t ki = glb(fa.k)[oi];
  const double qi = ki > 0 ? 100.0 / (double)ki : 0.0;
  const double si = (double)glb(fa.counts)[oi * kFpfhCountBytes + b] * qi;
  if (lane < kFpfhBins) glb(fa.out)[oi * kFpfhBins + lane] = (float)(kp > 0 ? si + acc / (double)kp : si);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

// ====================================================================== launchers
hipError_t launch_state_init(IterState* st, const double T[16], hipStream_t s) {
  Mat16 m;
  for (int k = 0; k < 16; ++k) m.v[k] = T[k];
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, s, st, m);
  return hipGetLastError();
}

template <int R, bool ROBUST>
void launch_pass_r(const PassArgs& a, int variant, int precision, bool write_corr, hipStream_t s) {
  const dim3 grid((unsigned)a.n_blocks), block(kBlock);
#define ICP_PASS(V, P, W) hipLaunchKernelGGL((pass_kernel<V, P, W, R, ROBUST>), grid, block, 0, s, a)
  if (write_corr) {
    if (variant == 1) { if (precision == 0) ICP_PASS(1, 0, true); else ICP_PASS(1, 1, true); }
    else { if (precision == 0) ICP_PASS(0, 0, true); else ICP_PASS(0, 1, true); }
  } else {
    if (variant == 1) { if (precision == 0) ICP_PASS(1, 0, false); else ICP_PASS(1, 1, false); }
    else { if (precision == 0) ICP_PASS(0, 0, false); else ICP_PASS(0, 1, false); }
  }
#undef ICP_PASS
}

hipError_t launch_pass(const PassArgs& a, int variant, int precision, bool write_corr, hipStream_t s) {
  // the robust weight is compiled only into the robust kernels
  const bool robust = a.loss != 0;
  if (a.g.sub == 2) {
    if (robust) launch_pass_r<2, true>(a, variant, precision, write_corr, s);
    else launch_pass_r<2, false>(a, variant, precision, write_corr, s);
  } else {
    if (robust) launch_pass_r<1, true>(a, variant, precision, write_corr, s);
    else launch_pass_r<1, false>(a, variant, precision, write_corr, s);
  }
  return hipGetLastError();
}

hipError_t launch_validate(const ValidateArgs& a, int sub, hipStream_t s) {
  if (a.n_hyp <= 0) return hipSuccess;
  const dim3 grid((unsigned)a.n_tiles, (unsigned)a.n_hyp);
  if (sub == 2)
    hipLaunchKernelGGL(validate_kernel<2>, grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(validate_kernel<1>, grid, dim3(kBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(validate_reduce_kernel, dim3((unsigned)a.n_hyp), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, double* red, hipStream_t s) {
  if (red && a.n_blocks > kTwoLevel) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)segs_of(a.n_blocks)), dim3(256), 0, s, a, red);
  } else {
    red = nullptr;
  }
  hipLaunchKernelGGL(solve_kernel, dim3(1), dim3(1024), 0, s, a, (const double*)red);
  return hipGetLastError();
}

template <int R, bool ROBUST>
void launch_batch_pass_r(const PassArgs* pairs, const uint2* items, int n_items, int variant,
                         int precision, hipStream_t s) {
  const dim3 grid((unsigned)n_items), block(kBlock);
#define ICP_BPASS(V, P) hipLaunchKernelGGL((batch_pass_kernel<V, P, R, ROBUST>), grid, block, 0, s, pairs, items)
  if (variant == 1) { if (precision == 0) ICP_BPASS(1, 0); else ICP_BPASS(1, 1); }
  else { if (precision == 0) ICP_BPASS(0, 0); else ICP_BPASS(0, 1); }
#undef ICP_BPASS
}

hipError_t launch_batch_pass(const PassArgs* pairs, const uint2* items, int n_items, int sub,
                             int variant, int precision, bool robust, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (sub == 2) {
    if (robust) launch_batch_pass_r<2, true>(pairs, items, n_items, variant, precision, s);
    else launch_batch_pass_r<2, false>(pairs, items, n_items, variant, precision, s);
  } else {
    if (robust) launch_batch_pass_r<1, true>(pairs, items, n_items, variant, precision, s);
    else launch_batch_pass_r<1, false>(pairs, items, n_items, variant, precision, s);
  }
  return hipGetLastError();
}

hipError_t launch_normals(const NormalArgs& a, int sub, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.max_nn < 1 || a.max_nn > kMaxNormalNN) return hipErrorInvalidValue;
  const dim3 grid((unsigned)ceil_div(a.n, kNormBlock)), block(kNormBlock);
  const size_t heap = sizeof(uint32_t) * (size_t)a.max_nn * kNormBlock;
  if (sub == 2)
    hipLaunchKernelGGL(normals_kernel<2>, grid, block, heap, s, a);
  else
    hipLaunchKernelGGL(normals_kernel<1>, grid, block, heap, s, a);
  return hipGetLastError();
}

hipError_t launch_fpfh(const FpfhArgs& a, int sub, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.max_nn < 1 || a.max_nn > kMaxFpfhNN) return hipErrorInvalidValue;
  const dim3 grid((unsigned)ceil_div(a.n, kFpfhBlock / kWave)), block(kFpfhBlock);
  if (sub == 2)
    hipLaunchKernelGGL(fpfh_select_kernel<2>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(fpfh_select_kernel<1>, grid, block, 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fpfh_pairs_kernel, grid, block, 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(fpfh_final_kernel, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_states(const SolveArgs* arr, int n, IterState* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_states_kernel, dim3((unsigned)n), dim3(64), 0, s, arr, n, out);
  return hipGetLastError();
}

hipError_t launch_batch_solve(const SolveArgs* arr, int n_pairs, hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_solve_kernel, dim3((unsigned)n_pairs), dim3(1024), 0, s, arr);
  return hipGetLastError();
}

void batch_pass_node(int sub, int variant, int precision, bool robust, hipKernelNodeParams* p) {
  void* f;
#define ICP_F(R, V, P)                                                                       \
  f = robust ? reinterpret_cast<void*>(&batch_pass_kernel<V, P, R, true>)                   \
             : reinterpret_cast<void*>(&batch_pass_kernel<V, P, R, false>)
  if (sub == 2) {
    if (variant == 1) { if (precision == 0) ICP_F(2, 1, 0); else ICP_F(2, 1, 1); }
    else { if (precision == 0) ICP_F(2, 0, 0); else ICP_F(2, 0, 1); }
  } else {
    if (variant == 1) { if (precision == 0) ICP_F(1, 1, 0); else ICP_F(1, 1, 1); }
    else { if (precision == 0) ICP_F(1, 0, 0); else ICP_F(1, 0, 1); }
  }
#undef ICP_F
  p->func = f;
  p->blockDim = dim3(kBlock);
  p->gridDim = dim3(1);
  p->sharedMemBytes = 0;
  p->extra = nullptr;
}

void batch_solve_node(hipKernelNodeParams* p) {
  p->func = reinterpret_cast<void*>(&batch_solve_kernel);
  p->blockDim = dim3(1024);
  p->gridDim = dim3(1);
  p->sharedMemBytes = 0;
  p->extra = nullptr;
}

}  // namespace icp
