// Per-call preparation kernels for gfx950: finiteness checks and bounding
// boxes, the dense target grid (cell table + cell-ordered target), and the
// Morton ordering of the source -- for any number of pairs at once.
//
// All pairs of a call are processed by the same launches ("segmented"
// kernels): a block finds its pair from a table of per-pair block offsets, the
// cell tables of all pairs are concatenated and prefix-summed by one scan, and
// the sources of all pairs are ordered by one stable LSD radix sort on the key
// (pair, Morton code), which yields, inside each pair, exactly the order that
// pair gets when it is prepared alone.

#include <math.h>

#include <algorithm>
#include <utility>

#include "icp_internal.h"

#pragma clang fp contract(off)

namespace icp {

namespace {

constexpr int kWave = 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline int lane_id() { return __lane_id(); }

// Largest p with off[p] <= x, for a non-decreasing off[0..n].
__device__ inline int find_segment(const int64_t* __restrict__ off, int n, int64_t x) {
  int lo = 0, hi = n;  // invariant: off[lo] <= x < off[hi] (off[n] > x)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------ bbox + finiteness
__global__ __launch_bounds__(256) void seg_bbox_kernel(const SegCloud* __restrict__ clouds, int n_clouds,
                                                       const int64_t* __restrict__ blk_off,
                                                       float* __restrict__ block_out) {
  const int c = find_segment(blk_off, n_clouds, blockIdx.x);
  const SegCloud cl = clouds[c];
  const int64_t nb = blk_off[c + 1] - blk_off[c];
  const int64_t lb = blockIdx.x - blk_off[c];
  float mn[3] = {INFINITY, INFINITY, INFINITY};
  float mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  float bad = 0.0f;
  for (int64_t i = lb * 256 + threadIdx.x; i < cl.n; i += nb * 256) {
    const float x = cl.pts[3 * i + 0], y = cl.pts[3 * i + 1], z = cl.pts[3 * i + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      bad = 1.0f;
    } else {
      mn[0] = fminf(mn[0], x); mn[1] = fminf(mn[1], y); mn[2] = fminf(mn[2], z);
      mx[0] = fmaxf(mx[0], x); mx[1] = fmaxf(mx[1], y); mx[2] = fmaxf(mx[2], z);
    }
    if (cl.nrm) {
      const float a = cl.nrm[3 * i + 0], b = cl.nrm[3 * i + 1], d = cl.nrm[3 * i + 2];
      if (!(isfinite(a) && isfinite(b) && isfinite(d))) bad = 1.0f;
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    for (int a = 0; a < 3; ++a) {
      mn[a] = fminf(mn[a], __shfl_xor(mn[a], off, kWave));
      mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], off, kWave));
    }
    bad = fmaxf(bad, __shfl_xor(bad, off, kWave));
  }
  __shared__ float red[4][8];
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    for (int a = 0; a < 3; ++a) { red[w][a] = mn[a]; red[w][3 + a] = mx[a]; }
    red[w][6] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int a = threadIdx.x;
    float v = red[0][a];
    for (int k = 1; k < 4; ++k) v = (a < 3) ? fminf(v, red[k][a]) : fmaxf(v, red[k][a]);
    block_out[(int64_t)blockIdx.x * 8 + a] = v;
  }
}

// One block per cloud: min / max / non-finite flag over the cloud's blocks.
__global__ __launch_bounds__(256) void seg_bbox_final_kernel(const int64_t* __restrict__ blk_off,
                                                             const float* __restrict__ block_out,
                                                             float* __restrict__ out) {
  const int c = blockIdx.x;
  const int64_t b0 = blk_off[c], b1 = blk_off[c + 1];
  __shared__ float red[7][256];
  for (int a = 0; a < 7; ++a) {
    float v = (a < 3) ? INFINITY : -INFINITY;
    if (a == 6) v = 0.0f;
    for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) {
      const float x = block_out[b * 8 + a];
      v = (a < 3) ? fminf(v, x) : fmaxf(v, x);
    }
    red[a][threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int a = threadIdx.x;
    float v = red[a][0];
    for (int t = 1; t < 256; ++t) v = (a < 3) ? fminf(v, red[a][t]) : fmaxf(v, red[a][t]);
    out[(int64_t)c * 8 + a] = v;
  }
}

// ------------------------------------------------------------------ exclusive scan (uint32)
// A tile of kScanTile words is handled by one block: thread t owns the
// 16-byte chunks t, t + 256, t + 512, t + 768 of the tile, so that every wave
// load or store covers 1 KiB of consecutive memory.  Chunks are scanned in
// memory order (chunk index j * 256 + t).  Scanned arrays start 16-byte
// aligned (the launcher checks).
constexpr int kScanThreads = 256;
constexpr int kScanVecs = 4;
constexpr int kScanTile = kScanThreads * kScanVecs * 4;
constexpr int kScanWaves = kScanThreads / kWave;

typedef uint32_t scan_u4 __attribute__((ext_vector_type(4)));
#define ICP_GLB __attribute__((address_space(1)))

__device__ inline scan_u4 scan_load(const uint32_t* d, int64_t i, int64_t n) {
  if (i + 4 <= n) return *(const ICP_GLB scan_u4*)(d + i);
  scan_u4 v = {0u, 0u, 0u, 0u};
  if (i < n) v.x = d[i];
  if (i + 1 < n) v.y = d[i + 1];
  if (i + 2 < n) v.z = d[i + 2];
  return v;
}

__device__ inline void scan_store(uint32_t* d, int64_t i, int64_t n, scan_u4 v) {
  if (i + 4 <= n) {
    *(ICP_GLB scan_u4*)(d + i) = v;
    return;
  }
  if (i < n) d[i] = v.x;
  if (i + 1 < n) d[i + 1] = v.y;
  if (i + 2 < n) d[i + 2] = v.z;
}

__device__ inline uint32_t wave_inclusive_sum(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ inline uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Exclusive scan of a value per thread over the block (thread order); the
// block total in *total.  Used where the order is the thread order.
template <int kThreads>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint32_t x = wave_inclusive_sum(v);
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int k = 0; k < kThreads / kWave; ++k) {
    if (k < w) before += wsum[k];
    all += wsum[k];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums_kernel(const uint32_t* __restrict__ d,
                                                                      int64_t n,
                                                                      uint32_t* __restrict__ sums) {
  __shared__ uint32_t wsum[kScanWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  scan_u4 v[kScanVecs];
#pragma unroll
  for (int j = 0; j < kScanVecs; ++j) v[j] = scan_load(d, base + (int64_t)j * 4 * kScanThreads, n);
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanVecs; ++j) s += (v[j].x + v[j].y) + (v[j].z + v[j].w);
  s = wave_sum(s);
  if (lane_id() == 0) wsum[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kScanWaves; ++k) t += wsum[k];
    sums[blockIdx.x] = t;
  }
}

// Single block: exclusive scan of nb tile sums in place (each thread owns a
// contiguous chunk; chunk totals are scanned across the block).
__global__ __launch_bounds__(1024) void scan_top_kernel(uint32_t* __restrict__ sums, int64_t nb) {
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  uint32_t s = 0;
  for (int64_t k = 0; k < per; ++k)
    if (b0 + k < nb) s += sums[b0 + k];
  uint32_t total;
  uint32_t run = block_exclusive_scan<1024>(s, &total);
  for (int64_t k = 0; k < per; ++k)
    if (b0 + k < nb) {
      const uint32_t v = sums[b0 + k];
      sums[b0 + k] = run;
      run += v;
    }
}

// Pair owning entry k of the concatenated cell tables.
__device__ inline int table_pair(const BuildPair* __restrict__ pairs, int n, uint64_t k) {
  int lo = 0, hi = n;  // pairs[lo].tab_off <= k < pairs[hi].tab_off (hi == n: end)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pairs[mid].tab_off <= k) lo = mid; else hi = mid;
  }
  return lo;
}

// Second pass: the tile's chunks are scanned in memory order on top of the
// tile's offset and written back in place.  With `pairs`, the data are the
// concatenated cell-count tables of n pairs, and each entry is written as
// its pair-local target position (global position minus the pair's target
// offset).
template <bool kLocal>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(uint32_t* __restrict__ d, int64_t n,
                                                                  const uint32_t* __restrict__ sums,
                                                                  const BuildPair* __restrict__ pairs,
                                                                  int n_pairs) {
  __shared__ uint32_t wsum[kScanVecs][kScanWaves];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  scan_u4 v[kScanVecs];
  uint32_t s[kScanVecs], x[kScanVecs];
#pragma unroll
  for (int j = 0; j < kScanVecs; ++j) v[j] = scan_load(d, base + (int64_t)j * 4 * kScanThreads, n);
#pragma unroll
  for (int j = 0; j < kScanVecs; ++j) {
    s[j] = (v[j].x + v[j].y) + (v[j].z + v[j].w);
    x[j] = wave_inclusive_sum(s[j]);
    if (lane == kWave - 1) wsum[j][w] = x[j];
  }
  __syncthreads();
  uint32_t run = sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanVecs; ++j) {
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kScanWaves; ++k) {
      if (k < w) before += wsum[j][k];
      all += wsum[j][k];
    }
    uint32_t e = run + before + x[j] - s[j];
    run += all;
    scan_u4 o;
    o.x = e; e += v[j].x;
    o.y = e; e += v[j].y;
    o.z = e; e += v[j].z;
    o.w = e;
    const int64_t i = base + (int64_t)j * 4 * kScanThreads;
    if (kLocal && i < n) {
      int p = table_pair(pairs, n_pairs, (uint64_t)i);
      uint32_t* oe = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        while (p + 1 < n_pairs && (uint64_t)(i + c) >= pairs[p + 1].tab_off) ++p;
        oe[c] -= (uint32_t)pairs[p].tgt_off;
      }
    }
    scan_store(d, i, n, o);
  }
}

// ------------------------------------------------------------------ target grid
__device__ inline int cell_of(float p, double o, double inv_h, int dim) {
  double u = ((double)p - o) * inv_h;
  u = fmin(fmax(u, -2.0), (double)dim + 1.0);
  return (int)floor(u);
}

// Cell key of every target point (global: offset by the pair's table; dense
// or hashed as the pair's grid says) and its rank among the points of its key (order of arrival; the search breaks ties
// by original index, so the order inside a cell never matters).
// With occ_raw, the cell's bit is also set in the pair's raw occupancy bitmap.
__global__ __launch_bounds__(256) void seg_target_key_kernel(const BuildPair* __restrict__ pairs, int n,
                                                             const int64_t* __restrict__ blk_off,
                                                             uint32_t* __restrict__ counts,
                                                             uint32_t* __restrict__ key,
                                                             uint32_t* __restrict__ rank,
                                                             uint32_t* __restrict__ occ_raw) {
  const int p = find_segment(blk_off, n, blockIdx.x);
  const BuildPair& bp = pairs[p];
  const int64_t i = (int64_t)(blockIdx.x - blk_off[p]) * 256 + threadIdx.x;
  if (i >= bp.n_tgt) return;
  const GridDesc g = bp.g;
  const float* t = bp.tgt + 3 * i;
  const int cx = min(max(cell_of(t[0], g.ox, g.inv_h, g.dx), 0), g.dx - 1);
  const int cy = min(max(cell_of(t[1], g.oy, g.inv_h, g.dy), 0), g.dy - 1);
  const int cz = min(max(cell_of(t[2], g.oz, g.inv_h, g.dz), 0), g.dz - 1);
  const uint32_t k = g.hashed ? hashed_slot(g, cx, cy, cz)
                             : ((uint32_t)cz * (uint32_t)g.dy + (uint32_t)cy) * (uint32_t)g.dx + (uint32_t)cx;
  const uint32_t gk = (uint32_t)bp.tab_off + k;
  key[bp.tgt_off + i] = gk;
  const uint32_t rk = atomicAdd(&counts[gk], 1u);
  rank[bp.tgt_off + i] = rk;
  // the first point to reach a cell marks it (one atomic per occupied cell)
  if (rk == 0 && occ_raw && bp.occ_dst && !g.hashed) {
    const uint64_t w = bp.occ_off + ((uint64_t)cz * (uint64_t)g.dy + (uint64_t)cy) * occ_row_words(g.dx) +
                       ((uint32_t)cx >> 5);
    atomicOr(&occ_raw[w], 1u << (cx & 31));
  }
}

// Occupancy of a hashed grid, dilated as it is built: after the scatter, a
// point sets the slots of the in-grid cells around its cell, per row one mask
// for each run that the row's x segment touches (a run's slots are
// consecutive bits of one word), unless one of the (at most 64) points before
// it among its slot's points lies in the same cell.  The first point of every
// cell always sets them, and setting a bit twice changes nothing, so the bound
// only limits the work per point (a cell of many points costs each of them
// 64 comparisons).
__global__ __launch_bounds__(256) void seg_hashed_occ_kernel(const BuildPair* __restrict__ pairs, int n,
                                                             const int64_t* __restrict__ blk_off,
                                                             uint32_t* __restrict__ occ_raw) {
  const int p = find_segment(blk_off, n, blockIdx.x);
  const BuildPair& bp = pairs[p];
  const int64_t j = (int64_t)(blockIdx.x - blk_off[p]) * 256 + threadIdx.x;
  const GridDesc g = bp.g;
  if (!g.hashed || !bp.occ_dst || j >= bp.n_tgt) return;
  auto cell = [&](const float4& q, int* c) {
    c[0] = min(max(cell_of(q.x, g.ox, g.inv_h, g.dx), 0), g.dx - 1);
    c[1] = min(max(cell_of(q.y, g.oy, g.inv_h, g.dy), 0), g.dy - 1);
    c[2] = min(max(cell_of(q.z, g.oz, g.inv_h, g.dz), 0), g.dz - 1);
  };
  int c[3];
  cell(bp.tp_dst[j], c);
  const uint32_t slot0 = hashed_slot(g, c[0], c[1], c[2]);
  const int64_t first = bp.cs_dst[slot0];
  for (int64_t k = j - 64 > first ? j - 64 : first; k < j; ++k) {
    int o[3];
    cell(bp.tp_dst[k], o);
    if (o[0] == c[0] && o[1] == c[1] && o[2] == c[2]) return;  // not the cell's first point
  }
  const int x0 = max(c[0] - 1, 0), x1 = min(c[0] + 1, g.dx - 1);
  const int xs = x1 & ~(kHashRun - 1);  // first x of x1's run
  for (int z = max(c[2] - 1, 0); z <= min(c[2] + 1, g.dz - 1); ++z)
    for (int y = max(c[1] - 1, 0); y <= min(c[1] + 1, g.dy - 1); ++y)
      for (int part = 0; part < 2; ++part) {
        if (part == 1 && xs <= x0) break;
        const int a = part == 0 ? x0 : xs;
        const int b = (part == 0 && xs > x0) ? xs - 1 : x1;
        const uint32_t slot = hashed_slot(g, a, y, z);
        const uint32_t mask = (uint32_t)((1ull << (b - a + 1)) - 1ull) << (slot & 31u);
        atomicOr(&occ_raw[bp.occ_off + (slot >> 5)], mask);
      }
}

// Dilation of each pair's raw occupancy bitmap over the 27-cell
// neighbourhood (a hashed grid's map is dilated as it is built and only
// copied): word (z, y, wi) of the result is the OR over the rows
// (y + dy, z + dz), |dy|, |dz| <= 1, inside the grid, of the row's words
// wi - 1 .. wi + 1 spread by one bit to each side.
__global__ __launch_bounds__(256) void occ_dilate_kernel(const BuildPair* __restrict__ pairs, int n,
                                                         const int64_t* __restrict__ blk_off,
                                                         const uint32_t* __restrict__ raw) {
  const int p = find_segment(blk_off, n, blockIdx.x);
  const BuildPair& bp = pairs[p];
  const GridDesc g = bp.g;
  const uint32_t W = occ_row_words(g.dx);
  const int64_t w = (int64_t)(blockIdx.x - blk_off[p]) * 256 + threadIdx.x;
  if (!bp.occ_dst || (uint64_t)w >= occ_words(g)) return;
  if (g.hashed) {  // dilated as it was built
    bp.occ_dst[w] = raw[bp.occ_off + w];
    return;
  }
  const int64_t row = w / W;
  const int wi = (int)(w - row * W);
  const int y = (int)(row % g.dy), z = (int)(row / g.dy);
  const uint32_t* base = raw + bp.occ_off;
  uint32_t d = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = z + dz;
    if (zz < 0 || zz >= g.dz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = y + dy;
      if (yy < 0 || yy >= g.dy) continue;
      const uint32_t* r = base + ((int64_t)zz * g.dy + yy) * W;
      const uint32_t c = r[wi];
      const uint32_t l = wi > 0 ? r[wi - 1] : 0u;
      const uint32_t h = wi + 1 < (int)W ? r[wi + 1] : 0u;
      // bit j of the row word covers x = 32 wi + j: its x - 1 neighbour is
      // bit j - 1 (or bit 31 of the word before), its x + 1 neighbour bit
      // j + 1 (or bit 0 of the word after)
      d |= c | (c << 1) | (c >> 1) | (l >> 31) | (h << 31);
    }
  }
  bp.occ_dst[w] = d;
}

// After the scan, the concatenated tables hold each cell's first position
// among its own pair's targets.
__global__ __launch_bounds__(256) void seg_target_scatter_kernel(
    const BuildPair* __restrict__ pairs, int n, const int64_t* __restrict__ blk_off,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
    const uint32_t* __restrict__ cs_all) {
  const int p = find_segment(blk_off, n, blockIdx.x);
  const BuildPair& bp = pairs[p];
  const int64_t i = (int64_t)(blockIdx.x - blk_off[p]) * 256 + threadIdx.x;
  if (i >= bp.n_tgt) return;
  const int64_t gi = bp.tgt_off + i;
  const uint32_t pos = cs_all[key[gi]] + rank[gi];
  const float* t = bp.tgt + 3 * i;
  bp.tp_dst[pos] = make_float4(t[0], t[1], t[2], __uint_as_float((uint32_t)i));
  if (bp.tgt_n && bp.tn_dst) {
    const float* m = bp.tgt_n + 3 * i;
    bp.tn_dst[pos] = make_float4(m[0], m[1], m[2], 0.0f);
  }
}

// Copy of each pair's table out of the concatenation into its own buffer
// (only launched when some pair's buffer is not its slice of the
// concatenation).
__global__ __launch_bounds__(256) void seg_table_copy_kernel(const BuildPair* __restrict__ pairs, int n,
                                                             const int64_t* __restrict__ blk_off,
                                                             const uint32_t* __restrict__ cs_all) {
  const int p = find_segment(blk_off, n, blockIdx.x);
  const BuildPair& bp = pairs[p];
  const int64_t k = (int64_t)(blockIdx.x - blk_off[p]) * 256 + threadIdx.x;
  if (k > (int64_t)bp.g.ncell || bp.cs_dst == cs_all + bp.tab_off) return;
  bp.cs_dst[k] = cs_all[bp.tab_off + k];
}

// ------------------------------------------------------------------ stable LSD radix sort
// Keys are one or two 32-bit words (lo, hi); the sort orders by hi, then lo,
// then by input position (stability).  Values ride along.  One pass per 8-bit
// digit: per-tile digit counts, a scan of each digit's column of counts, and
// a scatter that orders its tile in LDS before writing it out.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kWaveSpan = kWave * kSortRounds;  // consecutive items per wave
constexpr int kDigits = 256;

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                                  int64_t n, int shift,
                                                                  uint32_t* __restrict__ hist,
                                                                  int nblk) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  uint32_t d[kSortRounds];
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k) {
    const int64_t i = tile + k * kSortThreads + threadIdx.x;
    d[k] = i < n ? (keys[i] >> shift) & 255u : kDigits;
  }
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k)
    if (d[k] < kDigits) atomicAdd(&h[d[k]], 1u);
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Block d: exclusive scan in place of digit d's per-tile counts
// hist[d * nblk + b] over b; dtot[d] = the digit's count over all tiles.
__global__ __launch_bounds__(256) void radix_colscan_kernel(uint32_t* __restrict__ hist, int nblk,
                                                            uint32_t* __restrict__ dtot) {
  uint32_t* col = hist + (int64_t)blockIdx.x * nblk;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nblk; c0 += 4 * 256) {
    const int i = c0 + 4 * (int)threadIdx.x;
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (i + k < nblk) ? col[i + k] : 0u;
    uint32_t total;
    uint32_t e = carry + block_exclusive_scan<256>((v[0] + v[1]) + (v[2] + v[3]), &total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i + k < nblk) col[i + k] = e;
      e += v[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Stable scatter by one 8-bit digit of the lo (on_hi false) or hi key word.
// Wave w takes items [w * kWaveSpan, (w + 1) * kWaveSpan) of the tile; ranks
// inside a wave come from ballots on the digit bits and the wave's running
// per-digit counts, so the tile is ordered by (digit, input position) in LDS
// and written out in that order, each digit's run at its global offset.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ klo, const uint32_t* __restrict__ khi,
    const uint32_t* __restrict__ vals, int64_t n, bool on_hi, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dtot, int nblk,
    uint32_t* __restrict__ klo_out, uint32_t* __restrict__ khi_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t cnt[kSortWaves][kDigits];
  __shared__ uint32_t gstart[kDigits];
  __shared__ uint32_t s_lo[kSortTile], s_hi[kSortTile], s_val[kSortTile];
  const int t = threadIdx.x, w = t / kWave, lane = lane_id();
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  const int64_t wbase = tile + (int64_t)w * kWaveSpan;
  uint32_t lo[kSortRounds], hi[kSortRounds], va[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = wbase + r * kWave + lane;
    const bool valid = i < n;
    lo[r] = valid ? klo[i] : 0u;
    hi[r] = (valid && khi) ? khi[i] : 0u;
    va[r] = valid ? vals[i] : 0u;
  }
  const uint32_t my_tot = dtot[t];
  const uint32_t my_before = hist[(int64_t)t * nblk + blockIdx.x];
#pragma unroll
  for (int k = 0; k < kSortWaves; ++k) cnt[k][t] = 0;
  __syncthreads();

  // ranks inside the wave (the wave's own counters only: no block barrier)
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t rk[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool valid = wbase + r * kWave + lane < n;
    const uint32_t d = ((on_hi ? hi[r] : lo[r]) >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t before = cnt[w][d];
    rk[r] = before + below;
    if (valid && below == 0) cnt[w][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();

  // thread t = digit t: tile-local start of the digit and of each wave's part
  const uint32_t c0 = cnt[0][t], c1 = cnt[1][t], c2 = cnt[2][t], c3 = cnt[3][t];
  uint32_t tile_total, all;
  const uint32_t loc = block_exclusive_scan<kSortThreads>((c0 + c1) + (c2 + c3), &tile_total);
  const uint32_t dbase = block_exclusive_scan<kSortThreads>(my_tot, &all);
  static_assert(kSortWaves == 4, "wave parts below assume 4 waves");
  cnt[0][t] = loc;
  cnt[1][t] = loc + c0;
  cnt[2][t] = loc + c0 + c1;
  cnt[3][t] = loc + c0 + c1 + c2;
  gstart[t] = dbase + my_before - loc;
  __syncthreads();

#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    if (wbase + r * kWave + lane < n) {
      const uint32_t d = ((on_hi ? hi[r] : lo[r]) >> shift) & 255u;
      const uint32_t lp = cnt[w][d] + rk[r];
      s_lo[lp] = lo[r];
      s_hi[lp] = hi[r];
      s_val[lp] = va[r];
    }
  }
  __syncthreads();

  const int64_t valid_n = min((int64_t)kSortTile, n - tile);
#pragma unroll
  for (int k = 0; k < kSortRounds; ++k) {
    const int lp = k * kSortThreads + t;
    if (lp < valid_n) {
      const uint32_t xl = s_lo[lp], xh = s_hi[lp];
      const uint32_t d = ((on_hi ? xh : xl) >> shift) & 255u;
      const uint32_t dst = gstart[d] + (uint32_t)lp;
      klo_out[dst] = xl;
      if (khi_out) khi_out[dst] = xh;
      vals_out[dst] = s_val[lp];
    }
  }
}

// ------------------------------------------------------------------ source ordering
__device__ inline uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Morton code of every source point over 1024^3 cells spanning its own cloud's
// box (lo word), pair index (hi word), global index (value).
__global__ __launch_bounds__(256) void seg_source_key_kernel(const BuildPair* __restrict__ pairs, int n,
                                                             const int64_t* __restrict__ blk_off,
                                                             uint32_t* __restrict__ klo,
                                                             uint32_t* __restrict__ khi,
                                                             uint32_t* __restrict__ vals) {
  const int p = find_segment(blk_off, n, blockIdx.x);
  const BuildPair& bp = pairs[p];
  const int64_t i = (int64_t)(blockIdx.x - blk_off[p]) * 256 + threadIdx.x;
  if (i >= bp.n_src) return;
  const float* s = bp.src + 3 * i;
  const int cx = min(max(cell_of(s[0], bp.sox, bp.sinv_h, 1024), 0), 1023);
  const int cy = min(max(cell_of(s[1], bp.soy, bp.sinv_h, 1024), 0), 1023);
  const int cz = min(max(cell_of(s[2], bp.soz, bp.sinv_h, 1024), 0), 1023);
  const int64_t gi = bp.src_off + i;
  klo[gi] = spread10(cx) | (spread10(cy) << 1) | (spread10(cz) << 2);
  if (khi) khi[gi] = (uint32_t)p;
  vals[gi] = (uint32_t)gi;
}

// Ordered position -> pair (positions are grouped by pair after the sort),
// copy the point into the structure-of-arrays source and record its index
// inside its own cloud.
__global__ __launch_bounds__(256) void source_gather_kernel(const BuildPair* __restrict__ pairs, int n,
                                                            const int64_t* __restrict__ src_off,
                                                            int64_t total,
                                                            const uint32_t* __restrict__ sorted_vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int p = find_segment(src_off, n, i);
  const BuildPair& bp = pairs[p];
  const int64_t local = (int64_t)sorted_vals[i] - bp.src_off;
  const int64_t pos = i - bp.src_off;
  const float* s = bp.src + 3 * local;
  bp.sx_dst[pos] = s[0];
  bp.sy_dst[pos] = s[1];
  bp.sz_dst[pos] = s[2];
  bp.perm_dst[pos] = (uint32_t)local;
}

// ------------------------------------------------------------------ voxel downsampling
// Voxel key (< 2^48) split into words: lo = bits 0..31, hi = (cloud << 16) |
// bits 32..47, so one sort orders by cloud, then key, then original index.
__global__ __launch_bounds__(256) void seg_voxel_key_kernel(const VoxCloud* __restrict__ clouds, int n,
                                                            const int64_t* __restrict__ blk_off,
                                                            uint32_t* __restrict__ klo,
                                                            uint32_t* __restrict__ khi,
                                                            uint32_t* __restrict__ vals) {
  const int c = find_segment(blk_off, n, blockIdx.x);
  const VoxCloud& vc = clouds[c];
  const int64_t i = (int64_t)(blockIdx.x - blk_off[c]) * 256 + threadIdx.x;
  if (i >= vc.n) return;
  const float* p = vc.pts + 3 * i;
  const int cx = min(max(cell_of(p[0], vc.ox, vc.inv_v, vc.dx), 0), vc.dx - 1);
  const int cy = min(max(cell_of(p[1], vc.oy, vc.inv_v, vc.dy), 0), vc.dy - 1);
  const int cz = min(max(cell_of(p[2], vc.oz, vc.inv_v, vc.dz), 0), vc.dz - 1);
  const uint64_t key = ((uint64_t)cz * (uint64_t)vc.dy + (uint64_t)cy) * (uint64_t)vc.dx + (uint64_t)cx;
  const int64_t gi = vc.off + i;
  klo[gi] = (uint32_t)key;
  if (khi) khi[gi] = ((uint32_t)c << 16) | (uint32_t)(key >> 32);
  vals[gi] = (uint32_t)gi;
}

// flags[i] = 1 where a new voxel starts in the sorted order.
__global__ __launch_bounds__(256) void voxel_flag_kernel(const uint32_t* __restrict__ klo,
                                                         const uint32_t* __restrict__ khi,
                                                         int64_t total, uint32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  bool f = i == 0 || klo[i] != klo[i - 1];
  if (khi && i > 0) f = f || khi[i] != khi[i - 1];
  flags[i] = f ? 1u : 0u;
}

// After the exclusive scan of the flags (vid = voxel index of each start):
// starts[vid] = sorted position where the voxel begins.
__global__ __launch_bounds__(256) void voxel_start_kernel(const uint32_t* __restrict__ klo,
                                                          const uint32_t* __restrict__ khi,
                                                          const uint32_t* __restrict__ vid,
                                                          int64_t total, uint32_t* __restrict__ starts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  bool f = i == 0 || klo[i] != klo[i - 1];
  if (khi && i > 0) f = f || khi[i] != khi[i - 1];
  if (f) starts[vid[i]] = (uint32_t)i;
  if (i == total - 1) starts[vid[i] + (f ? 1u : 0u)] = (uint32_t)total;
}

// One thread per voxel: float64 sums over its members in sorted order (the
// stable sort keeps original-index order inside a voxel).
__global__ __launch_bounds__(256) void voxel_reduce_kernel(const VoxCloud* __restrict__ clouds, int n,
                                                           const int64_t* __restrict__ pt_off,
                                                           const uint32_t* __restrict__ vid,
                                                           const uint32_t* __restrict__ flags,
                                                           const uint32_t* __restrict__ starts,
                                                           const uint32_t* __restrict__ sorted_vals,
                                                           int64_t total) {
  const int64_t nvox = (int64_t)vid[total - 1] + (int64_t)flags[total - 1];
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  const uint32_t b = starts[v], e = starts[v + 1];
  const int c = find_segment(pt_off, n, (int64_t)b);
  const VoxCloud& vc = clouds[c];
  const int64_t local_v = v - (int64_t)vid[vc.off];
  if (local_v >= vc.out_cap) return;
  double sx = 0.0, sy = 0.0, sz = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
  for (uint32_t k = b; k < e; ++k) {
    const int64_t li = (int64_t)sorted_vals[k] - vc.off;
    const float* p = vc.pts + 3 * li;
    sx = sx + (double)p[0];
    sy = sy + (double)p[1];
    sz = sz + (double)p[2];
    if (vc.nrm) {
      const float* q = vc.nrm + 3 * li;
      nx = nx + (double)q[0];
      ny = ny + (double)q[1];
      nz = nz + (double)q[2];
    }
  }
  const double cnt = (double)(e - b);
  vc.out_pts[3 * local_v + 0] = (float)(sx / cnt);
  vc.out_pts[3 * local_v + 1] = (float)(sy / cnt);
  vc.out_pts[3 * local_v + 2] = (float)(sz / cnt);
  if (vc.nrm && vc.out_nrm) {
    const double len = sqrt((nx * nx + ny * ny) + nz * nz);
    float o0, o1, o2;
    if (len < 1e-12) {
      const float* q = vc.nrm + 3 * ((int64_t)sorted_vals[b] - vc.off);
      o0 = q[0]; o1 = q[1]; o2 = q[2];
    } else {
      o0 = (float)(nx / len); o1 = (float)(ny / len); o2 = (float)(nz / len);
    }
    vc.out_nrm[3 * local_v + 0] = o0;
    vc.out_nrm[3 * local_v + 1] = o1;
    vc.out_nrm[3 * local_v + 2] = o2;
  }
}

// Voxel count of every cloud: first voxel index of the next cloud minus its own.
__global__ void voxel_count_kernel(const VoxCloud* __restrict__ clouds, int n,
                                   const uint32_t* __restrict__ vid, const uint32_t* __restrict__ flags,
                                   int64_t total, int64_t* __restrict__ counts) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int64_t first = vid[clouds[c].off];
  const int64_t last_plus = (c + 1 < n) ? (int64_t)vid[clouds[c + 1].off]
                                        : (int64_t)vid[total - 1] + (int64_t)flags[total - 1];
  counts[c] = last_plus - first;
}

}  // namespace

// ====================================================================== launchers
int64_t scan_block_sums_needed(int64_t n) { return ceil_div(std::max<int64_t>(n, 1), kScanTile); }

// Exclusive scan in place; with `pairs`, of the n_pairs concatenated cell
// tables, written as pair-local positions.
static hipError_t scan_exclusive(uint32_t* data, int64_t n, uint32_t* block_sums, int64_t cap_blocks,
                                 const BuildPair* pairs, int n_pairs, hipStream_t s) {
  const int64_t nb = ceil_div(n, kScanTile);
  if (nb > cap_blocks || (reinterpret_cast<uintptr_t>(data) & 15u) != 0) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_tile_sums_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n,
                     block_sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, s, block_sums, nb);
  if (pairs)
    hipLaunchKernelGGL(scan_apply_kernel<true>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n,
                       block_sums, pairs, n_pairs);
  else
    hipLaunchKernelGGL(scan_apply_kernel<false>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n,
                       block_sums, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_scan_exclusive(uint32_t* data, int64_t n, uint32_t* block_sums, int64_t cap_blocks,
                                 hipStream_t s) {
  return scan_exclusive(data, n, block_sums, cap_blocks, nullptr, 0, s);
}

int64_t bbox_blocks(int64_t n) { return std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(n, 256))); }

hipError_t launch_seg_bbox(const SegCloud* clouds, int n_clouds, const int64_t* blk_off,
                           int64_t total_blocks, float* block_out, float* out, hipStream_t s) {
  hipLaunchKernelGGL(seg_bbox_kernel, dim3((unsigned)total_blocks), dim3(256), 0, s, clouds, n_clouds,
                     blk_off, block_out);
  hipLaunchKernelGGL(seg_bbox_final_kernel, dim3((unsigned)n_clouds), dim3(256), 0, s, blk_off,
                     block_out, out);
  return hipGetLastError();
}

hipError_t launch_seg_targets(const BuildPair* pairs, int n, const int64_t* blk_off,
                              int64_t total_blocks, const int64_t* tab_blk_off,
                              int64_t tab_blocks, uint64_t total_tab, uint32_t* counts,
                              uint32_t* key, uint32_t* rank, uint32_t* scan_tmp, int64_t scan_cap,
                              bool copy_tables, uint32_t* occ_raw, hipStream_t s) {
  hipError_t e = hipMemsetAsync(counts, 0, sizeof(uint32_t) * (size_t)total_tab, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(seg_target_key_kernel, dim3((unsigned)total_blocks), dim3(256), 0, s, pairs, n,
                     blk_off, counts, key, rank, occ_raw);
  e = scan_exclusive(counts, (int64_t)total_tab, scan_tmp, scan_cap, pairs, n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(seg_target_scatter_kernel, dim3((unsigned)total_blocks), dim3(256), 0, s, pairs,
                     n, blk_off, key, rank, counts);
  if (copy_tables)
    hipLaunchKernelGGL(seg_table_copy_kernel, dim3((unsigned)tab_blocks), dim3(256), 0, s, pairs, n,
                       tab_blk_off, counts);
  return hipGetLastError();
}

hipError_t launch_occ_clear(uint32_t* occ_raw, uint64_t total_occ, hipStream_t s) {
  return hipMemsetAsync(occ_raw, 0, sizeof(uint32_t) * (size_t)total_occ, s);
}

hipError_t launch_hashed_occ(const BuildPair* pairs, int n, const int64_t* blk_off, int64_t total_blocks,
                             uint32_t* occ_raw, hipStream_t s) {
  if (total_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(seg_hashed_occ_kernel, dim3((unsigned)total_blocks), dim3(256), 0, s, pairs, n, blk_off,
                     occ_raw);
  return hipGetLastError();
}

hipError_t launch_occ_dilate(const BuildPair* pairs, int n, const int64_t* occ_blk_off, int64_t occ_blocks,
                             const uint32_t* occ_raw, hipStream_t s) {
  if (occ_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(occ_dilate_kernel, dim3((unsigned)occ_blocks), dim3(256), 0, s, pairs, n, occ_blk_off,
                     occ_raw);
  return hipGetLastError();
}

int64_t voxel_scratch_words(int64_t total) { return total + 1; }

int64_t radix_hist_needed(int64_t n) {
  return (int64_t)kDigits * ceil_div(std::max<int64_t>(n, 1), kSortTile) + kDigits;
}

// Stable LSD sort of (lo, hi, val) triples: 8-bit digits of lo from bit 0 up
// to lo_bits, then of hi from bit hi_from up to hi_bits (hi only if `two`).
// *out_cur receives the buffer index (0 or 1) holding the result.
static hipError_t radix_sort(SortBufs sb, bool two, int64_t total, int lo_bits, int hi_from,
                             int hi_bits, uint32_t* hist, int64_t hist_cap, hipStream_t s,
                             int* out_cur) {
  const int nblk = (int)ceil_div(std::max<int64_t>(total, 1), kSortTile);
  if ((int64_t)kDigits * nblk + kDigits > hist_cap) return hipErrorInvalidValue;
  if (total >= (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  uint32_t* dtot = hist + (int64_t)kDigits * nblk;
  int cur = 0;
  auto pass = [&](bool on_hi, int shift) -> hipError_t {
    const uint32_t* dig = on_hi ? sb.khi[cur] : sb.klo[cur];
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblk), dim3(kSortThreads), 0, s, dig, total, shift,
                       hist, nblk);
    hipLaunchKernelGGL(radix_colscan_kernel, dim3(kDigits), dim3(256), 0, s, hist, nblk, dtot);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblk), dim3(kSortThreads), 0, s, sb.klo[cur],
                       two ? sb.khi[cur] : nullptr, sb.val[cur], total, on_hi, shift, hist, dtot, nblk,
                       sb.klo[cur ^ 1], two ? sb.khi[cur ^ 1] : nullptr, sb.val[cur ^ 1]);
    cur ^= 1;
    return hipGetLastError();
  };
  hipError_t e;
  for (int shift = 0; shift < lo_bits; shift += 8)
    if ((e = pass(false, shift)) != hipSuccess) return e;
  for (int shift = hi_from; two && shift < hi_bits; shift += 8)
    if ((e = pass(true, shift)) != hipSuccess) return e;
  *out_cur = cur;
  return hipSuccess;
}

hipError_t launch_seg_voxel(const VoxCloud* clouds, int n, bool wide_keys, const int64_t* blk_off,
                            int64_t total_blocks, const int64_t* pt_off, int64_t total, SortBufs sb,
                            uint32_t* hist, int64_t hist_cap, uint32_t* flags, uint32_t* starts,
                            uint32_t* scan_tmp, int64_t scan_cap, int64_t* counts_out,
                            hipStream_t s) {
  const bool two = n > 1 || wide_keys;
  hipLaunchKernelGGL(seg_voxel_key_kernel, dim3((unsigned)total_blocks), dim3(256), 0, s, clouds, n,
                     blk_off, sb.klo[0], two ? sb.khi[0] : nullptr, sb.val[0]);
  int cloud_bits = 0;
  while ((1 << cloud_bits) < n) ++cloud_bits;
  int cur = 0;
  hipError_t e = radix_sort(sb, two, total, 32, wide_keys ? 0 : 16, 16 + cloud_bits, hist, hist_cap,
                            s, &cur);
  if (e != hipSuccess) return e;
  const uint32_t* klo = sb.klo[cur];
  const uint32_t* khi = two ? sb.khi[cur] : nullptr;
  const unsigned nb = (unsigned)ceil_div(total, 256);
  hipLaunchKernelGGL(voxel_flag_kernel, dim3(nb), dim3(256), 0, s, klo, khi, total, flags);
  // vid = exclusive scan of a copy of the flags (kept for the counts)
  e = hipMemcpyAsync(starts, flags, sizeof(uint32_t) * (size_t)total, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  e = launch_scan_exclusive(starts, total, scan_tmp, scan_cap, s);
  if (e != hipSuccess) return e;
  // `starts` now holds vid; the voxel starts (nvox + 1 <= total + 1 entries)
  // go into the key buffer that the sort no longer needs, which the caller
  // sizes to total + 1 words
  uint32_t* vid = starts;
  uint32_t* vstart = sb.klo[cur ^ 1];
  hipLaunchKernelGGL(voxel_start_kernel, dim3(nb), dim3(256), 0, s, klo, khi, vid, total, vstart);
  hipLaunchKernelGGL(voxel_reduce_kernel, dim3(nb), dim3(256), 0, s, clouds, n, pt_off, vid, flags,
                     vstart, sb.val[cur], total);
  hipLaunchKernelGGL(voxel_count_kernel, dim3((unsigned)ceil_div(n, 64)), dim3(64), 0, s, clouds, n,
                     vid, flags, total, counts_out);
  return hipGetLastError();
}

hipError_t launch_seg_sources(const BuildPair* pairs, int n, const int64_t* blk_off,
                              int64_t total_blocks, const int64_t* src_off, int64_t total,
                              SortBufs sb, uint32_t* hist, int64_t hist_cap, hipStream_t s) {
  const bool two = n > 1;
  hipLaunchKernelGGL(seg_source_key_kernel, dim3((unsigned)total_blocks), dim3(256), 0, s, pairs, n,
                     blk_off, sb.klo[0], two ? sb.khi[0] : nullptr, sb.val[0]);
  int hi_bits = 0;
  while ((1 << hi_bits) < n) ++hi_bits;
  // Morton codes have 30 bits; pair indices hi_bits
  int cur = 0;
  const hipError_t e = radix_sort(sb, two, total, 30, 0, hi_bits, hist, hist_cap, s, &cur);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(source_gather_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, pairs,
                     n, src_off, total, sb.val[cur]);
  return hipGetLastError();
}

}  // namespace icp
