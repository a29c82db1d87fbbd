// Internal declarations shared by the kernel and runtime translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icp {

constexpr int kBlock = 256;        // threads per block of the pass kernel
constexpr int kTile = 256;         // queries per block of the pass kernel (one per thread)
constexpr int kNumSums = 29;       // 21 (J^T J upper) + 6 (J^T r) + sum d2 + count
constexpr int kSumD2 = 27;
constexpr int kSumCount = 28;
// Segments of a pair's tile partials in the two-level reduction (the reduce
// kernel's blocks; the solve adds the segment sums): 64, or kSegs for pairs
// of more than 4096 tiles.  Segment sums are stored with a stride of kSegs.
constexpr int kSegs = 256;
__host__ __device__ inline int segs_of(int n_blocks) { return n_blocks > 4096 ? kSegs : 64; }

// Uniform voxel grid over the target: cell = floor((p - origin) * inv_h) per
// axis in float64.  The cell edge is >= r (1 + 2^-10) / sub, so a query's
// candidates lie in the (2 sub + 1)^3 cells around its own.  The cell table
// holds, for each key, the first position of its points in the key-ordered
// target (ncell + 1 entries).
//   dense:  key = (cz * dy + cy) * dx + cx, one entry per cell of the box;
//   hashed: for boxes whose dense table would be too large (a few far
//           outliers, say), key = hashed_slot(cx, cy, cz) over ncell slots
//           (a power of two).  Distinct cells may share a slot: a lookup then
//           yields extra target points, which the distance test sorts out,
//           and never misses one.
struct GridDesc {
  double ox, oy, oz;
  double inv_h;
  int32_t dx, dy, dz;
  uint32_t ncell;   // dense: dx * dy * dz; hashed: number of slots
  int32_t sub;      // 1 or 2
  int32_t hashed;   // 0 dense, 1 hashed
};

// Hashed keys: the cells of a run of kHashRun consecutive x (same y, z, x
// aligned to the run) take kHashRun consecutive slots at a hashed position,
// so the cells [x0, x1] of one run form one slot range and one range of the
// target.  A row segment of at most 2 sub + 1 <= kHashRun cells spans at most
// two runs.
constexpr int kHashRunBits = 5;
constexpr int kHashRun = 1 << kHashRunBits;
__host__ __device__ inline uint32_t hashed_slot(const GridDesc& g, int32_t x, int32_t y, int32_t z) {
  uint32_t h = ((uint32_t)x >> kHashRunBits) * 0x9E3779B1u;
  h ^= (uint32_t)y * 0x85EBCA77u;
  h ^= (uint32_t)z * 0xC2B2AE3Du;
  // finalising mix (xor-shift / odd multiply rounds) so that the low bits
  // depend on every input bit
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  const uint32_t runs = g.ncell >> kHashRunBits;
  return ((h & (runs - 1u)) << kHashRunBits) | ((uint32_t)x & (uint32_t)(kHashRun - 1));
}

// Occupancy bitmap of a grid, read by the pass through the dilated map, whose
// bit for a cell is set when any of the 27 cells around it holds a target
// point.
//   dense:  one bit per cell, rows of the x axis padded to whole 32-bit words:
//           the bit of cell (x, y, z) is bit (x & 31) of word
//           (z * dy + y) * occ_row_words(dx) + (x >> 5);
//   hashed: one bit per slot (bit s & 31 of word s >> 5 for slot s); each
//           occupied cell sets the bits of its 27 neighbours' slots, so a
//           clear bit still proves an empty neighbourhood (cells that share a
//           slot can only set more bits).
__host__ __device__ inline uint32_t occ_row_words(int32_t dx) { return ((uint32_t)dx + 31u) >> 5; }
__host__ __device__ inline uint64_t occ_words(const GridDesc& g) {
  return g.hashed ? (uint64_t)(g.ncell >> 5) : (uint64_t)g.dy * (uint64_t)g.dz * occ_row_words(g.dx);
}

// Device-resident loop state of one registration.
struct IterState {
  double T[16];
  double fitness;
  double rmse;
  double e_prev;
  int64_t n_in;
  int64_t n_prev;
  int32_t k;       // index of the next pass
  int32_t done;    // set once the loop has stopped; later launches exit at once
  int32_t status;  // ICP_OK / ICP_CONVERGED / ICP_DEGENERATE
  int32_t pad;
  double sums[kNumSums];  // reduce-only mode output
};

struct PassArgs {
  const float* sx;        // cell-ordered source SoA
  const float* sy;
  const float* sz;
  const uint32_t* sperm;  // cell-ordered position -> original source index
  int32_t n_src;
  const float4* tp;       // cell-ordered target (x, y, z, bit pattern of original index)
  const float4* tn;       // cell-ordered target normals (nx, ny, nz, 0)
  const uint32_t* cs;     // cell start table, ncell + 1 entries (positions into tp)
  const uint32_t* occ;    // optional dilated occupancy bitmap of the grid (occ_words(g) words)
  GridDesc g;
  float r2f;              // (float)(max_corr_dist^2)
  float inv_h2;           // (float)(inv_h^2)
  int32_t n_tgt;
  uint32_t* jprev;        // optional per-query match of the previous pass (warm start), in/out
  const IterState* st;
  double* part;           // [kNumSums][n_blocks] block partials
  int32_t n_blocks;
  int32_t* idx_out;       // optional (correspondence hook)
  float* d2_out;
  // robust loss (IRLS): 0 none, 1 Huber, 2 Tukey, 3 Cauchy, scale k
  int32_t loss;
  float loss_k32;
  double loss_k;
};

// Normal estimation over one cloud that has been prepared as both source
// (Morton-ordered queries) and target (cell-ordered grid, one float4 per
// point).
constexpr int kNormBlock = 64;    // threads per block of the normals kernel (one wave)
constexpr int kMaxNormalNN = 64;  // largest max_nn (per-lane heap in LDS)
struct NormalArgs {
  const float* sx;        // Morton-ordered points
  const float* sy;
  const float* sz;
  const uint32_t* sperm;  // Morton position -> original index
  int32_t n;
  const float4* tp;       // cell-ordered points (x, y, z, original index bits)
  const uint32_t* cs;     // cell start table
  GridDesc g;
  float r2f;              // (float)(radius^2)
  float inv_h2;
  int32_t max_nn;
  double vx, vy, vz;      // viewpoint
  float* normals;         // (n, 3), original order
  int32_t* counts;        // (n), original order, or null
};

// RANSAC validation: hypothesis v's transform T[v] (3x4 row-major, FP64) is
// scored over every source point of a prepared pair with the pass's
// correspondence rule: count of inliers and sumq = sum of floor(d2 * 2^shift)
// over them (exact integers).  Blocks write per-tile partials
// [v][tile]; the reduction writes one (count, sumq) per hypothesis.
struct ValidateArgs {
  PassArgs p;                // prepared pair (st, part, jprev, outputs unused)
  const double* T;           // [n_hyp][12]
  int32_t n_hyp;
  int32_t n_tiles;
  double scale;              // 2^shift
  uint32_t* part_cnt;        // [n_hyp][n_tiles]
  uint64_t* part_sq;         // [n_hyp][n_tiles]
  int64_t* cnt_out;          // [n_hyp]
  uint64_t* sq_out;          // [n_hyp]
};
constexpr int kMaxValidateHyp = 65535;  // hypotheses per validation launch

// FPFH descriptors of one cloud prepared as both queries and grid (as for
// normals), one wave per point: the hybrid neighbourhood and its list, the
// SPFH bin counts of the pairs, then the distance-weighted sum.
constexpr int kFpfhBlock = 256;   // threads per block of the FPFH kernels (one wave per point)
constexpr int kMaxFpfhNN = 128;   // largest max_nn (counts fit a byte)
constexpr int kFpfhBins = 33;     // three 11-bin sub-histograms
constexpr int kFpfhCountBytes = 36;  // 33 byte counts per point, padded
struct FpfhArgs {
  const float* sx;        // Morton-ordered points
  const float* sy;
  const float* sz;
  const uint32_t* sperm;  // Morton position -> original index
  int32_t n;
  const float4* tp;       // cell-ordered points (x, y, z, original index bits)
  const uint32_t* cs;     // cell start table
  GridDesc g;
  float r2f;              // (float)(radius^2)
  float inv_h2;
  int32_t max_nn;
  const float* pts;       // (n, 3) original order
  const float* nrm;       // (n, 3) original order, unit normals
  uint8_t* counts;        // (n, 36) bytes: SPFH count of bin b at byte b
  int32_t* k;             // (n) pairs counted
  int32_t* nbr;           // (n, max_nn) neighbour original indices
  int32_t* nn;            // (n) neighbourhood sizes
  float* out;             // (n, 33) descriptors
};

struct SolveArgs {
  const double* part;
  int32_t n_blocks;
  IterState* st;
  int64_t n_src;
  int32_t max_iter;
  double rel_tol;
  int32_t reduce_only;
};

// ---- preparation (icp_build.hip) -----------------------------------------
struct SegCloud {
  const float* pts;  // (n, 3)
  const float* nrm;  // optional (n, 3), checked for finiteness only
  int64_t n;
};

// One pair of a segmented preparation call.  Counting and scanning use
// concatenated scratch (pair p's counts start at tab_off and have g.ncell + 1
// entries; its targets are counted from tgt_off, its sources from src_off);
// the results are written to the pair's own destinations with pair-local
// positions: cs_dst[k] = first position of cell k in tp_dst.
struct BuildPair {
  const float* src;
  const float* tgt;
  const float* tgt_n;  // null: no normals to gather
  int64_t n_src, n_tgt;
  int64_t src_off, tgt_off;
  uint64_t tab_off;
  GridDesc g;
  double sox, soy, soz, sinv_h;  // Morton grid of the source (1024 cells per axis)
  uint32_t* cs_dst;              // g.ncell + 1 entries
  float4* tp_dst;                // n_tgt
  float4* tn_dst;                // n_tgt, or null
  float* sx_dst;                 // n_src each
  float* sy_dst;
  float* sz_dst;
  uint32_t* perm_dst;            // n_src: ordered position -> original source index
  uint64_t occ_off;              // first word of the pair's raw bitmap in the call's scratch
  uint32_t* occ_dst;             // dilated occupancy bitmap (occ_words(g) words), or null
};

struct SortBufs {
  uint32_t* klo[2];
  uint32_t* khi[2];
  uint32_t* val[2];
};

int64_t bbox_blocks(int64_t n);
int64_t scan_block_sums_needed(int64_t n);
int64_t radix_hist_needed(int64_t n);
hipError_t launch_scan_exclusive(uint32_t* data, int64_t n, uint32_t* block_sums, int64_t cap_blocks,
                                 hipStream_t s);
// out: 8 floats per cloud (min xyz, max xyz, non-finite flag)
hipError_t launch_seg_bbox(const SegCloud* clouds, int n_clouds, const int64_t* blk_off,
                           int64_t total_blocks, float* block_out, float* out, hipStream_t s);
// counts: the concatenated tables (total_tab entries, 16-byte aligned); on
// return they hold pair-local cell starts.  copy_tables: also copy each
// pair's table to its cs_dst where that is not its slice of `counts`
// (tab_blk_off: per-pair block offsets over the tables, 256 entries a block).
hipError_t launch_seg_targets(const BuildPair* pairs, int n, const int64_t* blk_off,
                              int64_t total_blocks, const int64_t* tab_blk_off,
                              int64_t tab_blocks, uint64_t total_tab, uint32_t* counts,
                              uint32_t* key, uint32_t* rank, uint32_t* scan_tmp, int64_t scan_cap,
                              bool copy_tables, uint32_t* occ_raw, hipStream_t s);
// Dilated occupancy bitmaps of every pair that has an occ_dst: occ_raw is the
// call's concatenated raw bitmap (total_occ words, zeroed by this call and
// filled by the target key pass, so this runs before launch_seg_targets and
// launch_occ_dilate after it); occ_blk_off: per-pair block offsets over the
// raw words (256 words a block).
hipError_t launch_occ_clear(uint32_t* occ_raw, uint64_t total_occ, hipStream_t s);
hipError_t launch_occ_dilate(const BuildPair* pairs, int n, const int64_t* occ_blk_off, int64_t occ_blocks,
                             const uint32_t* occ_raw, hipStream_t s);
// Dilated occupancy of the pairs with hashed grids, into the raw words (after
// launch_seg_targets, before launch_occ_dilate; blk_off: per-pair blocks over
// the targets, as for launch_seg_targets).
hipError_t launch_hashed_occ(const BuildPair* pairs, int n, const int64_t* blk_off, int64_t total_blocks,
                             uint32_t* occ_raw, hipStream_t s);
hipError_t launch_seg_sources(const BuildPair* pairs, int n, const int64_t* blk_off,
                              int64_t total_blocks, const int64_t* src_off, int64_t total,
                              SortBufs sb, uint32_t* hist, int64_t hist_cap, hipStream_t s);

// ---- voxel downsampling (icp_build.hip) ----------------------------------
// One cloud of a segmented downsampling call.  Voxel of p: floor((p - o) /
// voxel) per axis in float64 (o = the cloud's box minimum), key = (cz * dy +
// cy) * dx + cx < 2^48.  Output (key order): mean position of each occupied
// voxel (float64 sum in original-index order, then rounded), and with normals
// the normalised float64 sum of the members' normals (the first member's
// normal if that sum is shorter than 1e-12).
struct VoxCloud {
  const float* pts;
  const float* nrm;  // optional
  int64_t n;
  int64_t off;       // offset in the concatenation of all clouds' points
  double ox, oy, oz, inv_v;
  int32_t dx, dy, dz;
  int32_t pad;
  float* out_pts;    // capacity out_cap voxels
  float* out_nrm;    // optional
  int64_t out_cap;
};

// counts_out: per cloud, the number of occupied voxels (written even if it
// exceeds out_cap; points beyond the capacity are not written).  Sort buffers,
// `flags` and `starts` hold at least total + 1 words.
// wide_keys: some cloud's key space exceeds 2^32; n <= 65535 clouds.
hipError_t launch_seg_voxel(const VoxCloud* clouds, int n, bool wide_keys, const int64_t* blk_off,
                            int64_t total_blocks, const int64_t* pt_off, int64_t total, SortBufs sb,
                            uint32_t* hist, int64_t hist_cap, uint32_t* flags, uint32_t* starts,
                            uint32_t* scan_tmp, int64_t scan_cap, int64_t* counts_out,
                            hipStream_t s);
int64_t voxel_scratch_words(int64_t total);  // words needed for `flags` and `starts` each

// ---- loop (icp_kernels.hip) ---------------------------------------------
hipError_t launch_state_init(IterState* st, const double T[16], hipStream_t s);
// FPFH descriptors of a prepared cloud (both passes).
hipError_t launch_fpfh(const FpfhArgs& a, int sub, hipStream_t s);
// Normals of a prepared cloud (sub: the grid's neighbourhood radius in cells).
hipError_t launch_normals(const NormalArgs& a, int sub, hipStream_t s);

hipError_t launch_pass(const PassArgs& a, int variant, int precision, bool write_corr, hipStream_t s);
// Scores of a.n_hyp <= kMaxValidateHyp hypotheses (pass kernel and reduction).
hipError_t launch_validate(const ValidateArgs& a, int sub, hipStream_t s);
// Solve of one pair.  `red` (kNumSums * kSegs doubles of scratch, or null) lets
// a pair of many pass blocks reduce its partials with many blocks first; the
// result is the same bits either way.
hipError_t launch_solve(const SolveArgs& a, double* red, hipStream_t s);

// Batched forms: `pairs` / `items` / `arr` are device arrays.
// robust: the pairs' PassArgs carry a loss (the IRLS-weighted kernels).
hipError_t launch_batch_pass(const PassArgs* pairs, const uint2* items, int n_items, int sub,
                             int variant, int precision, bool robust, hipStream_t s);
hipError_t launch_batch_solve(const SolveArgs* arr, int n_pairs, hipStream_t s);

// Graph-node forms of the batched launches: kernel, block and shared memory
// filled in; the caller sets gridDim (work items / pairs) and kernelParams
// ({&pairs, &items} / {&arr}).
void batch_pass_node(int sub, int variant, int precision, bool robust, hipKernelNodeParams* p);
void batch_solve_node(hipKernelNodeParams* p);
// Copies the loop states of `n` batched pairs into one array (one readback).
hipError_t launch_gather_states(const SolveArgs* arr, int n, IterState* out, hipStream_t s);

}  // namespace icp
