// Internal declarations shared by the kernel and runtime translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icp {

constexpr int kBlock = 256;        // threads per block of the pass kernel
constexpr int kTile = 1024;        // queries per block of the pass kernel (4 per thread)
constexpr int kNumSums = 29;       // 21 (J^T J upper) + 6 (J^T r) + sum d2 + count
constexpr int kSumD2 = 27;
constexpr int kSumCount = 28;

// Uniform voxel grid over the target: cell = floor((p - origin) * inv_h) per
// axis in float64; dense key = (cz * dy + cy) * dx + cx.  The cell edge is
// >= r (1 + 2^-10) / sub, so a query's candidates lie in the (2 sub + 1)^3
// cells around its own.
struct GridDesc {
  double ox, oy, oz;
  double inv_h;
  int32_t dx, dy, dz;
  uint32_t ncell;  // dx * dy * dz
  int32_t sub;     // 1 or 2
};

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
  const uint32_t* cs;     // cell start table, ncell + 1 entries
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

// ---- launchers (icp_kernels.hip) ---------------------------------------
hipError_t launch_bbox(const float* pts, const float* nrm, int64_t n, float* block_out, int nblk,
                       float* final_out, hipStream_t s);
int bbox_blocks(int64_t n);

hipError_t launch_scan_exclusive(uint32_t* data, int64_t n, uint32_t* block_sums, int64_t cap_blocks,
                                 hipStream_t s);
int64_t scan_block_sums_needed(int64_t n);

hipError_t launch_target_grid(const float* tgt, const float* tgt_n, int64_t n, const GridDesc& g,
                              uint32_t* key, uint32_t* rank, uint32_t* cs, float4* tp, float4* tn,
                              uint32_t* scan_tmp, int64_t scan_cap, hipStream_t s);

hipError_t launch_source_order(const float* src, int64_t n, double ox, double oy, double oz,
                               double inv_h, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                               uint32_t* vals_alt, uint32_t* hist, int64_t hist_cap, float* sx,
                               float* sy, float* sz, uint32_t** perm_out, hipStream_t s);
int64_t radix_hist_needed(int64_t n);

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                             int64_t n, int key_bits, uint32_t* hist, int64_t hist_cap,
                             uint32_t** keys_out, uint32_t** vals_out, hipStream_t s);

hipError_t launch_state_init(IterState* st, const double T[16], hipStream_t s);

hipError_t launch_pass(const PassArgs& a, int variant, int precision, bool write_corr, hipStream_t s);
hipError_t launch_solve(const SolveArgs& a, hipStream_t s);

// Batched forms: `pairs` / `items` / `arr` are device arrays.
hipError_t launch_batch_pass(const PassArgs* pairs, const uint2* items, int n_items, int sub,
                             int variant, int precision, hipStream_t s);
hipError_t launch_batch_solve(const SolveArgs* arr, int n_pairs, hipStream_t s);

}  // namespace icp
