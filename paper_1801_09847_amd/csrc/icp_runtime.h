// Host-side runtime shared by the C-ABI translation units (plain / batched
// registration, voxel downsampling, the request server).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/icp.h"
#include "icp_internal.h"

namespace icp_rt {

using namespace icp;

extern thread_local std::string g_last_error;

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define HIP_TRY(expr, what)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return ::icp_rt::hip_fail(e_, what); \
  } while (0)

// Fixed device arena of a context created with arena_bytes > 0: the
// buffers of a call are carved from it in turn (a bump pointer that the
// start of every call resets), so calls allocate no device memory, and a call
// whose buffers do not fit fails with ICP_E_OOM.  Resetting at the start of a
// call is safe: every kernel of the context runs on its stream, so the next
// call's work is ordered after the previous call's.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t top = 0;
  uint64_t epoch = 1;  // call counter: a buffer carved in an older call is stale
};

// A device buffer: without an arena it only grows (hipMalloc, reused across
// calls); with one it is carved from the arena once per call.
struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  Arena* arena = nullptr;
  uint64_t epoch = 0;
  hipError_t ensure(size_t bytes) {
    if (arena) {
      if (p && bytes <= cap && epoch == arena->epoch) return hipSuccess;
      const size_t off = (arena->top + 255) & ~(size_t)255;
      const size_t want = std::max<size_t>(bytes, 256);
      if (off > arena->size || want > arena->size - off) {
        p = nullptr;
        cap = 0;
        return hipErrorOutOfMemory;
      }
      p = arena->base + off;
      cap = want;
      epoch = arena->epoch;
      arena->top = off + want;
      return hipSuccess;
    }
    if (bytes <= cap && p) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      cap = 0;
      if (e != hipSuccess) return e;
    }
    const size_t want = std::max<size_t>(bytes + bytes / 8, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  void release() {
    if (p && !arena) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

constexpr size_t kHostBytes = 4096;
constexpr int kDefaultSub = 1;
// A call whose kernels allow it takes two cells per radius when each target
// holds at least this many points per cell of the one-cell-per-radius grid
// (over the whole box): the smaller cells then cut the candidates each query
// scans by more than the extra rows cost.
constexpr double kFineSubPoints = 2.0;

}  // namespace icp_rt

struct icp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // per-call descriptors, loop header, warm-start matches, partials, states
  icp_rt::Buf desc;
  // preparation scratch
  icp_rt::Buf bbox_part, t_key, t_rank, scan_tmp, s_hist;
  icp_rt::Buf sk[6];  // sort buffers: klo[2], khi[2], val[2]
  // prepared pairs (concatenated)
  icp_rt::Buf cs, tp, tn, sx, sy, sz, perm;
  // occupancy bitmaps: raw (scratch of a build) and dilated (read by the pass)
  icp_rt::Buf occ_raw, occ;
  // voxel downsampling: descriptors, scratch, multi-scale level clouds
  icp_rt::Buf vdesc, vflags, vstarts, lvl_src, lvl_tgt, lvl_tn;
  // pose-graph optimisation: poses, edges, terms, normal equations
  icp_rt::Buf pg;
  // RANSAC: hypothesis flags, survivors, validation partials, feature-match keys
  icp_rt::Buf rs;
  void* host = nullptr;  // pinned staging
  size_t host_cap = 0;
  // fixed device arena (arena_bytes > 0 at creation), else growing buffers
  icp_rt::Arena arena;
  bool fixed = false;
  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev;  // [0] call start, [1] call end, [2+2k]/[3+2k] around pass k
  hipEvent_t ev_build[2] = {nullptr, nullptr};  // around the last build (profiling)
  int64_t build_pending = 0;   // target points of a timed build not yet collected
  icp_profile_t prof{};
};

namespace icp_rt {

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int ctx_init(icp_ctx* c, int device, void* stream, size_t arena_bytes = 0);
// Every buffer of a context (arena wiring, release).
template <class F>
void for_each_buf(icp_ctx* c, F f) {
  Buf* bufs[] = {&c->desc, &c->bbox_part, &c->t_key, &c->t_rank, &c->scan_tmp, &c->s_hist,
                 &c->cs, &c->occ_raw, &c->occ, &c->tp, &c->tn, &c->sx, &c->sy, &c->sz, &c->perm, &c->vdesc,
                 &c->vflags, &c->vstarts, &c->lvl_src, &c->lvl_tgt, &c->lvl_tn, &c->pg, &c->rs};
  for (Buf* b : bufs) f(*b);
  for (Buf& b : c->sk) f(b);
}
// The given context, or this thread's default context of the current device.
int resolve_ctx(icp_ctx* in, icp_ctx** out);
// Cells per max_corr_dist along an axis for grids without a density choice
// (the environment override, else the default).
int grid_sub();
void ctx_free(icp_ctx* c);
int ensure_host(icp_ctx* c, size_t bytes);
int check_cloud(const float* p, int64_t n, const char* name);
int check_pose(const double* T, const char* name);
int check_common(const float* src, int64_t n_src, const float* tgt, const float* tgt_n,
                 int64_t n_tgt, const double* T, double r, int32_t variant, int32_t precision,
                 bool need_normals_for_plane);
int check_iteration(int32_t max_iter, double rel_tol);
// Robust loss arguments (kind in ICP_LOSS_*, finite positive scale).
int check_loss(int32_t loss, double k);
// Sets a pass's loss (and its float32 scale).
void set_loss(PassArgs* a, int32_t loss, double k);
size_t align256(size_t x);
int64_t tiles_of(int64_t n);

struct PairIn {
  const float* src;
  int64_t n_src;
  const float* tgt;
  const float* tgt_n;  // null: point-to-point (normals neither checked nor gathered)
  int64_t n_tgt;
  double r;
  bool hashed_ok = false;  // the call's kernels accept a hashed grid (the pass does)
  bool fine_ok = false;    // the call may take two cells per radius for a dense target
};

// Byte offsets of one call's descriptors; the same layout is used in pinned
// host staging and in the context's `desc` device buffer.
struct Layout {
  size_t clouds, blk_bbox, pairs, blk_t, blk_s, src_off, blk_tab, blk_occ;  // preparation
  size_t pargs, sargs, states, items;                                // loop header
  size_t header_end;                                                 // end of uploaded part
  size_t bbox_out, jprev, part, red;                                 // device only
  size_t total;
};

struct Prep {
  int n = 0;
  Layout L;
  std::vector<GridDesc> g;
  std::vector<int64_t> src_off, tgt_off, tile_off;
  std::vector<uint64_t> tab_off;
  std::vector<uint64_t> occ_off;  // per pair: first word of its raw occupancy bitmap
  int64_t total_src = 0, total_tgt = 0, total_tiles = 0;
  uint64_t total_tab = 0;
  uint64_t total_occ = 0;
  int sub = 1;
  bool normals = false;
};

// Destinations of one pair's prepared data (device); perm may alias scratch.
struct PairDst {
  uint32_t* cs;  // g.ncell + 1
  float4* tp;    // n_tgt
  float4* tn;    // n_tgt or null
  float* sx;     // n_src each
  float* sy;
  float* sz;
  uint32_t* perm;
  uint32_t* occ;  // occ_words(g), or null: no occupancy bitmap
};

// Boxes, finiteness and grid sizes of n pairs (one synchronisation).  On a
// non-finite input, *bad receives the pair index and ICP_E_NONFINITE is
// returned.
int plan_pairs(icp_ctx* c, int n, const PairIn* in, Prep* P, int* bad);
// Segmented build of a planned call into dst[] (null: the context's arrays).
int build_pairs(icp_ctx* c, Prep* P, const PairDst* dst);
int prepare_pairs(icp_ctx* c, int n, const PairIn* in, Prep* P);

struct VoxIn {
  const float* pts;
  const float* nrm;  // optional
  int64_t n;
  double voxel;
  float* out_pts;
  float* out_nrm;    // optional
  int64_t cap;
};
int downsample_clouds(icp_ctx* c, int m, const VoxIn* in, int64_t* counts, int* bad);

void to_result(const IterState& st, icp_result_t* out);

}  // namespace icp_rt
