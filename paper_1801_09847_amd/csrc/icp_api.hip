// Host runtime of libicp.so: argument validation, contexts and their device
// workspace, grid construction and the per-iteration launch sequence behind
// the C ABI declared in include/icp.h.
//
// One registration is: finiteness check + bounding boxes (one small readback
// that sizes the grid), target grid build, Morton ordering of the source, then
// max_iter + 1 passes.  Each pass is two launches on the context's stream: the
// fused correspondence / residual / block-reduction kernel and a single-block
// kernel that reduces the block partials in fixed order, solves the 6x6
// system and updates the pose on the device.  The loop state never leaves the
// device until the final readback; once a stopping rule fires, the remaining
// launches return immediately.

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/icp.h"
#include "icp_internal.h"

using namespace icp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? ICP_E_OOM
                                                                                : ICP_E_DEVICE;
  return fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                    \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// A device buffer that only grows (reused across calls).
struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      cap = 0;
      if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes + bytes / 8, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

}  // namespace

struct icp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // workspace
  Buf bbox_part, bbox_out;
  Buf t_key, t_rank, t_cs, t_tp, t_tn, scan_tmp;
  Buf s_keys, s_vals, s_keys2, s_vals2, s_hist, s_x, s_y, s_z;
  Buf part, state, jprev;
  Buf batch;  // persistent per-pair data of icp_register_batch
  void* host = nullptr;  // pinned readback area
  size_t host_cap = 0;
  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev;  // 2 per pass + call start/end
  icp_profile_t prof{};
};

namespace {

constexpr size_t kHostBytes = 4096;
constexpr int kDefaultSub = 1;

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

int ctx_init(icp_ctx* c, int device, void* stream) {
  c->device = device;
  DeviceGuard g(device);
  if (!g.ok) return fail(ICP_E_DEVICE, "cannot select device " + std::to_string(device));
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
    c->own_stream = true;
  }
  HIP_TRY(hipHostMalloc(&c->host, kHostBytes, hipHostMallocDefault), "hipHostMalloc");
  c->host_cap = kHostBytes;
  return ICP_SUCCESS;
}

void ctx_free(icp_ctx* c) {
  DeviceGuard g(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  Buf* bufs[] = {&c->bbox_part, &c->bbox_out, &c->t_key, &c->t_rank, &c->t_cs, &c->t_tp,
                 &c->t_tn, &c->scan_tmp, &c->s_keys, &c->s_vals, &c->s_keys2, &c->s_vals2,
                 &c->s_hist, &c->s_x, &c->s_y, &c->s_z, &c->part, &c->state, &c->jprev, &c->batch};
  for (Buf* b : bufs) b->release();
  if (c->host) (void)hipHostFree(c->host);
  c->host = nullptr;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  c->stream = nullptr;
}

// Per-thread default contexts, one per device.
struct DefaultCtx {
  icp_ctx* c[64] = {};
  ~DefaultCtx() {
    for (auto*& p : c)
      if (p) {
        ctx_free(p);
        delete p;
        p = nullptr;
      }
  }
};
thread_local DefaultCtx g_default;

int resolve_ctx(icp_ctx* in, icp_ctx** out) {
  if (in) {
    *out = in;
    return ICP_SUCCESS;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(ICP_E_DEVICE, "device index out of range");
  if (!g_default.c[dev]) {
    icp_ctx* c = new icp_ctx();
    const int rc = ctx_init(c, dev, nullptr);
    if (rc != ICP_SUCCESS) {
      ctx_free(c);
      delete c;
      return rc;
    }
    g_default.c[dev] = c;
  }
  *out = g_default.c[dev];
  return ICP_SUCCESS;
}

// ------------------------------------------------------------------ validation
int check_cloud(const float* p, int64_t n, const char* name) {
  if (!p) return fail(ICP_E_INVALID_ARG, std::string(name) + " is NULL");
  if (n < 1) return fail(ICP_E_INVALID_ARG, std::string(name) + ": point count must be >= 1");
  if (n > (int64_t)INT32_MAX) return fail(ICP_E_TOO_LARGE, std::string(name) + ": more than 2^31-1 points");
  if ((reinterpret_cast<uintptr_t>(p) & 3u) != 0)
    return fail(ICP_E_INVALID_ARG, std::string(name) + " is not 4-byte aligned");
  return ICP_SUCCESS;
}

int check_pose(const double* T, const char* name) {
  if (!T) return fail(ICP_E_INVALID_ARG, std::string(name) + " is NULL");
  for (int k = 0; k < 16; ++k)
    if (!std::isfinite(T[k])) return fail(ICP_E_INVALID_ARG, std::string(name) + " is not finite");
  if (T[12] != 0.0 || T[13] != 0.0 || T[14] != 0.0 || T[15] != 1.0)
    return fail(ICP_E_INVALID_ARG, std::string(name) + ": last row must be (0, 0, 0, 1)");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += T[4 * k + i] * T[4 * k + j];
      if (fabs(s - (i == j ? 1.0 : 0.0)) > 1e-6)
        return fail(ICP_E_INVALID_ARG, std::string(name) + ": rotation block is not orthonormal");
    }
  return ICP_SUCCESS;
}

int check_common(const float* src, int64_t n_src, const float* tgt, const float* tgt_n,
                 int64_t n_tgt, const double* T, double r, int32_t variant, int32_t precision,
                 bool need_normals_for_plane) {
  int rc;
  if ((rc = check_cloud(src, n_src, "src_xyz")) != 0) return rc;
  if ((rc = check_cloud(tgt, n_tgt, "tgt_xyz")) != 0) return rc;
  if ((rc = check_pose(T, "T")) != 0) return rc;
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite((float)(r * r)))
    return fail(ICP_E_INVALID_ARG, "max_corr_dist must be > 0 with a finite float32 square");
  if (variant != ICP_POINT_TO_POINT && variant != ICP_POINT_TO_PLANE)
    return fail(ICP_E_INVALID_ARG, "unknown variant");
  if (precision != ICP_PREC_F32_KAHAN_F64 && precision != ICP_PREC_F64)
    return fail(ICP_E_INVALID_ARG, "unknown precision");
  if (need_normals_for_plane && variant == ICP_POINT_TO_PLANE) {
    if (!tgt_n) return fail(ICP_E_INVALID_ARG, "tgt_normals is NULL (required for point-to-plane)");
    if ((reinterpret_cast<uintptr_t>(tgt_n) & 3u) != 0)
      return fail(ICP_E_INVALID_ARG, "tgt_normals is not 4-byte aligned");
  }
  return ICP_SUCCESS;
}

// ------------------------------------------------------------------ pair preparation
struct Prepared {
  PassArgs pa;
  int64_t n_src;
};

// Grid over the target: cell edge h >= r (1 + 2^-10) so that every point
// within r of a query lies in the 27 cells around the query's cell.  The
// dense table is capped at max(2^24, 32 n_tgt) cells; a larger extent grows h
// (still exact: any h >= r works, only the candidate count changes).
// The environment variable ICP_GRID_SCALE (>= 1, debugging and tests only)
// multiplies h; results must not change with it.
double grid_scale() {
  const char* e = getenv("ICP_GRID_SCALE");
  if (!e) return 1.0;
  const double v = atof(e);
  return (v >= 1.0 && v <= 64.0) ? v : 1.0;
}

// Cells per max_corr_dist along an axis (1: 27-cell neighbourhood, 2: 125
// smaller cells).  ICP_GRID_SUB overrides the default (debugging and tests).
int grid_sub() {
  const char* e = getenv("ICP_GRID_SUB");
  if (e && atoi(e) == 1) return 1;
  if (e && atoi(e) == 2) return 2;
  return kDefaultSub;
}

GridDesc make_grid(const float* mn, const float* mx, double r, int64_t n_tgt) {
  const double cap = std::min<double>(1073741824.0, std::max<double>(16777216.0, 32.0 * (double)n_tgt));
  const int sub = grid_sub();
  double h = r * (1.0 + 1.0 / 1024.0) * grid_scale() / sub;
  GridDesc g{};
  for (int it = 0; it < 64; ++it) {
    const double inv_h = 1.0 / h;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = floor(((double)mx[a] - (double)mn[a]) * inv_h) + 1.0;
    const double cells = d[0] * d[1] * d[2];
    if (cells <= cap) {
      g.ox = mn[0]; g.oy = mn[1]; g.oz = mn[2];
      g.inv_h = inv_h;
      g.dx = (int32_t)d[0]; g.dy = (int32_t)d[1]; g.dz = (int32_t)d[2];
      g.ncell = (uint32_t)cells;
      g.sub = sub;
      return g;
    }
    h *= std::cbrt(cells / cap) * 1.001;
  }
  return g;  // unreachable for finite inputs
}

int ensure_host(icp_ctx* c, size_t bytes) {
  if (bytes <= c->host_cap) return ICP_SUCCESS;
  HIP_TRY(hipStreamSynchronize(c->stream), "sync");
  if (c->host) (void)hipHostFree(c->host);
  c->host = nullptr;
  c->host_cap = 0;
  const size_t want = std::max(bytes + bytes / 4, kHostBytes);
  HIP_TRY(hipHostMalloc(&c->host, want, hipHostMallocDefault), "hipHostMalloc");
  c->host_cap = want;
  return ICP_SUCCESS;
}

struct CloudBox {
  float tmn[3], tmx[3], smn[3], smx[3];
};

// Finiteness check and bounding boxes of n pairs: all reductions are launched,
// then read back with a single synchronisation.  `which` receives the first
// pair with a non-finite value.
int bboxes(icp_ctx* c, int n, const float* const* src, const int64_t* n_src,
           const float* const* tgt, const float* const* tgt_n, const int64_t* n_tgt, CloudBox* out,
           int* which) {
  hipStream_t s = c->stream;
  size_t blocks = 0;
  for (int p = 0; p < n; ++p) blocks += (size_t)bbox_blocks(n_tgt[p]) + (size_t)bbox_blocks(n_src[p]);
  HIP_TRY(c->bbox_part.ensure(sizeof(float) * 8 * blocks), "alloc");
  HIP_TRY(c->bbox_out.ensure(sizeof(float) * 16 * (size_t)n), "alloc");
  int rc;
  if ((rc = ensure_host(c, sizeof(float) * 16 * (size_t)n)) != 0) return rc;
  float* bp = c->bbox_part.as<float>();
  float* bo = c->bbox_out.as<float>();
  for (int p = 0; p < n; ++p) {
    const int nb_t = bbox_blocks(n_tgt[p]), nb_s = bbox_blocks(n_src[p]);
    HIP_TRY(launch_bbox(tgt[p], tgt_n[p], n_tgt[p], bp, nb_t, bo + 16 * p, s), "bbox");
    bp += 8 * nb_t;
    HIP_TRY(launch_bbox(src[p], nullptr, n_src[p], bp, nb_s, bo + 16 * p + 8, s), "bbox");
    bp += 8 * nb_s;
  }
  float* hb = static_cast<float*>(c->host);
  HIP_TRY(hipMemcpyAsync(hb, bo, sizeof(float) * 16 * (size_t)n, hipMemcpyDeviceToHost, s), "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  for (int p = 0; p < n; ++p) {
    const float* h = hb + 16 * p;
    if (h[6] != 0.0f || h[14] != 0.0f) {
      *which = p;
      return fail(ICP_E_NONFINITE, (h[6] != 0.0f ? std::string("non-finite target coordinate or normal")
                                                 : std::string("non-finite source coordinate")) +
                                       (n > 1 ? " in pair " + std::to_string(p) : std::string()));
    }
    for (int k = 0; k < 3; ++k) {
      out[p].tmn[k] = h[k];
      out[p].tmx[k] = h[3 + k];
      out[p].smn[k] = h[8 + k];
      out[p].smx[k] = h[11 + k];
    }
  }
  return ICP_SUCCESS;
}

// Transient build buffers, shared by every pair built on the context's stream
// (the stream orders their reuse).
int ensure_scratch(icp_ctx* c, int64_t n_src, int64_t n_tgt, uint64_t ncell) {
  HIP_TRY(c->t_key.ensure(4 * (size_t)n_tgt), "alloc");
  HIP_TRY(c->t_rank.ensure(4 * (size_t)n_tgt), "alloc");
  HIP_TRY(c->scan_tmp.ensure(4 * (size_t)scan_block_sums_needed((int64_t)ncell + 1)), "alloc");
  HIP_TRY(c->s_keys.ensure(4 * (size_t)n_src), "alloc");
  HIP_TRY(c->s_vals.ensure(4 * (size_t)n_src), "alloc");
  HIP_TRY(c->s_keys2.ensure(4 * (size_t)n_src), "alloc");
  HIP_TRY(c->s_vals2.ensure(4 * (size_t)n_src), "alloc");
  HIP_TRY(c->s_hist.ensure(4 * (size_t)radix_hist_needed(n_src)), "alloc");
  return ICP_SUCCESS;
}

struct PairDst {
  uint32_t* cs;
  float4* tp;
  float4* tn;  // may be null (point-to-point)
  float* sx;
  float* sy;
  float* sz;
};

// Builds the target grid (cell table + cell-ordered target) and the
// Morton-ordered source of one pair into `d`.  *perm_out (transient, valid
// until the next build) maps ordered source positions to original indices.
int build_pair(icp_ctx* c, const float* src, int64_t n_src, const float* tgt, const float* tgt_n,
               int64_t n_tgt, const GridDesc& g, const CloudBox& b, const PairDst& d,
               uint32_t** perm_out) {
  hipStream_t s = c->stream;
  const int64_t scan_cap = scan_block_sums_needed((int64_t)g.ncell + 1);
  HIP_TRY(launch_target_grid(tgt, d.tn ? tgt_n : nullptr, n_tgt, g, c->t_key.as<uint32_t>(),
                             c->t_rank.as<uint32_t>(), d.cs, d.tp, d.tn, c->scan_tmp.as<uint32_t>(),
                             scan_cap, s),
          "target grid");
  // Morton curve over 1024^3 cells spanning the source box.  It depends on the
  // source cloud only, so the summation order (and every result bit) does not
  // change with the grid's cell size.
  double ext = 0.0;
  for (int a = 0; a < 3; ++a) ext = std::max(ext, (double)b.smx[a] - (double)b.smn[a]);
  const double hs = ext > 0.0 ? ext / 1023.5 : 1.0;
  HIP_TRY(launch_source_order(src, n_src, b.smn[0], b.smn[1], b.smn[2], 1.0 / hs,
                              c->s_keys.as<uint32_t>(), c->s_vals.as<uint32_t>(),
                              c->s_keys2.as<uint32_t>(), c->s_vals2.as<uint32_t>(),
                              c->s_hist.as<uint32_t>(), radix_hist_needed(n_src), d.sx, d.sy, d.sz,
                              perm_out, s),
          "source order");
  return ICP_SUCCESS;
}

void fill_pass_args(PassArgs& a, const PairDst& d, const uint32_t* perm, int64_t n_src,
                    int64_t n_tgt, const GridDesc& g, double r, IterState* st, double* part,
                    uint32_t* jprev) {
  memset(&a, 0, sizeof a);
  a.sx = d.sx;
  a.sy = d.sy;
  a.sz = d.sz;
  a.sperm = perm;
  a.n_src = (int32_t)n_src;
  a.tp = d.tp;
  a.tn = d.tn;
  a.cs = d.cs;
  a.g = g;
  a.r2f = (float)(r * r);
  a.inv_h2 = (float)(g.inv_h * g.inv_h);
  a.n_tgt = (int32_t)n_tgt;
  a.jprev = jprev;
  a.st = st;
  a.part = part;
  a.n_blocks = (int32_t)((n_src + kTile - 1) / kTile);
}

int prepare(icp_ctx* c, const float* src, int64_t n_src, const float* tgt, const float* tgt_n,
            int64_t n_tgt, double r, bool with_normals, Prepared* P) {
  CloudBox b;
  int which = -1, rc;
  const float* tn = with_normals ? tgt_n : nullptr;
  if ((rc = bboxes(c, 1, &src, &n_src, &tgt, &tn, &n_tgt, &b, &which)) != 0) return rc;
  const GridDesc g = make_grid(b.tmn, b.tmx, r, n_tgt);
  if ((rc = ensure_scratch(c, n_src, n_tgt, g.ncell)) != 0) return rc;
  HIP_TRY(c->t_cs.ensure(4 * ((size_t)g.ncell + 1)), "alloc");
  HIP_TRY(c->t_tp.ensure(16 * (size_t)n_tgt), "alloc");
  if (with_normals) HIP_TRY(c->t_tn.ensure(16 * (size_t)n_tgt), "alloc");
  HIP_TRY(c->s_x.ensure(4 * (size_t)n_src), "alloc");
  HIP_TRY(c->s_y.ensure(4 * (size_t)n_src), "alloc");
  HIP_TRY(c->s_z.ensure(4 * (size_t)n_src), "alloc");
  const PairDst d{c->t_cs.as<uint32_t>(), c->t_tp.as<float4>(),
                  with_normals ? c->t_tn.as<float4>() : nullptr, c->s_x.as<float>(),
                  c->s_y.as<float>(), c->s_z.as<float>()};
  uint32_t* perm = nullptr;
  if ((rc = build_pair(c, src, n_src, tgt, tgt_n, n_tgt, g, b, d, &perm)) != 0) return rc;
  const int32_t n_blocks = (int32_t)((n_src + kTile - 1) / kTile);
  HIP_TRY(c->part.ensure(sizeof(double) * kNumSums * (size_t)n_blocks), "alloc");
  HIP_TRY(c->state.ensure(sizeof(IterState)), "alloc");
  fill_pass_args(P->pa, d, perm, n_src, n_tgt, g, r, c->state.as<IterState>(), c->part.as<double>(),
                 nullptr);
  P->n_src = n_src;
  return ICP_SUCCESS;
}

int read_state(icp_ctx* c, IterState* out) {
  HIP_TRY(hipMemcpyAsync(c->host, c->state.p, sizeof(IterState), hipMemcpyDeviceToHost, c->stream),
          "readback");
  HIP_TRY(hipStreamSynchronize(c->stream), "sync");
  memcpy(out, c->host, sizeof(IterState));
  return ICP_SUCCESS;
}

// Event slots: [0] call start, [1] call end, [2 + 2k] / [3 + 2k] around pass k.
int ensure_events(icp_ctx* c, int passes) {
  const size_t need = 2 + 2 * (size_t)passes;
  while (c->ev.size() < need) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    c->ev.push_back(e);
  }
  return ICP_SUCCESS;
}

int collect_profile(icp_ctx* c, int counted_passes, int64_t n_src) {
  float ms = 0.0f;
  for (int k = 0; k < counted_passes; ++k) {
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[2 + 2 * k], c->ev[3 + 2 * k]), "hipEventElapsedTime");
    c->prof.pass_ms += ms;
    c->prof.pass_launches += 1;
    c->prof.pass_points += n_src;
  }
  HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]), "hipEventElapsedTime");
  c->prof.call_ms += ms;
  c->prof.calls += 1;
  return ICP_SUCCESS;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* icp_version(void) { return "icp-mi355x 0.1 (gfx950)"; }

const char* icp_strerror(int code) {
  switch (code) {
    case ICP_SUCCESS: return "success";
    case ICP_E_INVALID_ARG: return "invalid argument";
    case ICP_E_NONFINITE: return "non-finite input";
    case ICP_E_TOO_LARGE: return "input too large";
    case ICP_E_OOM: return "out of device memory";
    case ICP_E_DEVICE: return "device (HIP) error";
    case ICP_E_CANCELLED: return "cancelled";
    case ICP_E_NOT_FOUND: return "not found";
    default: return "unknown error code";
  }
}

const char* icp_last_error(void) { return g_last_error.c_str(); }

int icp_ctx_create(int device, void* hip_stream, icp_ctx_t** out) {
  if (!out) return fail(ICP_E_INVALID_ARG, "out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(ICP_E_INVALID_ARG, "device index out of range");
  icp_ctx* c = new icp_ctx();
  const int rc = ctx_init(c, device, hip_stream);
  if (rc != ICP_SUCCESS) {
    ctx_free(c);
    delete c;
    return rc;
  }
  *out = c;
  return ICP_SUCCESS;
}

int icp_ctx_set_profiling(icp_ctx_t* ctx, int enable) {
  if (!ctx) return fail(ICP_E_INVALID_ARG, "ctx is NULL");
  ctx->profiling = enable != 0;
  ctx->prof = icp_profile_t{};
  return ICP_SUCCESS;
}

int icp_ctx_get_profile(icp_ctx_t* ctx, icp_profile_t* out) {
  if (!ctx || !out) return fail(ICP_E_INVALID_ARG, "ctx or out is NULL");
  *out = ctx->prof;
  return ICP_SUCCESS;
}

int icp_ctx_destroy(icp_ctx_t* ctx) {
  if (!ctx) return ICP_SUCCESS;
  ctx_free(ctx);
  delete ctx;
  return ICP_SUCCESS;
}

int icp_register(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const float* tgt_xyz,
                 const float* tgt_normals, int64_t n_tgt, const double T_init[16],
                 double max_corr_dist, int32_t max_iter, double rel_tol, int32_t variant,
                 int32_t precision, icp_result_t* out) {
  int rc = check_common(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T_init, max_corr_dist, variant,
                        precision, true);
  if (rc) return rc;
  if (max_iter < 0) return fail(ICP_E_INVALID_ARG, "max_iter must be >= 0");
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol))
    return fail(ICP_E_INVALID_ARG, "rel_tol must be finite and >= 0");
  if (!out) return fail(ICP_E_INVALID_ARG, "out is NULL");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  Prepared P;
  if ((rc = prepare(c, src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, max_corr_dist, plane, &P)) != 0)
    return rc;
  HIP_TRY(c->jprev.ensure(4 * (size_t)n_src), "alloc");
  HIP_TRY(hipMemsetAsync(c->jprev.p, 0xff, 4 * (size_t)n_src, c->stream), "memset");
  P.pa.jprev = c->jprev.as<uint32_t>();
  const bool prof = c->profiling;
  if (prof && (rc = ensure_events(c, max_iter + 1)) != 0) return rc;
  if (prof) HIP_TRY(hipEventRecord(c->ev[0], c->stream), "hipEventRecord");
  HIP_TRY(launch_state_init(c->state.as<IterState>(), T_init, c->stream), "state init");
  SolveArgs sa{P.pa.part, P.pa.n_blocks, c->state.as<IterState>(), n_src, max_iter, rel_tol, 0};
  for (int32_t k = 0; k <= max_iter; ++k) {
    if (prof) HIP_TRY(hipEventRecord(c->ev[2 + 2 * k], c->stream), "hipEventRecord");
    HIP_TRY(launch_pass(P.pa, variant, precision, false, c->stream), "pass");
    if (prof) HIP_TRY(hipEventRecord(c->ev[3 + 2 * k], c->stream), "hipEventRecord");
    HIP_TRY(launch_solve(sa, c->stream), "solve");
  }
  if (prof) HIP_TRY(hipEventRecord(c->ev[1], c->stream), "hipEventRecord");
  IterState st;
  if ((rc = read_state(c, &st)) != 0) return rc;
  if (prof && (rc = collect_profile(c, st.k + 1, n_src)) != 0) return rc;
  for (int k = 0; k < 12; ++k) out->T[k] = st.T[k];
  out->T[12] = 0.0; out->T[13] = 0.0; out->T[14] = 0.0; out->T[15] = 1.0;
  out->fitness = st.fitness;
  out->inlier_rmse = st.rmse;
  out->n_inliers = st.n_in;
  out->n_iter = st.k;
  out->status = st.status;
  return ICP_SUCCESS;
}

int icp_register_batch(icp_ctx_t* ctx, const icp_pair_t* pairs, int32_t n_pairs, int32_t variant,
                       int32_t precision, icp_result_t* out) {
  if (!pairs || !out) return fail(ICP_E_INVALID_ARG, "pairs / out is NULL");
  if (n_pairs < 1) return fail(ICP_E_INVALID_ARG, "n_pairs must be >= 1");
  int rc;
  int64_t total_src = 0, total_tgt = 0;
  int32_t iters = 0;
  for (int p = 0; p < n_pairs; ++p) {
    const icp_pair_t& q = pairs[p];
    if ((rc = check_common(q.src_xyz, q.n_src, q.tgt_xyz, q.tgt_normals, q.n_tgt, q.T_init,
                           q.max_corr_dist, variant, precision, true)) != 0 ||
        (q.max_iter < 0 && (rc = fail(ICP_E_INVALID_ARG, "max_iter must be >= 0")) != 0) ||
        ((!(q.rel_tol >= 0.0) || !std::isfinite(q.rel_tol)) &&
         (rc = fail(ICP_E_INVALID_ARG, "rel_tol must be finite and >= 0")) != 0) ||
        (q.reserved != 0 && (rc = fail(ICP_E_INVALID_ARG, "reserved must be 0")) != 0)) {
      g_last_error += " (pair " + std::to_string(p) + ")";
      return rc;
    }
    total_src += q.n_src;
    total_tgt += q.n_tgt;
    iters = std::max(iters, q.max_iter);
  }
  if (total_src > (int64_t)INT32_MAX || total_tgt > (int64_t)INT32_MAX)
    return fail(ICP_E_TOO_LARGE, "more than 2^31-1 points in one batch");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  const int n = n_pairs;

  std::vector<const float*> srcs(n), tgts(n), tns(n);
  std::vector<int64_t> ns(n), nt(n);
  for (int p = 0; p < n; ++p) {
    srcs[p] = pairs[p].src_xyz;
    tgts[p] = pairs[p].tgt_xyz;
    tns[p] = plane ? pairs[p].tgt_normals : nullptr;
    ns[p] = pairs[p].n_src;
    nt[p] = pairs[p].n_tgt;
  }
  std::vector<CloudBox> box(n);
  int which = -1;
  if ((rc = bboxes(c, n, srcs.data(), ns.data(), tgts.data(), tns.data(), nt.data(), box.data(),
                   &which)) != 0)
    return rc;

  // layout of the batch region: header (pass args, solve args, states, work
  // items) first, then every pair's persistent arrays
  std::vector<GridDesc> grid(n);
  int64_t n_items = 0, max_src = 0, max_tgt = 0;
  uint64_t max_cell = 0;
  for (int p = 0; p < n; ++p) {
    grid[p] = make_grid(box[p].tmn, box[p].tmx, pairs[p].max_corr_dist, nt[p]);
    n_items += (ns[p] + kTile - 1) / kTile;
    max_src = std::max(max_src, ns[p]);
    max_tgt = std::max(max_tgt, nt[p]);
    max_cell = std::max<uint64_t>(max_cell, grid[p].ncell);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = (off + 255) & ~(size_t)255;
    off = o + bytes;
    return o;
  };
  const size_t o_pargs = take(sizeof(PassArgs) * n);
  const size_t o_sargs = take(sizeof(SolveArgs) * n);
  const size_t o_states = take(sizeof(IterState) * n);
  const size_t o_items = take(sizeof(uint2) * (size_t)n_items);
  const size_t header = off;
  const size_t o_jprev = take(4 * (size_t)total_src);
  struct Offs { size_t cs, tp, tn, sx, sy, sz, part; };
  std::vector<Offs> po(n);
  for (int p = 0; p < n; ++p) {
    po[p].cs = take(4 * ((size_t)grid[p].ncell + 1));
    po[p].tp = take(16 * (size_t)nt[p]);
    po[p].tn = plane ? take(16 * (size_t)nt[p]) : 0;
    po[p].sx = take(4 * (size_t)ns[p]);
    po[p].sy = take(4 * (size_t)ns[p]);
    po[p].sz = take(4 * (size_t)ns[p]);
    po[p].part = take(sizeof(double) * kNumSums * (size_t)((ns[p] + kTile - 1) / kTile));
  }
  HIP_TRY(c->batch.ensure(off), "alloc");
  if ((rc = ensure_scratch(c, max_src, max_tgt, max_cell)) != 0) return rc;
  if ((rc = ensure_host(c, std::max(header, sizeof(IterState) * n))) != 0) return rc;
  char* base = c->batch.as<char>();

  char* hh = static_cast<char*>(c->host);
  PassArgs* hp = reinterpret_cast<PassArgs*>(hh + o_pargs);
  SolveArgs* hs = reinterpret_cast<SolveArgs*>(hh + o_sargs);
  IterState* hst = reinterpret_cast<IterState*>(hh + o_states);
  uint2* hit = reinterpret_cast<uint2*>(hh + o_items);
  IterState* dst_states = reinterpret_cast<IterState*>(base + o_states);
  uint32_t* jprev = reinterpret_cast<uint32_t*>(base + o_jprev);
  int64_t item = 0, src_off = 0;
  for (int p = 0; p < n; ++p) {
    const PairDst d{reinterpret_cast<uint32_t*>(base + po[p].cs), reinterpret_cast<float4*>(base + po[p].tp),
                    plane ? reinterpret_cast<float4*>(base + po[p].tn) : nullptr,
                    reinterpret_cast<float*>(base + po[p].sx), reinterpret_cast<float*>(base + po[p].sy),
                    reinterpret_cast<float*>(base + po[p].sz)};
    uint32_t* perm = nullptr;
    if ((rc = build_pair(c, srcs[p], ns[p], tgts[p], pairs[p].tgt_normals, nt[p], grid[p], box[p], d,
                         &perm)) != 0)
      return rc;
    double* part = reinterpret_cast<double*>(base + po[p].part);
    fill_pass_args(hp[p], d, nullptr, ns[p], nt[p], grid[p], pairs[p].max_corr_dist, dst_states + p,
                   part, jprev + src_off);
    hs[p] = SolveArgs{part, hp[p].n_blocks, dst_states + p, ns[p], pairs[p].max_iter,
                      pairs[p].rel_tol, 0};
    IterState& st = hst[p];
    memset(&st, 0, sizeof st);
    for (int k = 0; k < 16; ++k) st.T[k] = pairs[p].T_init[k];
    for (int t = 0; t < hp[p].n_blocks; ++t) hit[item++] = make_uint2((uint32_t)p, (uint32_t)t);
    src_off += ns[p];
  }
  HIP_TRY(hipMemsetAsync(jprev, 0xff, 4 * (size_t)total_src, c->stream), "memset");
  HIP_TRY(hipMemcpyAsync(base, hh, header, hipMemcpyHostToDevice, c->stream), "upload");
  const PassArgs* dp = reinterpret_cast<const PassArgs*>(base + o_pargs);
  const SolveArgs* ds = reinterpret_cast<const SolveArgs*>(base + o_sargs);
  const uint2* di = reinterpret_cast<const uint2*>(base + o_items);
  const int sub = grid[0].sub;
  const bool prof = c->profiling;
  if (prof && (rc = ensure_events(c, iters + 1)) != 0) return rc;
  if (prof) HIP_TRY(hipEventRecord(c->ev[0], c->stream), "hipEventRecord");
  for (int32_t k = 0; k <= iters; ++k) {
    if (prof) HIP_TRY(hipEventRecord(c->ev[2 + 2 * k], c->stream), "hipEventRecord");
    HIP_TRY(launch_batch_pass(dp, di, (int)n_items, sub, variant, precision, c->stream), "pass");
    if (prof) HIP_TRY(hipEventRecord(c->ev[3 + 2 * k], c->stream), "hipEventRecord");
    HIP_TRY(launch_batch_solve(ds, n, c->stream), "solve");
  }
  if (prof) HIP_TRY(hipEventRecord(c->ev[1], c->stream), "hipEventRecord");
  HIP_TRY(hipMemcpyAsync(hh, dst_states, sizeof(IterState) * n, hipMemcpyDeviceToHost, c->stream),
          "readback");
  HIP_TRY(hipStreamSynchronize(c->stream), "sync");
  const IterState* res = reinterpret_cast<const IterState*>(hh);
  int32_t max_k = 0;
  int64_t evals = 0;
  for (int p = 0; p < n; ++p) {
    const IterState& st = res[p];
    for (int k = 0; k < 12; ++k) out[p].T[k] = st.T[k];
    out[p].T[12] = 0.0; out[p].T[13] = 0.0; out[p].T[14] = 0.0; out[p].T[15] = 1.0;
    out[p].fitness = st.fitness;
    out[p].inlier_rmse = st.rmse;
    out[p].n_inliers = st.n_in;
    out[p].n_iter = st.k;
    out[p].status = st.status;
    max_k = std::max(max_k, st.k);
    evals += (int64_t)(st.k + 1) * ns[p];
  }
  if (prof) {
    if ((rc = collect_profile(c, max_k + 1, 0)) != 0) return rc;
    c->prof.pass_points += evals;
  }
  return ICP_SUCCESS;
}

int icp_correspondences(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const double T[16],
                        const float* tgt_xyz, int64_t n_tgt, double max_corr_dist, int32_t* idx_out,
                        float* d2_out) {
  int rc = check_common(src_xyz, n_src, tgt_xyz, nullptr, n_tgt, T, max_corr_dist,
                        ICP_POINT_TO_POINT, ICP_PREC_F32_KAHAN_F64, false);
  if (rc) return rc;
  if (!idx_out || !d2_out) return fail(ICP_E_INVALID_ARG, "idx_out / d2_out is NULL");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  Prepared P;
  if ((rc = prepare(c, src_xyz, n_src, tgt_xyz, nullptr, n_tgt, max_corr_dist, false, &P)) != 0)
    return rc;
  P.pa.idx_out = idx_out;
  P.pa.d2_out = d2_out;
  HIP_TRY(launch_state_init(c->state.as<IterState>(), T, c->stream), "state init");
  HIP_TRY(launch_pass(P.pa, ICP_POINT_TO_POINT, ICP_PREC_F32_KAHAN_F64, true, c->stream), "pass");
  HIP_TRY(hipStreamSynchronize(c->stream), "sync");
  return ICP_SUCCESS;
}

int icp_normal_equations(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const double T[16],
                         const float* tgt_xyz, const float* tgt_normals, int64_t n_tgt,
                         double max_corr_dist, int32_t variant, int32_t precision, double AtA21[21],
                         double Atb6[6], double* sum_d2, int64_t* n_in) {
  int rc = check_common(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T, max_corr_dist, variant,
                        precision, true);
  if (rc) return rc;
  if (!AtA21 || !Atb6 || !sum_d2 || !n_in) return fail(ICP_E_INVALID_ARG, "output pointer is NULL");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  Prepared P;
  if ((rc = prepare(c, src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, max_corr_dist, plane, &P)) != 0)
    return rc;
  HIP_TRY(launch_state_init(c->state.as<IterState>(), T, c->stream), "state init");
  HIP_TRY(launch_pass(P.pa, variant, precision, false, c->stream), "pass");
  SolveArgs sa{P.pa.part, P.pa.n_blocks, c->state.as<IterState>(), n_src, 0, 0.0, 1};
  HIP_TRY(launch_solve(sa, c->stream), "reduce");
  IterState st;
  if ((rc = read_state(c, &st)) != 0) return rc;
  for (int k = 0; k < 21; ++k) AtA21[k] = st.sums[k];
  for (int k = 0; k < 6; ++k) Atb6[k] = st.sums[21 + k];
  *sum_d2 = st.sums[kSumD2];
  *n_in = (int64_t)st.sums[kSumCount];
  return ICP_SUCCESS;
}

}  // extern "C"
