// Host runtime of libicp.so: argument validation, contexts and their device
// workspace, grid sizing and the per-iteration launch sequence behind the C
// ABI declared in include/icp.h.
//
// Every registration call, plain or batched, is:
//   1. finiteness + bounding boxes of all clouds (one segmented reduction and
//      one small readback that sizes the grids);
//   2. segmented build of every pair's target grid and Morton-ordered source
//      (a fixed number of launches, independent of the number of pairs);
//   3. max_iter + 1 passes of two launches each: the fused correspondence /
//      normal-equation kernel over all source tiles, then the kernel that
//      reduces the tile partials in fixed order, solves the 6x6 system and
//      updates the pose on the device.  Loop state never leaves the device;
//      launches after a pair's stopping rule fired return immediately;
//   4. one readback of the final states.

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
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

#define HIP_TRY(expr, what)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, what);   \
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
    if (p) (void)hipFree(p);
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

}  // namespace

struct icp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // per-call descriptors, loop header, warm-start matches, partials, states
  Buf desc;
  // preparation scratch
  Buf bbox_part, t_key, t_rank, scan_tmp, s_hist;
  Buf sk[6];  // sort buffers: klo[2], khi[2], val[2]
  // prepared pairs (concatenated)
  Buf cs, tp, tn, sx, sy, sz, perm;
  void* host = nullptr;  // pinned staging
  size_t host_cap = 0;
  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev;  // [0] call start, [1] call end, [2+2k]/[3+2k] around pass k
  icp_profile_t prof{};
};

namespace {

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
  Buf* bufs[] = {&c->desc, &c->bbox_part, &c->t_key, &c->t_rank, &c->scan_tmp, &c->s_hist,
                 &c->cs, &c->tp, &c->tn, &c->sx, &c->sy, &c->sz, &c->perm};
  for (Buf* b : bufs) b->release();
  for (Buf& b : c->sk) b.release();
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

// ------------------------------------------------------------------ validation
int check_cloud(const float* p, int64_t n, const char* name) {
  if (!p) return fail(ICP_E_INVALID_ARG, std::string(name) + " is NULL");
  if (n < 1) return fail(ICP_E_INVALID_ARG, std::string(name) + ": point count must be >= 1");
  if (n > (int64_t)INT32_MAX)
    return fail(ICP_E_TOO_LARGE, std::string(name) + ": more than 2^31-1 points");
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

int check_iteration(int32_t max_iter, double rel_tol) {
  if (max_iter < 0) return fail(ICP_E_INVALID_ARG, "max_iter must be >= 0");
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol))
    return fail(ICP_E_INVALID_ARG, "rel_tol must be finite and >= 0");
  return ICP_SUCCESS;
}

// ------------------------------------------------------------------ grids
// The environment variable ICP_GRID_SCALE (>= 1, debugging and tests only)
// multiplies the cell edge; results must not change with it.
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

// Grid over a target box: cell edge h >= r (1 + 2^-10) / sub so that every
// point within r of a query lies in the (2 sub + 1)^3 cells around the query's
// cell.  The dense table is capped at max(2^24, 32 n_tgt) cells; a larger
// extent grows h (still exact: any h above the bound works, only the candidate
// count changes).
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

// ------------------------------------------------------------------ call layout
struct PairIn {
  const float* src;
  int64_t n_src;
  const float* tgt;
  const float* tgt_n;  // null: point-to-point (normals neither checked nor gathered)
  int64_t n_tgt;
  double r;
};

// Byte offsets of one call's descriptors; the same layout is used in pinned
// host staging and in the context's `desc` device buffer.
struct Layout {
  size_t clouds, blk_bbox, pairs, blk_t, blk_s, src_off;  // preparation
  size_t pargs, sargs, states, items;                       // loop header
  size_t header_end;                                        // end of uploaded part
  size_t bbox_out, jprev, part;                             // device only
  size_t total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(int n, int64_t n_items, int64_t total_src, int64_t total_tiles) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align256(off);
    off = o + bytes;
    return o;
  };
  L.clouds = take(sizeof(SegCloud) * 2 * n);
  L.blk_bbox = take(sizeof(int64_t) * (2 * n + 1));
  L.pairs = take(sizeof(BuildPair) * n);
  L.blk_t = take(sizeof(int64_t) * (n + 1));
  L.blk_s = take(sizeof(int64_t) * (n + 1));
  L.src_off = take(sizeof(int64_t) * (n + 1));
  L.pargs = take(sizeof(PassArgs) * n);
  L.sargs = take(sizeof(SolveArgs) * n);
  L.states = take(sizeof(IterState) * n);
  L.items = take(sizeof(uint2) * (size_t)std::max<int64_t>(n_items, 1));
  L.header_end = align256(off);
  L.bbox_out = take(sizeof(float) * 16 * n);
  L.jprev = take(sizeof(uint32_t) * (size_t)total_src);
  L.part = take(sizeof(double) * kNumSums * (size_t)total_tiles);
  L.total = align256(off);
  return L;
}

struct Prep {
  int n = 0;
  Layout L;
  std::vector<GridDesc> g;
  std::vector<int64_t> src_off, tgt_off, tile_off;
  std::vector<uint64_t> tab_off;
  int64_t total_src = 0, total_tgt = 0, total_tiles = 0;
  uint64_t total_tab = 0;
  int sub = 1;
};

int64_t tiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

// Steps 1 and 2 of a call for n pairs: checks, boxes, grids and the
// segmented build into the context's concatenated arrays.
int prepare_pairs(icp_ctx* c, int n, const PairIn* in, Prep* P) {
  hipStream_t s = c->stream;
  P->n = n;
  P->src_off.assign(n + 1, 0);
  P->tgt_off.assign(n + 1, 0);
  P->tile_off.assign(n + 1, 0);
  for (int p = 0; p < n; ++p) {
    P->src_off[p + 1] = P->src_off[p] + in[p].n_src;
    P->tgt_off[p + 1] = P->tgt_off[p] + in[p].n_tgt;
    P->tile_off[p + 1] = P->tile_off[p] + tiles_of(in[p].n_src);
  }
  P->total_src = P->src_off[n];
  P->total_tgt = P->tgt_off[n];
  P->total_tiles = P->tile_off[n];
  if (P->total_src > (int64_t)INT32_MAX || P->total_tgt > (int64_t)INT32_MAX)
    return fail(ICP_E_TOO_LARGE, "more than 2^31-1 points in one call");
  P->L = make_layout(n, P->total_tiles, P->total_src, P->total_tiles);
  const Layout& L = P->L;
  int rc;
  if ((rc = ensure_host(c, L.total)) != 0) return rc;
  HIP_TRY(c->desc.ensure(L.total), "alloc");
  char* hh = static_cast<char*>(c->host);
  char* dd = c->desc.as<char>();

  // 1. boxes and finiteness of all clouds (target with its normals, source)
  SegCloud* cl = reinterpret_cast<SegCloud*>(hh + L.clouds);
  int64_t* bo = reinterpret_cast<int64_t*>(hh + L.blk_bbox);
  bo[0] = 0;
  for (int p = 0; p < n; ++p) {
    cl[2 * p] = SegCloud{in[p].tgt, in[p].tgt_n, in[p].n_tgt};
    cl[2 * p + 1] = SegCloud{in[p].src, nullptr, in[p].n_src};
    bo[2 * p + 1] = bo[2 * p] + bbox_blocks(in[p].n_tgt);
    bo[2 * p + 2] = bo[2 * p + 1] + bbox_blocks(in[p].n_src);
  }
  const int64_t bbox_total = bo[2 * n];
  HIP_TRY(c->bbox_part.ensure(sizeof(float) * 8 * (size_t)bbox_total), "alloc");
  HIP_TRY(hipMemcpyAsync(dd, hh, L.pairs, hipMemcpyHostToDevice, s), "upload");
  float* dbox = reinterpret_cast<float*>(dd + L.bbox_out);
  HIP_TRY(launch_seg_bbox(reinterpret_cast<SegCloud*>(dd + L.clouds), 2 * n,
                          reinterpret_cast<int64_t*>(dd + L.blk_bbox), bbox_total,
                          c->bbox_part.as<float>(), dbox, s),
          "bbox");
  float* hbox = reinterpret_cast<float*>(hh + L.bbox_out);
  HIP_TRY(hipMemcpyAsync(hbox, dbox, sizeof(float) * 16 * n, hipMemcpyDeviceToHost, s), "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  for (int p = 0; p < n; ++p) {
    const float* t = hbox + 16 * p;
    const float* q = t + 8;
    if (t[6] != 0.0f || q[6] != 0.0f)
      return fail(ICP_E_NONFINITE, (t[6] != 0.0f ? std::string("non-finite target coordinate or normal")
                                                 : std::string("non-finite source coordinate")) +
                                       (n > 1 ? " in pair " + std::to_string(p) : std::string()));
  }

  // 2. grids, offsets and the segmented build
  P->g.resize(n);
  P->tab_off.assign(n + 1, 0);
  BuildPair* bp = reinterpret_cast<BuildPair*>(hh + L.pairs);
  int64_t* bt = reinterpret_cast<int64_t*>(hh + L.blk_t);
  int64_t* bs = reinterpret_cast<int64_t*>(hh + L.blk_s);
  int64_t* so = reinterpret_cast<int64_t*>(hh + L.src_off);
  bt[0] = 0;
  bs[0] = 0;
  for (int p = 0; p < n; ++p) {
    const float* t = hbox + 16 * p;
    const float* q = t + 8;
    P->g[p] = make_grid(t, t + 3, in[p].r, in[p].n_tgt);
    P->tab_off[p + 1] = P->tab_off[p] + (uint64_t)P->g[p].ncell + 1;
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, (double)q[3 + a] - (double)q[a]);
    // Morton grid of the source: 1024 cells per axis over the source's own box,
    // so the order (and the summation order) depends on the source only
    const double hs = ext > 0.0 ? ext / 1023.5 : 1.0;
    bp[p] = BuildPair{in[p].src, in[p].tgt, in[p].tgt_n, in[p].n_src, in[p].n_tgt,
                      P->src_off[p], P->tgt_off[p], P->tab_off[p], P->g[p],
                      (double)q[0], (double)q[1], (double)q[2], 1.0 / hs};
    bt[p + 1] = bt[p] + (in[p].n_tgt + 255) / 256;
    bs[p + 1] = bs[p] + (in[p].n_src + 255) / 256;
    so[p] = P->src_off[p];
  }
  so[n] = P->src_off[n];
  P->total_tab = P->tab_off[n];
  if (P->total_tab >= (uint64_t)UINT32_MAX)
    return fail(ICP_E_TOO_LARGE, "grid tables of one call exceed 2^32 cells");
  P->sub = P->g[0].sub;
  const bool normals = in[0].tgt_n != nullptr;
  const int64_t scan_cap = scan_block_sums_needed((int64_t)P->total_tab);
  const int64_t hist_cap = radix_hist_needed(P->total_src);
  HIP_TRY(c->cs.ensure(4 * (size_t)P->total_tab), "alloc");
  HIP_TRY(c->tp.ensure(16 * (size_t)P->total_tgt), "alloc");
  if (normals) HIP_TRY(c->tn.ensure(16 * (size_t)P->total_tgt), "alloc");
  HIP_TRY(c->sx.ensure(4 * (size_t)P->total_src), "alloc");
  HIP_TRY(c->sy.ensure(4 * (size_t)P->total_src), "alloc");
  HIP_TRY(c->sz.ensure(4 * (size_t)P->total_src), "alloc");
  HIP_TRY(c->perm.ensure(4 * (size_t)P->total_src), "alloc");
  HIP_TRY(c->t_key.ensure(4 * (size_t)P->total_tgt), "alloc");
  HIP_TRY(c->t_rank.ensure(4 * (size_t)P->total_tgt), "alloc");
  HIP_TRY(c->scan_tmp.ensure(4 * (size_t)scan_cap), "alloc");
  HIP_TRY(c->s_hist.ensure(4 * (size_t)hist_cap), "alloc");
  for (Buf& b : c->sk) HIP_TRY(b.ensure(4 * (size_t)P->total_src), "alloc");
  HIP_TRY(hipMemcpyAsync(dd + L.pairs, hh + L.pairs, L.pargs - L.pairs, hipMemcpyHostToDevice, s),
          "upload");
  const BuildPair* dbp = reinterpret_cast<const BuildPair*>(dd + L.pairs);
  HIP_TRY(launch_seg_targets(dbp, n, reinterpret_cast<const int64_t*>(dd + L.blk_t), bt[n],
                             P->total_tab, c->cs.as<uint32_t>(), c->t_key.as<uint32_t>(),
                             c->t_rank.as<uint32_t>(), c->scan_tmp.as<uint32_t>(), scan_cap,
                             c->tp.as<float4>(), normals ? c->tn.as<float4>() : nullptr, s),
          "target grid");
  SortBufs sb;
  for (int k = 0; k < 2; ++k) {
    sb.klo[k] = c->sk[k].as<uint32_t>();
    sb.khi[k] = c->sk[2 + k].as<uint32_t>();
    sb.val[k] = c->sk[4 + k].as<uint32_t>();
  }
  HIP_TRY(launch_seg_sources(dbp, n, reinterpret_cast<const int64_t*>(dd + L.blk_s), bs[n],
                             reinterpret_cast<const int64_t*>(dd + L.src_off), P->total_src, sb,
                             c->s_hist.as<uint32_t>(), hist_cap, c->sx.as<float>(),
                             c->sy.as<float>(), c->sz.as<float>(), c->perm.as<uint32_t>(), s),
          "source order");
  return ICP_SUCCESS;
}

// Pass arguments of pair p of a prepared call (pointers into the device
// buffers; `st`, `part`, `jprev` inside the call's desc region).
PassArgs pass_args(icp_ctx* c, const Prep& P, int p, double r, bool with_jprev, bool normals) {
  const Layout& L = P.L;
  char* dd = c->desc.as<char>();
  PassArgs a;
  memset(&a, 0, sizeof a);
  a.sx = c->sx.as<float>() + P.src_off[p];
  a.sy = c->sy.as<float>() + P.src_off[p];
  a.sz = c->sz.as<float>() + P.src_off[p];
  a.sperm = c->perm.as<uint32_t>() + P.src_off[p];
  a.n_src = (int32_t)(P.src_off[p + 1] - P.src_off[p]);
  a.tp = c->tp.as<float4>();
  a.tn = normals ? c->tn.as<float4>() : nullptr;
  a.cs = c->cs.as<uint32_t>() + P.tab_off[p];
  a.g = P.g[p];
  a.r2f = (float)(r * r);
  a.inv_h2 = (float)(P.g[p].inv_h * P.g[p].inv_h);
  a.n_tgt = (int32_t)(P.tgt_off[p + 1] - P.tgt_off[p]);
  a.jprev = with_jprev ? reinterpret_cast<uint32_t*>(dd + L.jprev) + P.src_off[p] : nullptr;
  a.st = reinterpret_cast<IterState*>(dd + L.states) + p;
  a.part = reinterpret_cast<double*>(dd + L.part) + (size_t)kNumSums * P.tile_off[p];
  a.n_blocks = (int32_t)(P.tile_off[p + 1] - P.tile_off[p]);
  return a;
}

int ensure_events(icp_ctx* c, int passes) {
  const size_t need = 2 + 2 * (size_t)passes;
  while (c->ev.size() < need) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    c->ev.push_back(e);
  }
  return ICP_SUCCESS;
}

int collect_profile(icp_ctx* c, int counted_passes, int64_t evals) {
  float ms = 0.0f;
  for (int k = 0; k < counted_passes; ++k) {
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[2 + 2 * k], c->ev[3 + 2 * k]), "hipEventElapsedTime");
    c->prof.pass_ms += ms;
    c->prof.pass_launches += 1;
  }
  c->prof.pass_points += evals;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]), "hipEventElapsedTime");
  c->prof.call_ms += ms;
  c->prof.calls += 1;
  return ICP_SUCCESS;
}

void to_result(const IterState& st, icp_result_t* out) {
  for (int k = 0; k < 12; ++k) out->T[k] = st.T[k];
  out->T[12] = 0.0; out->T[13] = 0.0; out->T[14] = 0.0; out->T[15] = 1.0;
  out->fitness = st.fitness;
  out->inlier_rmse = st.rmse;
  out->n_inliers = st.n_in;
  out->n_iter = st.k;
  out->status = st.status;
}

struct LoopIn {
  const double* T_init;  // 16 doubles
  double r;
  int32_t max_iter;
  double rel_tol;
};

// Steps 3 and 4 for n prepared pairs: initial states, loop, readback.  A
// single pair runs the per-pair kernels with arguments by value; several pairs
// run the batched kernels over the (pair, tile) item list.
int run_loop(icp_ctx* c, const Prep& P, const LoopIn* in, bool normals, int variant,
             int precision, icp_result_t* out) {
  hipStream_t s = c->stream;
  const Layout& L = P.L;
  const int n = P.n;
  int rc;
  // results are read back behind the staged header
  if ((rc = ensure_host(c, L.total + sizeof(IterState) * n)) != 0) return rc;
  char* hh = static_cast<char*>(c->host);
  char* dd = c->desc.as<char>();
  PassArgs* hp = reinterpret_cast<PassArgs*>(hh + L.pargs);
  SolveArgs* hs = reinterpret_cast<SolveArgs*>(hh + L.sargs);
  IterState* hst = reinterpret_cast<IterState*>(hh + L.states);
  uint2* hit = reinterpret_cast<uint2*>(hh + L.items);
  int32_t iters = 0;
  int64_t item = 0;
  for (int p = 0; p < n; ++p) {
    hp[p] = pass_args(c, P, p, in[p].r, true, normals);
    hs[p] = SolveArgs{hp[p].part, hp[p].n_blocks, const_cast<IterState*>(hp[p].st),
                      P.src_off[p + 1] - P.src_off[p], in[p].max_iter, in[p].rel_tol, 0};
    memset(&hst[p], 0, sizeof(IterState));
    for (int k = 0; k < 16; ++k) hst[p].T[k] = in[p].T_init[k];
    for (int t = 0; t < hp[p].n_blocks; ++t) hit[item++] = make_uint2((uint32_t)p, (uint32_t)t);
    iters = std::max(iters, in[p].max_iter);
  }
  HIP_TRY(hipMemsetAsync(dd + L.jprev, 0xff, 4 * (size_t)P.total_src, s), "memset");
  HIP_TRY(hipMemcpyAsync(dd + L.pargs, hh + L.pargs, L.header_end - L.pargs, hipMemcpyHostToDevice, s),
          "upload");
  const bool prof = c->profiling;
  if (prof && (rc = ensure_events(c, iters + 1)) != 0) return rc;
  if (prof) HIP_TRY(hipEventRecord(c->ev[0], s), "hipEventRecord");
  const PassArgs* dp = reinterpret_cast<const PassArgs*>(dd + L.pargs);
  const SolveArgs* ds = reinterpret_cast<const SolveArgs*>(dd + L.sargs);
  const uint2* di = reinterpret_cast<const uint2*>(dd + L.items);
  for (int32_t k = 0; k <= iters; ++k) {
    if (prof) HIP_TRY(hipEventRecord(c->ev[2 + 2 * k], s), "hipEventRecord");
    if (n == 1)
      HIP_TRY(launch_pass(hp[0], variant, precision, false, s), "pass");
    else
      HIP_TRY(launch_batch_pass(dp, di, (int)P.total_tiles, P.sub, variant, precision, s), "pass");
    if (prof) HIP_TRY(hipEventRecord(c->ev[3 + 2 * k], s), "hipEventRecord");
    if (n == 1)
      HIP_TRY(launch_solve(hs[0], s), "solve");
    else
      HIP_TRY(launch_batch_solve(ds, n, s), "solve");
  }
  if (prof) HIP_TRY(hipEventRecord(c->ev[1], s), "hipEventRecord");
  IterState* res = reinterpret_cast<IterState*>(hh + L.total);
  HIP_TRY(hipMemcpyAsync(res, dd + L.states, sizeof(IterState) * n, hipMemcpyDeviceToHost, s),
          "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  int32_t max_k = 0;
  int64_t evals = 0;
  for (int p = 0; p < n; ++p) {
    to_result(res[p], out + p);
    max_k = std::max(max_k, res[p].k);
    evals += (int64_t)(res[p].k + 1) * (P.src_off[p + 1] - P.src_off[p]);
  }
  if (prof && (rc = collect_profile(c, max_k + 1, evals)) != 0) return rc;
  return ICP_SUCCESS;
}

// One pass at a given pose for a single prepared pair (test hooks).
int single_pass(icp_ctx* c, const Prep& P, double r, const double T[16], bool normals, int variant,
                int precision, int32_t* idx_out, float* d2_out, bool reduce, IterState* st_out) {
  hipStream_t s = c->stream;
  PassArgs a = pass_args(c, P, 0, r, false, normals);
  a.idx_out = idx_out;
  a.d2_out = d2_out;
  HIP_TRY(launch_state_init(const_cast<IterState*>(a.st), T, s), "state init");
  HIP_TRY(launch_pass(a, variant, precision, idx_out != nullptr, s), "pass");
  if (reduce) {
    SolveArgs sa{a.part, a.n_blocks, const_cast<IterState*>(a.st), P.src_off[1], 0, 0.0, 1};
    HIP_TRY(launch_solve(sa, s), "reduce");
    int rc;
    if ((rc = ensure_host(c, P.L.total + sizeof(IterState))) != 0) return rc;
    IterState* res = reinterpret_cast<IterState*>(static_cast<char*>(c->host) + P.L.total);
    HIP_TRY(hipMemcpyAsync(res, a.st, sizeof(IterState), hipMemcpyDeviceToHost, s), "readback");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    *st_out = *res;
  } else {
    HIP_TRY(hipStreamSynchronize(s), "sync");
  }
  return ICP_SUCCESS;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* icp_version(void) { return "icp-mi355x 0.2 (gfx950)"; }

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

int icp_ctx_destroy(icp_ctx_t* ctx) {
  if (!ctx) return ICP_SUCCESS;
  ctx_free(ctx);
  delete ctx;
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

int icp_register(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const float* tgt_xyz,
                 const float* tgt_normals, int64_t n_tgt, const double T_init[16],
                 double max_corr_dist, int32_t max_iter, double rel_tol, int32_t variant,
                 int32_t precision, icp_result_t* out) {
  int rc = check_common(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T_init, max_corr_dist, variant,
                        precision, true);
  if (rc) return rc;
  if ((rc = check_iteration(max_iter, rel_tol)) != 0) return rc;
  if (!out) return fail(ICP_E_INVALID_ARG, "out is NULL");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  const PairIn in{src_xyz, n_src, tgt_xyz, plane ? tgt_normals : nullptr, n_tgt, max_corr_dist};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  const LoopIn li{T_init, max_corr_dist, max_iter, rel_tol};
  return run_loop(c, P, &li, plane, variant, precision, out);
}

int icp_register_batch(icp_ctx_t* ctx, const icp_pair_t* pairs, int32_t n_pairs, int32_t variant,
                       int32_t precision, icp_result_t* out) {
  if (!pairs || !out) return fail(ICP_E_INVALID_ARG, "pairs / out is NULL");
  if (n_pairs < 1) return fail(ICP_E_INVALID_ARG, "n_pairs must be >= 1");
  int rc;
  int64_t total_src = 0, total_tgt = 0;
  for (int p = 0; p < n_pairs; ++p) {
    const icp_pair_t& q = pairs[p];
    rc = check_common(q.src_xyz, q.n_src, q.tgt_xyz, q.tgt_normals, q.n_tgt, q.T_init,
                      q.max_corr_dist, variant, precision, true);
    if (!rc) rc = check_iteration(q.max_iter, q.rel_tol);
    if (!rc && q.reserved != 0) rc = fail(ICP_E_INVALID_ARG, "reserved must be 0");
    if (rc) {
      g_last_error += " (pair " + std::to_string(p) + ")";
      return rc;
    }
    total_src += q.n_src;
    total_tgt += q.n_tgt;
  }
  if (total_src > (int64_t)INT32_MAX || total_tgt > (int64_t)INT32_MAX)
    return fail(ICP_E_TOO_LARGE, "more than 2^31-1 points in one batch");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  std::vector<PairIn> in(n_pairs);
  std::vector<LoopIn> li(n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    const icp_pair_t& q = pairs[p];
    in[p] = PairIn{q.src_xyz, q.n_src, q.tgt_xyz, plane ? q.tgt_normals : nullptr, q.n_tgt,
                   q.max_corr_dist};
    li[p] = LoopIn{q.T_init, q.max_corr_dist, q.max_iter, q.rel_tol};
  }
  Prep P;
  if ((rc = prepare_pairs(c, n_pairs, in.data(), &P)) != 0) return rc;
  return run_loop(c, P, li.data(), plane, variant, precision, out);
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
  const PairIn in{src_xyz, n_src, tgt_xyz, nullptr, n_tgt, max_corr_dist};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  return single_pass(c, P, max_corr_dist, T, false, ICP_POINT_TO_POINT, ICP_PREC_F32_KAHAN_F64,
                     idx_out, d2_out, false, nullptr);
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
  const PairIn in{src_xyz, n_src, tgt_xyz, plane ? tgt_normals : nullptr, n_tgt, max_corr_dist};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  IterState st;
  if ((rc = single_pass(c, P, max_corr_dist, T, plane, variant, precision, nullptr, nullptr, true,
                        &st)) != 0)
    return rc;
  for (int k = 0; k < 21; ++k) AtA21[k] = st.sums[k];
  for (int k = 0; k < 6; ++k) Atb6[k] = st.sums[21 + k];
  *sum_d2 = st.sums[kSumD2];
  *n_in = (int64_t)st.sums[kSumCount];
  return ICP_SUCCESS;
}

}  // extern "C"
