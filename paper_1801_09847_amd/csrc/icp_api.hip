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

#include "icp_runtime.h"

using namespace icp;

namespace icp_rt {

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

int ctx_init(icp_ctx* c, int device, void* stream, size_t arena_bytes) {
  c->device = device;
  DeviceGuard g(device);
  if (!g.ok) return fail(ICP_E_DEVICE, "cannot select device " + std::to_string(device));
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
    c->own_stream = true;
  }
  size_t host_bytes = kHostBytes;
  if (arena_bytes > 0) {
    // one device allocation for the context's life; pinned staging sized
    // with it (a call's descriptors and results are far smaller than its
    // device buffers)
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&c->arena.base), arena_bytes), "hipMalloc (arena)");
    c->arena.size = arena_bytes;
    c->fixed = true;
    for_each_buf(c, [c](Buf& b) { b.arena = &c->arena; });
    host_bytes = std::min<size_t>(std::max<size_t>(arena_bytes / 256, (size_t)16 << 20), (size_t)256 << 20);
  }
  HIP_TRY(hipHostMalloc(&c->host, host_bytes, hipHostMallocDefault), "hipHostMalloc");
  c->host_cap = host_bytes;
  return ICP_SUCCESS;
}

void ctx_free(icp_ctx* c) {
  DeviceGuard g(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for_each_buf(c, [](Buf& b) { b.release(); });
  if (c->arena.base) (void)hipFree(c->arena.base);
  c->arena = Arena{};
  if (c->host) (void)hipHostFree(c->host);
  c->host = nullptr;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  for (hipEvent_t& e : c->ev_build)
    if (e) (void)hipEventDestroy(e), e = nullptr;
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
    // a new call: the arena's buffers are carved afresh
    if (in->fixed) {
      in->arena.top = 0;
      ++in->arena.epoch;
    }
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
  if (c->fixed)
    return fail(ICP_E_OOM, "call needs " + std::to_string(bytes) + " bytes of pinned staging; the context's is " +
                               std::to_string(c->host_cap) + " (arena_bytes / 256, at least 16 MiB)");
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
// smaller cells).  ICP_GRID_SUB overrides the default and the density choice
// (debugging and tests).
int grid_sub_env() {
  const char* e = getenv("ICP_GRID_SUB");
  if (e && atoi(e) == 1) return 1;
  if (e && atoi(e) == 2) return 2;
  return 0;
}

int grid_sub() {
  const int e = grid_sub_env();
  return e ? e : kDefaultSub;
}

// True when the target holds at least kFineSubPoints points per cell of the
// one-cell-per-radius grid over its box.
bool dense_target(const float* mn, const float* mx, double r, int64_t n_tgt) {
  const double inv_h = 1.0 / (r * (1.0 + 1.0 / 1024.0) * grid_scale());
  double cells = 1.0;
  for (int a = 0; a < 3; ++a) cells *= floor(((double)mx[a] - (double)mn[a]) * inv_h) + 1.0;
  return (double)n_tgt >= kFineSubPoints * cells;
}

// ICP_GRID_HASH=1 (debugging and tests only) gives every grid that may be
// hashed a hashed table, whatever its extent; results must not change.
bool grid_force_hash() {
  const char* e = getenv("ICP_GRID_HASH");
  return e && atoi(e) == 1;
}

// Grid over a target box: cell edge h >= r (1 + 2^-10) / sub so that every
// point within r of a query lies in the (2 sub + 1)^3 cells around the query's
// cell.  The dense table is capped at max(2^24, 32 n_tgt) cells.  A larger
// box gets a hashed table of 16 n_tgt slots (rounded up to a power of two, at
// least 2^16) at the same h when the call's kernels accept one (`hashed_ok`),
// else a grown h (still exact: any h above the bound works, only the
// candidate count changes).  A hashed grid still grows h if an axis would
// exceed 2^24 cells.
GridDesc make_grid(const float* mn, const float* mx, double r, int64_t n_tgt, bool hashed_ok, int sub) {
  // below 2^30 entries: the pass addresses the table with 32-bit byte offsets
  const double cap = std::min<double>(1073741824.0 - 1024.0, std::max<double>(16777216.0, 32.0 * (double)n_tgt));
  const double axis_cap = 16777216.0;
  const bool force = hashed_ok && grid_force_hash();
  double h = r * (1.0 + 1.0 / 1024.0) * grid_scale() / sub;
  GridDesc g{};
  for (int it = 0; it < 64; ++it) {
    const double inv_h = 1.0 / h;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = floor(((double)mx[a] - (double)mn[a]) * inv_h) + 1.0;
    const double cells = d[0] * d[1] * d[2];
    const double dmax = std::max(d[0], std::max(d[1], d[2]));
    const bool dense = cells <= cap && !force;
    const bool hashed = !dense && hashed_ok && dmax <= axis_cap;
    if (dense || hashed) {
      g.ox = mn[0]; g.oy = mn[1]; g.oz = mn[2];
      g.inv_h = inv_h;
      g.dx = (int32_t)d[0]; g.dy = (int32_t)d[1]; g.dz = (int32_t)d[2];
      g.sub = sub;
      g.hashed = hashed ? 1 : 0;
      if (dense) {
        g.ncell = (uint32_t)cells;
      } else {
        uint32_t slots = 1u << 16;
        while ((double)slots < 16.0 * (double)n_tgt && slots < (1u << 29)) slots <<= 1;
        g.ncell = slots;
      }
      return g;
    }
    h *= (hashed_ok ? dmax / axis_cap : std::cbrt(cells / cap)) * 1.001;
  }
  return g;  // unreachable for finite inputs
}

// ------------------------------------------------------------------ call layout
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
  L.blk_tab = take(sizeof(int64_t) * (n + 1));
  L.blk_occ = take(sizeof(int64_t) * (n + 1));
  L.pargs = take(sizeof(PassArgs) * n);
  L.sargs = take(sizeof(SolveArgs) * n);
  L.states = take(sizeof(IterState) * n);
  L.items = take(sizeof(uint2) * (size_t)std::max<int64_t>(n_items, 1));
  L.header_end = align256(off);
  L.bbox_out = take(sizeof(float) * 16 * n);
  L.jprev = take(sizeof(uint32_t) * (size_t)total_src);
  L.part = take(sizeof(double) * kNumSums * (size_t)total_tiles);
  L.red = take(sizeof(double) * kNumSums * kSegs);  // segment sums of a single pair's solve
  L.total = align256(off);
  return L;
}

int64_t tiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

// Step 1 of a call for n pairs: checks, boxes and grid sizes.  The staged
// build descriptors stay in pinned host memory for build_pairs.
int plan_pairs(icp_ctx* c, int n, const PairIn* in, Prep* P, int* bad) {
  hipStream_t s = c->stream;
  *bad = -1;
  P->n = n;
  P->normals = in[0].tgt_n != nullptr;
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

  // boxes and finiteness of all clouds (target with its normals, source)
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
    if (t[6] != 0.0f || q[6] != 0.0f) {
      *bad = p;
      return fail(ICP_E_NONFINITE, (t[6] != 0.0f ? std::string("non-finite target coordinate or normal")
                                                 : std::string("non-finite source coordinate")) +
                                       (n > 1 ? " in pair " + std::to_string(p) : std::string()));
    }
  }

  // grids and offsets
  P->g.resize(n);
  P->tab_off.assign(n + 1, 0);
  BuildPair* bp = reinterpret_cast<BuildPair*>(hh + L.pairs);
  int64_t* bt = reinterpret_cast<int64_t*>(hh + L.blk_t);
  int64_t* bs = reinterpret_cast<int64_t*>(hh + L.blk_s);
  int64_t* so = reinterpret_cast<int64_t*>(hh + L.src_off);
  int64_t* bk = reinterpret_cast<int64_t*>(hh + L.blk_tab);
  int64_t* bo2 = reinterpret_cast<int64_t*>(hh + L.blk_occ);
  P->occ_off.assign(n + 1, 0);
  bt[0] = 0;
  bs[0] = 0;
  bk[0] = 0;
  bo2[0] = 0;
  // one cell size per call (the batched kernels take it as a template
  // argument): two cells per radius only if every pair allows it and has a
  // dense target
  int sub = grid_sub();
  if (!grid_sub_env()) {
    bool fine = true;
    for (int p = 0; p < n && fine; ++p)
      fine = in[p].fine_ok && dense_target(hbox + 16 * p, hbox + 16 * p + 3, in[p].r, in[p].n_tgt);
    if (fine) sub = 2;
  }
  for (int p = 0; p < n; ++p) {
    const float* t = hbox + 16 * p;
    const float* q = t + 8;
    P->g[p] = make_grid(t, t + 3, in[p].r, in[p].n_tgt, in[p].hashed_ok, sub);
    P->tab_off[p + 1] = P->tab_off[p] + (uint64_t)P->g[p].ncell + 1;
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, (double)q[3 + a] - (double)q[a]);
    // Morton grid of the source: 1024 cells per axis over the source's own box,
    // so the order (and the summation order) depends on the source only
    const double hs = ext > 0.0 ? ext / 1023.5 : 1.0;
    bp[p] = BuildPair{in[p].src, in[p].tgt, in[p].tgt_n, in[p].n_src, in[p].n_tgt,
                      P->src_off[p], P->tgt_off[p], P->tab_off[p], P->g[p],
                      (double)q[0], (double)q[1], (double)q[2], 1.0 / hs,
                      nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                      P->occ_off[p], nullptr};
    bt[p + 1] = bt[p] + (in[p].n_tgt + 255) / 256;
    bs[p + 1] = bs[p] + (in[p].n_src + 255) / 256;
    bk[p + 1] = bk[p] + ((int64_t)P->g[p].ncell + 1 + 255) / 256;
    P->occ_off[p + 1] = P->occ_off[p] + occ_words(P->g[p]);
    bo2[p + 1] = bo2[p] + (int64_t)((occ_words(P->g[p]) + 255) / 256);
    so[p] = P->src_off[p];
  }
  so[n] = P->src_off[n];
  P->total_tab = P->tab_off[n];
  P->total_occ = P->occ_off[n];
  if (P->total_tab >= (uint64_t)UINT32_MAX)
    return fail(ICP_E_TOO_LARGE, "grid tables of one call exceed 2^32 cells");
  P->sub = P->g[0].sub;
  return ICP_SUCCESS;
}

// Step 2: segmented build of a planned call into dst[] (null: slices of the
// context's concatenated arrays; the cell tables are then localised in place).
int build_pairs(icp_ctx* c, Prep* P, const PairDst* dst) {
  hipStream_t s = c->stream;
  const Layout& L = P->L;
  const int n = P->n;
  const bool normals = P->normals;
  char* hh = static_cast<char*>(c->host);
  char* dd = c->desc.as<char>();
  BuildPair* bp = reinterpret_cast<BuildPair*>(hh + L.pairs);
  const int64_t* bt = reinterpret_cast<const int64_t*>(hh + L.blk_t);
  const int64_t* bs = reinterpret_cast<const int64_t*>(hh + L.blk_s);
  const int64_t* bk = reinterpret_cast<const int64_t*>(hh + L.blk_tab);
  const int64_t scan_cap = scan_block_sums_needed((int64_t)P->total_tab);
  const int64_t hist_cap = radix_hist_needed(P->total_src);
  HIP_TRY(c->cs.ensure(4 * (size_t)P->total_tab), "alloc");
  HIP_TRY(c->perm.ensure(4 * (size_t)P->total_src), "alloc");
  HIP_TRY(c->occ_raw.ensure(4 * (size_t)std::max<uint64_t>(P->total_occ, 1)), "alloc");
  if (!dst) {
    HIP_TRY(c->occ.ensure(4 * (size_t)std::max<uint64_t>(P->total_occ, 1)), "alloc");
    HIP_TRY(c->tp.ensure(16 * (size_t)P->total_tgt), "alloc");
    if (normals) HIP_TRY(c->tn.ensure(16 * (size_t)P->total_tgt), "alloc");
    HIP_TRY(c->sx.ensure(4 * (size_t)P->total_src), "alloc");
    HIP_TRY(c->sy.ensure(4 * (size_t)P->total_src), "alloc");
    HIP_TRY(c->sz.ensure(4 * (size_t)P->total_src), "alloc");
  }
  HIP_TRY(c->t_key.ensure(4 * (size_t)P->total_tgt), "alloc");
  HIP_TRY(c->t_rank.ensure(4 * (size_t)P->total_tgt), "alloc");
  HIP_TRY(c->scan_tmp.ensure(4 * (size_t)scan_cap), "alloc");
  HIP_TRY(c->s_hist.ensure(4 * (size_t)hist_cap), "alloc");
  for (Buf& b : c->sk) HIP_TRY(b.ensure(4 * ((size_t)P->total_src + 1)), "alloc");
  for (int p = 0; p < n; ++p) {
    if (dst) {
      bp[p].cs_dst = dst[p].cs;
      bp[p].tp_dst = dst[p].tp;
      bp[p].tn_dst = normals ? dst[p].tn : nullptr;
      bp[p].sx_dst = dst[p].sx;
      bp[p].sy_dst = dst[p].sy;
      bp[p].sz_dst = dst[p].sz;
      bp[p].perm_dst = dst[p].perm ? dst[p].perm : c->perm.as<uint32_t>() + P->src_off[p];
      bp[p].occ_dst = dst[p].occ;
    } else {
      bp[p].cs_dst = c->cs.as<uint32_t>() + P->tab_off[p];
      bp[p].tp_dst = c->tp.as<float4>() + P->tgt_off[p];
      bp[p].tn_dst = normals ? c->tn.as<float4>() + P->tgt_off[p] : nullptr;
      bp[p].sx_dst = c->sx.as<float>() + P->src_off[p];
      bp[p].sy_dst = c->sy.as<float>() + P->src_off[p];
      bp[p].sz_dst = c->sz.as<float>() + P->src_off[p];
      bp[p].perm_dst = c->perm.as<uint32_t>() + P->src_off[p];
      bp[p].occ_dst = c->occ.as<uint32_t>() + P->occ_off[p];
    }
  }
  HIP_TRY(hipMemcpyAsync(dd + L.pairs, hh + L.pairs, L.pargs - L.pairs, hipMemcpyHostToDevice, s),
          "upload");
  const BuildPair* dbp = reinterpret_cast<const BuildPair*>(dd + L.pairs);
  if (c->profiling) {
    for (hipEvent_t& e : c->ev_build)
      if (!e) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    HIP_TRY(hipEventRecord(c->ev_build[0], s), "hipEventRecord");
  }
  HIP_TRY(launch_occ_clear(c->occ_raw.as<uint32_t>(), P->total_occ, s), "occupancy clear");
  HIP_TRY(launch_seg_targets(dbp, n, reinterpret_cast<const int64_t*>(dd + L.blk_t), bt[n],
                             reinterpret_cast<const int64_t*>(dd + L.blk_tab), bk[n],
                             P->total_tab, c->cs.as<uint32_t>(), c->t_key.as<uint32_t>(),
                             c->t_rank.as<uint32_t>(), c->scan_tmp.as<uint32_t>(), scan_cap,
                             dst != nullptr, c->occ_raw.as<uint32_t>(), s),
          "target grid");
  bool any_hashed = false;
  for (int p = 0; p < n; ++p) any_hashed = any_hashed || P->g[p].hashed;
  if (any_hashed)
    HIP_TRY(launch_hashed_occ(dbp, n, reinterpret_cast<const int64_t*>(dd + L.blk_t), bt[n],
                              c->occ_raw.as<uint32_t>(), s),
            "hashed occupancy");
  {
    const int64_t* bo2 = reinterpret_cast<const int64_t*>(hh + L.blk_occ);
    HIP_TRY(launch_occ_dilate(dbp, n, reinterpret_cast<const int64_t*>(dd + L.blk_occ), bo2[n],
                              c->occ_raw.as<uint32_t>(), s),
            "occupancy dilation");
  }
  SortBufs sb;
  for (int k = 0; k < 2; ++k) {
    sb.klo[k] = c->sk[k].as<uint32_t>();
    sb.khi[k] = c->sk[2 + k].as<uint32_t>();
    sb.val[k] = c->sk[4 + k].as<uint32_t>();
  }
  HIP_TRY(launch_seg_sources(dbp, n, reinterpret_cast<const int64_t*>(dd + L.blk_s), bs[n],
                             reinterpret_cast<const int64_t*>(dd + L.src_off), P->total_src, sb,
                             c->s_hist.as<uint32_t>(), hist_cap, s),
          "source order");
  if (c->profiling) {
    HIP_TRY(hipEventRecord(c->ev_build[1], s), "hipEventRecord");
    c->build_pending = P->total_tgt;
    for (int p = 0; p < n; ++p) {
      c->prof.hashed_grids += P->g[p].hashed;
      c->prof.fine_grids += P->g[p].sub == 2;
    }
  }
  return ICP_SUCCESS;
}

int prepare_pairs(icp_ctx* c, int n, const PairIn* in, Prep* P) {
  int bad = -1, rc;
  if ((rc = plan_pairs(c, n, in, P, &bad)) != 0) return rc;
  return build_pairs(c, P, nullptr);
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
  a.tp = c->tp.as<float4>() + P.tgt_off[p];
  a.tn = normals ? c->tn.as<float4>() + P.tgt_off[p] : nullptr;
  a.cs = c->cs.as<uint32_t>() + P.tab_off[p];
  a.occ = c->occ.as<uint32_t>() + P.occ_off[p];
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
  if (c->build_pending) {
    HIP_TRY(hipEventElapsedTime(&ms, c->ev_build[0], c->ev_build[1]), "hipEventElapsedTime");
    c->prof.build_ms += ms;
    c->prof.builds += 1;
    c->prof.build_points += c->build_pending;
    c->build_pending = 0;
  }
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
  int32_t loss = 0;      // robust loss (0: none)
  double loss_k = 1.0;
};

int check_loss(int32_t loss, double k) {
  if (loss < ICP_LOSS_NONE || loss > ICP_LOSS_CAUCHY) return fail(ICP_E_INVALID_ARG, "unknown loss");
  if (loss != ICP_LOSS_NONE && !(k > 0.0 && std::isfinite(k) && (float)k > 0.0f && std::isfinite((float)k)))
    return fail(ICP_E_INVALID_ARG, "loss_k must be finite and > 0 (also in float32)");
  return ICP_SUCCESS;
}

void set_loss(PassArgs* a, int32_t loss, double k) {
  a->loss = loss;
  a->loss_k = k;
  a->loss_k32 = (float)k;
}

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
  bool robust = false;
  for (int p = 0; p < n; ++p) {
    robust = robust || in[p].loss != ICP_LOSS_NONE;
    hp[p] = pass_args(c, P, p, in[p].r, true, normals);
    set_loss(&hp[p], in[p].loss, in[p].loss_k);
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
      HIP_TRY(launch_batch_pass(dp, di, (int)P.total_tiles, P.sub, variant, precision, robust, s), "pass");
    if (prof) HIP_TRY(hipEventRecord(c->ev[3 + 2 * k], s), "hipEventRecord");
    if (n == 1)
      HIP_TRY(launch_solve(hs[0], reinterpret_cast<double*>(dd + L.red), s), "solve");
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
                int precision, int32_t* idx_out, float* d2_out, bool reduce, IterState* st_out,
                int32_t loss, double loss_k) {
  hipStream_t s = c->stream;
  PassArgs a = pass_args(c, P, 0, r, false, normals);
  set_loss(&a, loss, loss_k);
  a.idx_out = idx_out;
  a.d2_out = d2_out;
  HIP_TRY(launch_state_init(const_cast<IterState*>(a.st), T, s), "state init");
  HIP_TRY(launch_pass(a, variant, precision, idx_out != nullptr, s), "pass");
  if (reduce) {
    SolveArgs sa{a.part, a.n_blocks, const_cast<IterState*>(a.st), P.src_off[1], 0, 0.0, 1};
    HIP_TRY(launch_solve(sa, nullptr, s), "reduce");
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

// ------------------------------------------------------------------ voxel downsampling
// Downsamples m clouds in one segmented call; counts[c] receives the number of
// occupied voxels of cloud c (outputs beyond cap are not written).  `bad`
// receives the first cloud with a non-finite value, or -1.
int downsample_clouds(icp_ctx* c, int m, const VoxIn* in, int64_t* counts, int* bad) {
  hipStream_t s = c->stream;
  *bad = -1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align256(off);
    off = o + bytes;
    return o;
  };
  const size_t o_clouds = take(sizeof(SegCloud) * m);
  const size_t o_bblk = take(sizeof(int64_t) * (m + 1));
  const size_t o_vox = take(sizeof(VoxCloud) * m);
  const size_t o_vblk = take(sizeof(int64_t) * (m + 1));
  const size_t o_ptoff = take(sizeof(int64_t) * (m + 1));
  const size_t o_upload = align256(off);
  const size_t o_box = take(sizeof(float) * 8 * m);
  const size_t o_counts = take(sizeof(int64_t) * m);
  const size_t total_bytes = align256(off);
  int rc;
  if ((rc = ensure_host(c, total_bytes)) != 0) return rc;
  HIP_TRY(c->vdesc.ensure(total_bytes), "alloc");
  char* hh = static_cast<char*>(c->host);
  char* dd = c->vdesc.as<char>();
  SegCloud* cl = reinterpret_cast<SegCloud*>(hh + o_clouds);
  int64_t* bb = reinterpret_cast<int64_t*>(hh + o_bblk);
  bb[0] = 0;
  int64_t total = 0;
  for (int k = 0; k < m; ++k) {
    cl[k] = SegCloud{in[k].pts, in[k].nrm, in[k].n};
    bb[k + 1] = bb[k] + bbox_blocks(in[k].n);
    total += in[k].n;
  }
  if (total > (int64_t)INT32_MAX) return fail(ICP_E_TOO_LARGE, "more than 2^31-1 points in one call");
  HIP_TRY(c->bbox_part.ensure(sizeof(float) * 8 * (size_t)bb[m]), "alloc");
  HIP_TRY(hipMemcpyAsync(dd, hh, o_vox, hipMemcpyHostToDevice, s), "upload");
  HIP_TRY(launch_seg_bbox(reinterpret_cast<SegCloud*>(dd + o_clouds), m,
                          reinterpret_cast<int64_t*>(dd + o_bblk), bb[m], c->bbox_part.as<float>(),
                          reinterpret_cast<float*>(dd + o_box), s),
          "bbox");
  float* hbox = reinterpret_cast<float*>(hh + o_box);
  HIP_TRY(hipMemcpyAsync(hbox, dd + o_box, sizeof(float) * 8 * m, hipMemcpyDeviceToHost, s), "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  VoxCloud* vc = reinterpret_cast<VoxCloud*>(hh + o_vox);
  int64_t* vb = reinterpret_cast<int64_t*>(hh + o_vblk);
  int64_t* po = reinterpret_cast<int64_t*>(hh + o_ptoff);
  vb[0] = 0;
  po[0] = 0;
  bool wide = false;
  if (m > 65535) return fail(ICP_E_TOO_LARGE, "more than 65535 clouds in one downsampling call");
  for (int k = 0; k < m; ++k) {
    const float* b = hbox + 8 * k;
    if (b[6] != 0.0f) {
      *bad = k;
      return fail(ICP_E_NONFINITE, "non-finite coordinate or normal in a cloud to downsample");
    }
    const double inv_v = 1.0 / in[k].voxel;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = floor(((double)b[3 + a] - (double)b[a]) * inv_v) + 1.0;
    if (d[0] * d[1] * d[2] >= 281474976710656.0)
      return fail(ICP_E_TOO_LARGE, "voxel grid of a cloud exceeds 2^48 voxels");
    if (d[0] * d[1] * d[2] >= 4294967296.0) wide = true;
    vc[k] = VoxCloud{in[k].pts, in[k].nrm, in[k].n, po[k], (double)b[0], (double)b[1], (double)b[2],
                     inv_v, (int32_t)d[0], (int32_t)d[1], (int32_t)d[2], 0, in[k].out_pts,
                     in[k].out_nrm, in[k].cap};
    vb[k + 1] = vb[k] + (in[k].n + 255) / 256;
    po[k + 1] = po[k] + in[k].n;
  }
  const int64_t hist_cap = radix_hist_needed(total);
  const int64_t scan_cap = std::max(scan_block_sums_needed(total), (int64_t)1);
  for (Buf& b : c->sk) HIP_TRY(b.ensure(4 * ((size_t)total + 1)), "alloc");
  HIP_TRY(c->s_hist.ensure(4 * (size_t)hist_cap), "alloc");
  HIP_TRY(c->scan_tmp.ensure(4 * (size_t)scan_cap), "alloc");
  HIP_TRY(c->vflags.ensure(4 * (size_t)voxel_scratch_words(total)), "alloc");
  HIP_TRY(c->vstarts.ensure(4 * (size_t)voxel_scratch_words(total)), "alloc");
  HIP_TRY(hipMemcpyAsync(dd + o_vox, hh + o_vox, o_upload - o_vox, hipMemcpyHostToDevice, s), "upload");
  SortBufs sb;
  for (int k = 0; k < 2; ++k) {
    sb.klo[k] = c->sk[k].as<uint32_t>();
    sb.khi[k] = c->sk[2 + k].as<uint32_t>();
    sb.val[k] = c->sk[4 + k].as<uint32_t>();
  }
  HIP_TRY(launch_seg_voxel(reinterpret_cast<VoxCloud*>(dd + o_vox), m, wide,
                           reinterpret_cast<int64_t*>(dd + o_vblk), vb[m],
                           reinterpret_cast<int64_t*>(dd + o_ptoff), total, sb,
                           c->s_hist.as<uint32_t>(), hist_cap, c->vflags.as<uint32_t>(),
                           c->vstarts.as<uint32_t>(), c->scan_tmp.as<uint32_t>(), scan_cap,
                           reinterpret_cast<int64_t*>(dd + o_counts), s),
          "voxel downsample");
  int64_t* hc = reinterpret_cast<int64_t*>(hh + o_counts);
  HIP_TRY(hipMemcpyAsync(hc, dd + o_counts, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s), "readback");
  HIP_TRY(hipStreamSynchronize(s), "sync");
  for (int k = 0; k < m; ++k) counts[k] = hc[k];
  return ICP_SUCCESS;
}

}  // namespace icp_rt

using namespace icp_rt;

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

int icp_ctx_create(int device, void* hip_stream, size_t arena_bytes, icp_ctx_t** out) {
  if (!out) return fail(ICP_E_INVALID_ARG, "out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(ICP_E_INVALID_ARG, "device index out of range");
  icp_ctx* c = new icp_ctx();
  const int rc = ctx_init(c, device, hip_stream, arena_bytes);
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
  ctx->build_pending = 0;
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
  return icp_register_robust(ctx, src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T_init, max_corr_dist,
                             max_iter, rel_tol, variant, precision, ICP_LOSS_NONE, 1.0, out);
}

int icp_register_robust(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const float* tgt_xyz,
                        const float* tgt_normals, int64_t n_tgt, const double T_init[16],
                        double max_corr_dist, int32_t max_iter, double rel_tol, int32_t variant,
                        int32_t precision, int32_t loss, double loss_k, icp_result_t* out) {
  int rc = check_common(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T_init, max_corr_dist, variant,
                        precision, true);
  if (rc) return rc;
  if ((rc = check_iteration(max_iter, rel_tol)) != 0) return rc;
  if ((rc = check_loss(loss, loss_k)) != 0) return rc;
  if (!out) return fail(ICP_E_INVALID_ARG, "out is NULL");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  const PairIn in{src_xyz, n_src, tgt_xyz, plane ? tgt_normals : nullptr, n_tgt, max_corr_dist, true, true};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  LoopIn li{T_init, max_corr_dist, max_iter, rel_tol};
  li.loss = loss;
  li.loss_k = loss_k;
  return run_loop(c, P, &li, plane, variant, precision, out);
}

int icp_register_batch(icp_ctx_t* ctx, const icp_pair_t* pairs, int32_t n_pairs, int32_t variant,
                       int32_t precision, icp_result_t* out) {
  return icp_register_batch_robust(ctx, pairs, n_pairs, variant, precision, ICP_LOSS_NONE, 1.0, out);
}

int icp_register_batch_robust(icp_ctx_t* ctx, const icp_pair_t* pairs, int32_t n_pairs, int32_t variant,
                              int32_t precision, int32_t loss, double loss_k, icp_result_t* out) {
  if (!pairs || !out) return fail(ICP_E_INVALID_ARG, "pairs / out is NULL");
  if (n_pairs < 1) return fail(ICP_E_INVALID_ARG, "n_pairs must be >= 1");
  int rc;
  if ((rc = check_loss(loss, loss_k)) != 0) return rc;
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
                   q.max_corr_dist, true, true};
    li[p] = LoopIn{q.T_init, q.max_corr_dist, q.max_iter, q.rel_tol, loss, loss_k};
  }
  Prep P;
  if ((rc = prepare_pairs(c, n_pairs, in.data(), &P)) != 0) return rc;
  return run_loop(c, P, li.data(), plane, variant, precision, out);
}

int icp_voxel_downsample(icp_ctx_t* ctx, const float* pts, const float* normals, int64_t n,
                         double voxel, float* out_pts, float* out_normals, int64_t cap,
                         int64_t* n_out) {
  int rc;
  if ((rc = check_cloud(pts, n, "pts")) != 0) return rc;
  if (!(voxel > 0.0) || !std::isfinite(voxel)) return fail(ICP_E_INVALID_ARG, "voxel must be finite and > 0");
  if (!out_pts || !n_out || cap < 1) return fail(ICP_E_INVALID_ARG, "out_pts / n_out is NULL or cap < 1");
  if (normals && !out_normals) return fail(ICP_E_INVALID_ARG, "out_normals is NULL while normals are given");
  if ((reinterpret_cast<uintptr_t>(out_pts) & 3u) || (normals && (reinterpret_cast<uintptr_t>(normals) & 3u)) ||
      (out_normals && (reinterpret_cast<uintptr_t>(out_normals) & 3u)))
    return fail(ICP_E_INVALID_ARG, "pointer is not 4-byte aligned");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const VoxIn in{pts, normals, n, voxel, out_pts, normals ? out_normals : nullptr, cap};
  int64_t cnt = 0;
  int bad = -1;
  if ((rc = downsample_clouds(c, 1, &in, &cnt, &bad)) != 0) return rc;
  *n_out = cnt;
  if (cnt > cap) return fail(ICP_E_TOO_LARGE, "output capacity too small: " + std::to_string(cnt) + " voxels");
  return ICP_SUCCESS;
}

int icp_estimate_normals(icp_ctx_t* ctx, const float* pts, int64_t n, double radius, int32_t max_nn,
                         const double viewpoint[3], float* normals_out, int32_t* counts_out) {
  int rc;
  if ((rc = check_cloud(pts, n, "pts")) != 0) return rc;
  if (!(radius > 0.0) || !std::isfinite(radius) || !std::isfinite((float)(radius * radius)))
    return fail(ICP_E_INVALID_ARG, "radius must be > 0 with a finite float32 square");
  if (max_nn < 1 || max_nn > kMaxNormalNN)
    return fail(ICP_E_INVALID_ARG, "max_nn must be in [1, " + std::to_string(kMaxNormalNN) + "]");
  if (!viewpoint || !std::isfinite(viewpoint[0]) || !std::isfinite(viewpoint[1]) ||
      !std::isfinite(viewpoint[2]))
    return fail(ICP_E_INVALID_ARG, "viewpoint is NULL or not finite");
  if (!normals_out) return fail(ICP_E_INVALID_ARG, "normals_out is NULL");
  if ((reinterpret_cast<uintptr_t>(normals_out) & 3u) || (reinterpret_cast<uintptr_t>(counts_out) & 3u))
    return fail(ICP_E_INVALID_ARG, "output pointer is not 4-byte aligned");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  // the cloud is prepared as both the queries (Morton order) and the grid
  const PairIn in{pts, n, pts, nullptr, n, radius};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  NormalArgs a;
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
  a.vx = viewpoint[0];
  a.vy = viewpoint[1];
  a.vz = viewpoint[2];
  a.normals = normals_out;
  a.counts = counts_out;
  HIP_TRY(launch_normals(a, P.g[0].sub, c->stream), "normals");
  HIP_TRY(hipStreamSynchronize(c->stream), "sync");
  return ICP_SUCCESS;
}

int icp_register_multiscale(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const float* tgt_xyz,
                            const float* tgt_normals, int64_t n_tgt, const double T_init[16],
                            int32_t n_levels, const double* voxel, const int32_t* max_iter,
                            const double* max_corr_dist, double rel_tol, int32_t variant,
                            int32_t precision, icp_result_t* out) {
  return icp_register_multiscale_robust(ctx, src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T_init, n_levels,
                                        voxel, max_iter, max_corr_dist, rel_tol, variant, precision,
                                        ICP_LOSS_NONE, 1.0, out);
}

int icp_register_multiscale_robust(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const float* tgt_xyz,
                                   const float* tgt_normals, int64_t n_tgt, const double T_init[16],
                                   int32_t n_levels, const double* voxel, const int32_t* max_iter,
                                   const double* max_corr_dist, double rel_tol, int32_t variant,
                                   int32_t precision, int32_t loss, double loss_k, icp_result_t* out) {
  if (check_loss(loss, loss_k) != 0) return ICP_E_INVALID_ARG;
  if (n_levels < 1 || n_levels > 16 || !voxel || !max_iter || !max_corr_dist)
    return fail(ICP_E_INVALID_ARG, "n_levels must be in [1, 16] with voxel / max_iter / max_corr_dist given");
  int rc;
  for (int l = 0; l < n_levels; ++l) {
    rc = check_common(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T_init, max_corr_dist[l], variant,
                      precision, true);
    if (!rc) rc = check_iteration(max_iter[l], rel_tol);
    if (!rc && !(voxel[l] >= 0.0 && std::isfinite(voxel[l])))
      rc = fail(ICP_E_INVALID_ARG, "voxel must be finite and >= 0 (0: no downsampling)");
    if (rc) {
      g_last_error += " (level " + std::to_string(l) + ")";
      return rc;
    }
  }
  if (!out) return fail(ICP_E_INVALID_ARG, "out is NULL");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  double T[16];
  memcpy(T, T_init, sizeof T);
  icp_result_t res{};
  int32_t iters_total = 0;
  for (int l = 0; l < n_levels; ++l) {
    const float* s = src_xyz;
    const float* t = tgt_xyz;
    const float* tn = plane ? tgt_normals : nullptr;
    int64_t ns = n_src, nt = n_tgt;
    if (voxel[l] > 0.0) {
      HIP_TRY(c->lvl_src.ensure(12 * (size_t)n_src), "alloc");
      HIP_TRY(c->lvl_tgt.ensure(12 * (size_t)n_tgt), "alloc");
      if (plane) HIP_TRY(c->lvl_tn.ensure(12 * (size_t)n_tgt), "alloc");
      const VoxIn vin[2] = {{src_xyz, nullptr, n_src, voxel[l], c->lvl_src.as<float>(), nullptr, n_src},
                            {tgt_xyz, tn, n_tgt, voxel[l], c->lvl_tgt.as<float>(),
                             plane ? c->lvl_tn.as<float>() : nullptr, n_tgt}};
      int64_t cnt[2];
      int bad = -1;
      if ((rc = downsample_clouds(c, 2, vin, cnt, &bad)) != 0) return rc;
      s = c->lvl_src.as<float>();
      t = c->lvl_tgt.as<float>();
      tn = plane ? c->lvl_tn.as<float>() : nullptr;
      ns = cnt[0];
      nt = cnt[1];
    }
    const PairIn in{s, ns, t, tn, nt, max_corr_dist[l], true, true};
    Prep P;
    if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
    const LoopIn li{T, max_corr_dist[l], max_iter[l], rel_tol, loss, loss_k};
    if ((rc = run_loop(c, P, &li, plane, variant, precision, &res)) != 0) return rc;
    iters_total += res.n_iter;
    memcpy(T, res.T, sizeof T);
    if (res.status == ICP_DEGENERATE) break;
  }
  res.n_iter = iters_total;
  *out = res;
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
  const PairIn in{src_xyz, n_src, tgt_xyz, nullptr, n_tgt, max_corr_dist, true, true};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  return single_pass(c, P, max_corr_dist, T, false, ICP_POINT_TO_POINT, ICP_PREC_F32_KAHAN_F64,
                     idx_out, d2_out, false, nullptr, ICP_LOSS_NONE, 1.0);
}

int icp_normal_equations(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src, const double T[16],
                         const float* tgt_xyz, const float* tgt_normals, int64_t n_tgt,
                         double max_corr_dist, int32_t variant, int32_t precision, double AtA21[21],
                         double Atb6[6], double* sum_d2, int64_t* n_in) {
  return icp_normal_equations_robust(ctx, src_xyz, n_src, T, tgt_xyz, tgt_normals, n_tgt,
                                     max_corr_dist, variant, precision, ICP_LOSS_NONE, 1.0, AtA21,
                                     Atb6, sum_d2, n_in);
}

int icp_normal_equations_robust(icp_ctx_t* ctx, const float* src_xyz, int64_t n_src,
                                const double T[16], const float* tgt_xyz, const float* tgt_normals,
                                int64_t n_tgt, double max_corr_dist, int32_t variant,
                                int32_t precision, int32_t loss, double loss_k, double AtA21[21],
                                double Atb6[6], double* sum_d2, int64_t* n_in) {
  int rc = check_common(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, T, max_corr_dist, variant,
                        precision, true);
  if (rc) return rc;
  if ((rc = check_loss(loss, loss_k)) != 0) return rc;
  if (!AtA21 || !Atb6 || !sum_d2 || !n_in) return fail(ICP_E_INVALID_ARG, "output pointer is NULL");
  icp_ctx* c = nullptr;
  if ((rc = resolve_ctx(ctx, &c)) != 0) return rc;
  DeviceGuard dg(c->device);
  const bool plane = variant == ICP_POINT_TO_PLANE;
  const PairIn in{src_xyz, n_src, tgt_xyz, plane ? tgt_normals : nullptr, n_tgt, max_corr_dist, true, true};
  Prep P;
  if ((rc = prepare_pairs(c, 1, &in, &P)) != 0) return rc;
  IterState st;
  if ((rc = single_pass(c, P, max_corr_dist, T, plane, variant, precision, nullptr, nullptr, true,
                        &st, loss, loss_k)) != 0)
    return rc;
  for (int k = 0; k < 21; ++k) AtA21[k] = st.sums[k];
  for (int k = 0; k < 6; ++k) Atb6[k] = st.sums[21 + k];
  *sum_d2 = st.sums[kSumD2];
  *n_in = (int64_t)st.sums[kSumCount];
  return ICP_SUCCESS;
}

}  // extern "C"
