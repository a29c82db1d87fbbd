// Request server: continuous batching of coarse-to-fine registrations.
//
// Life of a request: submit (inputs copied into the server's memory pool, or
// into host memory when the pool is momentarily full) -> queued -> admitted
// into a free slot -> per level: voxel downsampling of both clouds, grid build
// and Morton ordering (segmented over every request entering a level in the
// same step), then ICP iterations run together with all other running
// requests -> completion.  All device memory of a request comes from one
// first-fit pool of the configured budget, so the step loop never calls
// hipMalloc.  Each step uploads the slot table (pass arguments, solve
// arguments, (slot, tile) work items) and replays one instantiated graph: a
// chain of `iters_per_step` (batched pass, batched solve) kernel nodes whose
// grids are set to the step's item and slot counts before the replay.  A slot
// whose level finished mid-step is skipped on device by its done flag.

#include <string.h>
#include <time.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "icp_runtime.h"

using namespace icp;
using namespace icp_rt;

namespace {

int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

// First-fit pool over one device allocation (offsets 256-byte aligned).
struct Pool {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  void init(char* b, size_t c) {
    base = b;
    cap = c & ~(size_t)255;
    free_.clear();
    free_[0] = cap;
    used = 0;
  }
  void* alloc(size_t bytes) {
    bytes = align256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used += bytes;
      return base + off;
    }
    return nullptr;
  }
  void release(void* p, size_t bytes) {
    if (!p) return;
    bytes = align256(std::max<size_t>(bytes, 1));
    size_t off = static_cast<char*>(p) - base;
    used -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
};

enum ReqState { kQueued = 0, kPrep = 1, kRun = 2 };

struct Req {
  uint64_t ticket = 0, tag = 0;
  int64_t n_src = 0, n_tgt = 0;
  double T[16];
  double rel_tol = 0.0, spacing = 0.0;
  // inputs: in the pool, or on the host until admission
  float *src = nullptr, *tgt = nullptr, *tgt_n = nullptr;
  size_t in_bytes = 0;
  std::vector<float> h_src, h_tgt, h_tn;
  // current level
  int level = 0;
  int state = kQueued;
  int32_t iters_total = 0;
  float *ls = nullptr, *lt = nullptr, *ltn = nullptr;  // downsampled clouds (or inputs)
  void* lvl_mem = nullptr;
  size_t lvl_bytes = 0;
  int64_t lns = 0, lnt = 0;
  void* prep_mem = nullptr;
  size_t prep_bytes = 0;
  PassArgs pa;
  SolveArgs sa;
  int64_t t_submit = 0, t_admit = 0;
};

}  // namespace

struct icp_server {
  icp_server_cfg_t cfg;
  icp_ctx* ctx = nullptr;
  hipStream_t copy_stream = nullptr;
  Buf pool_mem;
  Pool pool;
  Buf table;  // PassArgs[slots] | SolveArgs[slots] | uint2 items[items_cap] | IterState[slots]
  size_t o_pargs = 0, o_sargs = 0, o_items = 0, o_states = 0, table_bytes = 0;
  int64_t items_cap = 0;
  void* host_table = nullptr;  // pinned mirror
  // step graph: nodes[2k] = pass of iteration k, nodes[2k+1] = its solve
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipGraphNode_t> nodes;
  std::vector<hipKernelNodeParams> node_params;
  const PassArgs* d_pargs = nullptr;  // kernel argument values the nodes point at
  const uint2* d_items = nullptr;
  const SolveArgs* d_sargs = nullptr;
  void* pass_args[2] = {nullptr, nullptr};
  void* solve_args[1] = {nullptr};
  uint64_t fault_tag = 0;
  bool fault_on = false;
  // host-forced step failure (failure-handling tests): step number fault_step
  // returns ICP_E_DEVICE before any device work
  int64_t fault_step = -1;
  int64_t step_count = 0;
  // bookkeeping (mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::vector<Req*> active;
  std::unordered_map<uint64_t, int> pending;  // ticket -> 1 while not completed
  std::deque<icp_completion_t> done;
  uint64_t next_ticket = 1;
  std::thread worker;
  bool stop = false;
  bool broken = false;
  std::mutex step_mu;  // one step at a time
};

namespace {

double level_dist(const icp_server* s, const Req* r, int l) {
  if (s->cfg.corr_dist[l] > 0.0) return s->cfg.corr_dist[l];
  return s->cfg.corr_factor * std::max(s->cfg.voxel[l], r->spacing);
}

// (mu held) posts a completion and releases all of the request's memory
void complete(icp_server* s, Req* r, int error, const icp_result_t* res) {
  icp_completion_t c{};
  c.ticket = r->ticket;
  c.user_tag = r->tag;
  if (res) c.result = *res;
  c.result.n_iter = r->iters_total;
  c.error = error;
  c.t_submit_ns = r->t_submit;
  c.t_admit_ns = r->t_admit;
  c.t_done_ns = now_ns();
  s->pool.release(r->prep_mem, r->prep_bytes);
  if (r->lvl_mem) s->pool.release(r->lvl_mem, r->lvl_bytes);
  if (r->src) s->pool.release(r->src, r->in_bytes);
  s->pending.erase(r->ticket);
  s->done.push_back(c);
  delete r;
  s->cv_done.notify_all();
}

// Allocates a request's device input copy in the pool (mu held); false if full.
bool alloc_inputs(icp_server* s, Req* r) {
  char* p = static_cast<char*>(s->pool.alloc(r->in_bytes));
  if (!p) return false;
  r->src = reinterpret_cast<float*>(p);
  r->tgt = reinterpret_cast<float*>(p + align256(12 * (size_t)r->n_src));
  r->tgt_n = reinterpret_cast<float*>(p + align256(12 * (size_t)r->n_src) + align256(12 * (size_t)r->n_tgt));
  return true;
}

size_t input_bytes(int64_t ns, int64_t nt) {
  return align256(12 * (size_t)ns) + 2 * align256(12 * (size_t)nt);
}

// Prepares the given requests for their current level (no locks held; the
// requests are owned by this step).  Requests that cannot get memory now stay
// in kPrep; requests with bad data or an injected fault are returned in
// `failed` with their error code.
int prepare_level(icp_server* s, std::vector<Req*>& list, std::vector<std::pair<Req*, int>>& failed) {
  icp_ctx* c = s->ctx;
  const bool plane = s->cfg.variant == ICP_POINT_TO_PLANE;
  std::vector<Req*> ok;
  // injected faults (failure isolation tests)
  for (Req* r : list) {
    if (s->fault_on && r->tag == s->fault_tag) failed.push_back({r, ICP_E_DEVICE});
    else ok.push_back(r);
  }
  list.swap(ok);
  ok.clear();
  // 1. level clouds: downsampled into pool memory, or the inputs themselves
  std::vector<Req*> ds;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (Req* r : list) {
      const double v = s->cfg.voxel[r->level];
      if (v <= 0.0) {
        r->ls = r->src; r->lt = r->tgt; r->ltn = plane ? r->tgt_n : nullptr;
        r->lns = r->n_src; r->lnt = r->n_tgt;
        ok.push_back(r);
        continue;
      }
      r->lvl_bytes = input_bytes(r->n_src, r->n_tgt);
      char* p = static_cast<char*>(s->pool.alloc(r->lvl_bytes));
      if (!p) continue;  // retry next step
      r->lvl_mem = p;
      r->ls = reinterpret_cast<float*>(p);
      r->lt = reinterpret_cast<float*>(p + align256(12 * (size_t)r->n_src));
      r->ltn = plane ? reinterpret_cast<float*>(p + align256(12 * (size_t)r->n_src) +
                                                align256(12 * (size_t)r->n_tgt))
                     : nullptr;
      ds.push_back(r);
    }
  }
  int rc;
  while (!ds.empty()) {
    std::vector<VoxIn> vin;
    for (Req* r : ds) {
      const double v = s->cfg.voxel[r->level];
      vin.push_back(VoxIn{r->src, nullptr, r->n_src, v, r->ls, nullptr, r->n_src});
      vin.push_back(VoxIn{r->tgt, plane ? r->tgt_n : nullptr, r->n_tgt, v, r->lt, r->ltn, r->n_tgt});
    }
    std::vector<int64_t> cnt(vin.size());
    int bad = -1;
    rc = downsample_clouds(c, (int)vin.size(), vin.data(), cnt.data(), &bad);
    if (rc == ICP_E_NONFINITE && bad >= 0) {
      failed.push_back({ds[bad / 2], ICP_E_NONFINITE});
      ds.erase(ds.begin() + bad / 2);
      continue;
    }
    if (rc) return rc;
    for (size_t k = 0; k < ds.size(); ++k) {
      ds[k]->lns = cnt[2 * k];
      ds[k]->lnt = cnt[2 * k + 1];
      ok.push_back(ds[k]);
    }
    break;
  }
  list.swap(ok);
  // 2. plan all of them (boxes, finiteness, grid sizes)
  Prep P;
  std::vector<PairIn> in;
  for (;;) {
    if (list.empty()) return ICP_SUCCESS;
    in.clear();
    for (Req* r : list)
      in.push_back(PairIn{r->ls, r->lns, r->lt, r->ltn, r->lnt, level_dist(s, r, r->level), true});
    int bad = -1;
    rc = plan_pairs(c, (int)list.size(), in.data(), &P, &bad);
    if (rc == ICP_E_NONFINITE && bad >= 0) {
      failed.push_back({list[bad], ICP_E_NONFINITE});
      list.erase(list.begin() + bad);
      continue;
    }
    if (rc) return rc;
    break;
  }
  // 3. per-request working memory, in list order.  Requests that do not fit
  //    wait for the next step (their level buffers are returned); if nothing
  //    running could free memory, queued requests' inputs are moved to host
  //    memory first; a request that cannot fit even alone fails.
  std::vector<size_t> need(list.size());
  for (size_t k = 0; k < list.size(); ++k) {
    const int64_t tiles = tiles_of(list[k]->lns);
    need[k] = align256(4 * ((size_t)P.g[k].ncell + 1)) + align256(4 * (size_t)occ_words(P.g[k])) +
              2 * align256(16 * (size_t)list[k]->lnt) +
              4 * align256(4 * (size_t)list[k]->lns) + align256(sizeof(double) * kNumSums * tiles) +
              align256(sizeof(IterState));
  }
  size_t fit = 0;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    for (; fit < list.size(); ++fit) {
      Req* r = list[fit];
      r->prep_bytes = need[fit];
      r->prep_mem = s->pool.alloc(r->prep_bytes);
      if (!r->prep_mem) break;
    }
    if (fit == 0) {
      Req* r = list[0];
      const size_t alone = r->in_bytes + r->lvl_bytes + need[0];
      bool running_holds = false;
      for (Req* a : s->active)
        if (a->state == kRun && a->prep_mem) running_holds = true;
      if (alone > s->pool.cap) {
        failed.push_back({r, ICP_E_TOO_LARGE});
        list.erase(list.begin());
        need.erase(need.begin());
      } else if (!running_holds) {
        // evict queued inputs (newest first) until the request fits
        for (auto it = s->queue.rbegin(); it != s->queue.rend() && !r->prep_mem; ++it) {
          Req* q = *it;
          if (!q->src) continue;
          q->h_src.resize(3 * (size_t)q->n_src);
          q->h_tgt.resize(3 * (size_t)q->n_tgt);
          HIP_TRY(hipMemcpy(q->h_src.data(), q->src, 12 * (size_t)q->n_src, hipMemcpyDeviceToHost), "evict");
          HIP_TRY(hipMemcpy(q->h_tgt.data(), q->tgt, 12 * (size_t)q->n_tgt, hipMemcpyDeviceToHost), "evict");
          if (plane) {
            q->h_tn.resize(3 * (size_t)q->n_tgt);
            HIP_TRY(hipMemcpy(q->h_tn.data(), q->tgt_n, 12 * (size_t)q->n_tgt, hipMemcpyDeviceToHost), "evict");
          }
          s->pool.release(q->src, q->in_bytes);
          q->src = q->tgt = q->tgt_n = nullptr;
          r->prep_bytes = need[0];
          r->prep_mem = s->pool.alloc(r->prep_bytes);
        }
        if (r->prep_mem) fit = 1;
      }
    }
    for (size_t k = fit; k < list.size(); ++k) {
      Req* r = list[k];
      if (r->lvl_mem) s->pool.release(r->lvl_mem, r->lvl_bytes);
      r->lvl_mem = nullptr;
      r->ls = r->lt = r->ltn = nullptr;
      r->prep_mem = nullptr;
    }
  }
  if (fit == 0) return ICP_SUCCESS;
  if (fit < P.n) {
    // plan again for the requests that got memory (their grids are unchanged)
    list.resize(fit);
    in.clear();
    for (Req* r : list)
      in.push_back(PairIn{r->ls, r->lns, r->lt, r->ltn, r->lnt, level_dist(s, r, r->level), true});
    int bad = -1;
    if ((rc = plan_pairs(c, (int)list.size(), in.data(), &P, &bad)) != 0) return rc;
  }
  std::vector<PairDst> dst(list.size());
  // 4. build into the requests' memory, then initialise their loop state
  for (size_t k = 0; k < list.size(); ++k) {
    Req* r = list[k];
    char* p = static_cast<char*>(r->prep_mem);
    size_t o = 0;
    auto take = [&](size_t bytes) {
      char* q = p + o;
      o += align256(bytes);
      return q;
    };
    dst[k].cs = reinterpret_cast<uint32_t*>(take(4 * ((size_t)P.g[k].ncell + 1)));
    dst[k].occ = occ_words(P.g[k]) ? reinterpret_cast<uint32_t*>(take(4 * (size_t)occ_words(P.g[k]))) : nullptr;
    dst[k].tp = reinterpret_cast<float4*>(take(16 * (size_t)r->lnt));
    dst[k].tn = reinterpret_cast<float4*>(take(16 * (size_t)r->lnt));
    dst[k].sx = reinterpret_cast<float*>(take(4 * (size_t)r->lns));
    dst[k].sy = reinterpret_cast<float*>(take(4 * (size_t)r->lns));
    dst[k].sz = reinterpret_cast<float*>(take(4 * (size_t)r->lns));
    dst[k].perm = nullptr;
    uint32_t* jprev = reinterpret_cast<uint32_t*>(take(4 * (size_t)r->lns));
    const int64_t tiles = tiles_of(r->lns);
    double* part = reinterpret_cast<double*>(take(sizeof(double) * kNumSums * tiles));
    IterState* st = reinterpret_cast<IterState*>(take(sizeof(IterState)));
    const double rr = level_dist(s, r, r->level);
    PassArgs& a = r->pa;
    memset(&a, 0, sizeof a);
    a.sx = dst[k].sx; a.sy = dst[k].sy; a.sz = dst[k].sz;
    a.sperm = nullptr;
    a.n_src = (int32_t)r->lns;
    a.tp = dst[k].tp;
    a.tn = plane ? dst[k].tn : nullptr;
    a.cs = dst[k].cs;
    a.occ = dst[k].occ;
    a.g = P.g[k];
    a.r2f = (float)(rr * rr);
    a.inv_h2 = (float)(P.g[k].inv_h * P.g[k].inv_h);
    a.n_tgt = (int32_t)r->lnt;
    a.jprev = jprev;
    a.st = st;
    a.part = part;
    a.n_blocks = (int32_t)tiles;
    set_loss(&a, s->cfg.loss, s->cfg.loss_k);
    r->sa = SolveArgs{part, (int32_t)tiles, st, r->lns, s->cfg.iters[r->level], r->rel_tol, 0};
  }
  if ((rc = build_pairs(c, &P, dst.data())) != 0) return rc;
  for (Req* r : list) {
    HIP_TRY(hipMemsetAsync(r->pa.jprev, 0xff, 4 * (size_t)r->lns, c->stream), "memset");
    HIP_TRY(launch_state_init(const_cast<IterState*>(r->pa.st), r->T, c->stream), "state init");
    r->state = kRun;
  }
  return ICP_SUCCESS;
}

// Stops a server after a failed step (mu not held): every queued and running
// request completes with ICP_E_DEVICE and waiters wake up.
void stop_broken(icp_server* s) {
  std::lock_guard<std::mutex> g(s->mu);
  s->broken = true;
  for (Req* r : s->queue) complete(s, r, ICP_E_DEVICE, nullptr);
  s->queue.clear();
  for (Req* r : s->active) complete(s, r, ICP_E_DEVICE, nullptr);
  s->active.clear();
  s->cv_done.notify_all();
}

int server_step_body(icp_server* s, int32_t* n_busy);

// One server step.  Only one step runs at a time (step_mu).  Any failure
// stops the server (stop_broken).
int server_step(icp_server* s, int32_t* n_busy) {
  std::lock_guard<std::mutex> step_lock(s->step_mu);
  if (s->broken) return fail(ICP_E_DEVICE, "server stopped after a device error");
  int rc;
  if (s->fault_step >= 0 && s->step_count == s->fault_step)
    rc = fail(ICP_E_DEVICE, "step failure forced by ICP_FAULT_INJECT_STEP");
  else
    rc = server_step_body(s, n_busy);
  s->step_count += 1;
  if (rc != ICP_SUCCESS) {
    const std::string msg = g_last_error;
    stop_broken(s);
    g_last_error = msg;
  }
  return rc;
}

int server_step_body(icp_server* s, int32_t* n_busy) {
  icp_ctx* c = s->ctx;
  DeviceGuard dg(c->device);
  std::vector<Req*> prep, upload;
  {
    // admission: FIFO while a slot is free and the inputs are (or can be) in device memory
    std::lock_guard<std::mutex> g(s->mu);
    while ((int)s->active.size() < s->cfg.max_slots && !s->queue.empty()) {
      Req* r = s->queue.front();
      if (!r->src) {
        if (!alloc_inputs(s, r)) break;
        upload.push_back(r);
      }
      s->queue.pop_front();
      r->state = kPrep;
      r->t_admit = now_ns();
      s->active.push_back(r);
    }
    for (Req* r : s->active)
      if (r->state == kPrep) prep.push_back(r);
  }
  for (Req* r : upload) {
    HIP_TRY(hipMemcpyAsync(r->src, r->h_src.data(), 12 * (size_t)r->n_src, hipMemcpyHostToDevice, c->stream),
            "upload");
    HIP_TRY(hipMemcpyAsync(r->tgt, r->h_tgt.data(), 12 * (size_t)r->n_tgt, hipMemcpyHostToDevice, c->stream),
            "upload");
    if (!r->h_tn.empty())
      HIP_TRY(hipMemcpyAsync(r->tgt_n, r->h_tn.data(), 12 * (size_t)r->n_tgt, hipMemcpyHostToDevice,
                             c->stream),
              "upload");
  }
  if (!upload.empty()) {
    HIP_TRY(hipStreamSynchronize(c->stream), "sync");
    for (Req* r : upload) {
      r->h_src = std::vector<float>();
      r->h_tgt = std::vector<float>();
      r->h_tn = std::vector<float>();
    }
  }
  int rc;
  std::vector<std::pair<Req*, int>> failed;
  if (!prep.empty() && (rc = prepare_level(s, prep, failed)) != 0) return rc;
  if (!failed.empty()) {
    std::lock_guard<std::mutex> g(s->mu);
    for (auto& f : failed) {
      s->active.erase(std::find(s->active.begin(), s->active.end(), f.first));
      complete(s, f.first, f.second, nullptr);
    }
  }
  // slot table of the running requests
  std::vector<Req*> run;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (Req* r : s->active)
      if (r->state == kRun) run.push_back(r);
  }
  // (the first running request always fits the item table: its tiles are
  // bounded by its memory, which the pool budget bounds)
  if (!run.empty()) {
    char* hh = static_cast<char*>(s->host_table);
    PassArgs* hp = reinterpret_cast<PassArgs*>(hh + s->o_pargs);
    SolveArgs* hs = reinterpret_cast<SolveArgs*>(hh + s->o_sargs);
    uint2* hi = reinterpret_cast<uint2*>(hh + s->o_items);
    int64_t items = 0;
    std::vector<Req*> slot;
    for (Req* r : run) {
      if (items + r->pa.n_blocks > s->items_cap) continue;  // waits for room in the table
      const int b = (int)slot.size();
      hp[b] = r->pa;
      hs[b] = r->sa;
      for (int t = 0; t < r->pa.n_blocks; ++t) hi[items++] = make_uint2((uint32_t)b, (uint32_t)t);
      slot.push_back(r);
    }
    if (slot.empty()) return fail(ICP_E_DEVICE, "slot table: no running request fits the item table");
    char* dd = s->table.as<char>();
    hipStream_t st = c->stream;
    HIP_TRY(hipMemcpyAsync(dd, hh, s->o_items + sizeof(uint2) * (size_t)items, hipMemcpyHostToDevice, st),
            "upload");
    for (size_t k = 0; k < s->nodes.size(); ++k) {
      hipKernelNodeParams& p = s->node_params[k];
      p.gridDim = dim3((unsigned)((k & 1) ? slot.size() : (size_t)items));
      HIP_TRY(hipGraphExecKernelNodeSetParams(s->exec, s->nodes[k], &p), "graph node update");
    }
    HIP_TRY(hipGraphLaunch(s->exec, st), "hipGraphLaunch");
    IterState* dstates = reinterpret_cast<IterState*>(dd + s->o_states);
    HIP_TRY(launch_gather_states(reinterpret_cast<const SolveArgs*>(dd + s->o_sargs), (int)slot.size(),
                                 dstates, st),
            "gather");
    IterState* hst = reinterpret_cast<IterState*>(hh + s->o_states);
    HIP_TRY(hipMemcpyAsync(hst, dstates, sizeof(IterState) * slot.size(), hipMemcpyDeviceToHost, st),
            "readback");
    HIP_TRY(hipStreamSynchronize(st), "sync");
    // retire finished levels and requests
    std::lock_guard<std::mutex> g(s->mu);
    for (size_t b = 0; b < slot.size(); ++b) {
      const IterState& x = hst[b];
      if (!x.done) continue;
      Req* r = slot[b];
      r->iters_total += x.k;
      for (int k = 0; k < 12; ++k) r->T[k] = x.T[k];
      icp_result_t res;
      to_result(x, &res);
      s->pool.release(r->prep_mem, r->prep_bytes);
      r->prep_mem = nullptr;
      if (r->lvl_mem) s->pool.release(r->lvl_mem, r->lvl_bytes);
      r->lvl_mem = nullptr;
      if (x.status == ICP_DEGENERATE || r->level + 1 >= s->cfg.n_levels) {
        s->active.erase(std::find(s->active.begin(), s->active.end(), r));
        complete(s, r, ICP_SUCCESS, &res);
      } else {
        r->level += 1;
        r->state = kPrep;
      }
    }
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (n_busy) *n_busy = (int32_t)(s->queue.size() + s->active.size());
  }
  return ICP_SUCCESS;
}

void worker_loop(icp_server* s) {
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->active.empty(); });
      if (s->stop) return;
    }
    if (server_step(s, nullptr) != ICP_SUCCESS) {
      std::lock_guard<std::mutex> g(s->mu);
      s->cv_done.notify_all();
      return;
    }
  }
}

// Builds the step graph: a chain of iters_per_step (pass, solve) kernel nodes
// over the device slot table.
int build_graph(icp_server* s) {
  char* dd = s->table.as<char>();
  s->d_pargs = reinterpret_cast<const PassArgs*>(dd + s->o_pargs);
  s->d_items = reinterpret_cast<const uint2*>(dd + s->o_items);
  s->d_sargs = reinterpret_cast<const SolveArgs*>(dd + s->o_sargs);
  s->pass_args[0] = &s->d_pargs;
  s->pass_args[1] = &s->d_items;
  s->solve_args[0] = &s->d_sargs;
  HIP_TRY(hipGraphCreate(&s->graph, 0), "hipGraphCreate");
  const int n = 2 * s->cfg.iters_per_step;
  s->nodes.assign(n, nullptr);
  s->node_params.assign(n, hipKernelNodeParams{});
  for (int k = 0; k < n; ++k) {
    hipKernelNodeParams& p = s->node_params[k];
    if (k & 1) {
      batch_solve_node(&p);
      p.kernelParams = s->solve_args;
    } else {
      batch_pass_node(grid_sub(), s->cfg.variant, s->cfg.precision, s->cfg.loss != ICP_LOSS_NONE, &p);
      p.kernelParams = s->pass_args;
    }
    const hipGraphNode_t* dep = k ? &s->nodes[k - 1] : nullptr;
    HIP_TRY(hipGraphAddKernelNode(&s->nodes[k], s->graph, dep, k ? 1 : 0, &p), "hipGraphAddKernelNode");
  }
  HIP_TRY(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  return ICP_SUCCESS;
}

void server_free(icp_server* s) {
  if (s->ctx) {
    DeviceGuard dg(s->ctx->device);
    if (s->ctx->stream) (void)hipStreamSynchronize(s->ctx->stream);
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->pool_mem.release();
    s->table.release();
    if (s->host_table) (void)hipHostFree(s->host_table);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    ctx_free(s->ctx);
    delete s->ctx;
  }
}

}  // namespace

extern "C" {

int icp_server_create(const icp_server_cfg_t* cfg, icp_server_t** out) {
  if (!cfg || !out) return fail(ICP_E_INVALID_ARG, "cfg / out is NULL");
  const icp_server_cfg_t& k = *cfg;
  if (k.max_slots < 1 || k.max_slots > 65535) return fail(ICP_E_INVALID_ARG, "max_slots must be in [1, 65535]");
  if (check_loss(k.loss, k.loss_k) != 0) return ICP_E_INVALID_ARG;
  if (k.n_levels < 1 || k.n_levels > 4) return fail(ICP_E_INVALID_ARG, "n_levels must be in [1, 4]");
  if (k.iters_per_step < 1 || k.iters_per_step > 64)
    return fail(ICP_E_INVALID_ARG, "iters_per_step must be in [1, 64]");
  if (k.hbm_budget_bytes < (1u << 20)) return fail(ICP_E_INVALID_ARG, "hbm_budget_bytes must be >= 1 MiB");
  if (k.variant != ICP_POINT_TO_PLANE && k.variant != ICP_POINT_TO_POINT)
    return fail(ICP_E_INVALID_ARG, "unknown variant");
  if (k.precision != ICP_PREC_F32_KAHAN_F64 && k.precision != ICP_PREC_F64)
    return fail(ICP_E_INVALID_ARG, "unknown precision");
  for (int l = 0; l < k.n_levels; ++l) {
    if (k.iters[l] < 0) return fail(ICP_E_INVALID_ARG, "iters must be >= 0");
    if (!(k.voxel[l] >= 0.0) || !std::isfinite(k.voxel[l])) return fail(ICP_E_INVALID_ARG, "voxel must be finite and >= 0");
    if (!(k.corr_dist[l] >= 0.0) || !std::isfinite(k.corr_dist[l]))
      return fail(ICP_E_INVALID_ARG, "corr_dist must be finite and >= 0");
    if (k.corr_dist[l] == 0.0 && !(k.corr_factor > 0.0 && std::isfinite(k.corr_factor)))
      return fail(ICP_E_INVALID_ARG, "corr_factor must be > 0 when a level has no corr_dist");
  }
  int n_dev = 0;
  HIP_TRY(hipGetDeviceCount(&n_dev), "hipGetDeviceCount");
  if (k.device < 0 || k.device >= n_dev) return fail(ICP_E_INVALID_ARG, "device index out of range");
  icp_server* s = new icp_server();
  s->cfg = k;
  s->ctx = new icp_ctx();
  int rc = ctx_init(s->ctx, k.device, nullptr);
  auto bail = [&](int code) {
    server_free(s);
    delete s;
    return code;
  };
  if (rc) return bail(rc);
  DeviceGuard dg(k.device);
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking)) != hipSuccess)
    return bail(hip_fail(e, "hipStreamCreate"));
  if ((e = s->pool_mem.ensure(k.hbm_budget_bytes)) != hipSuccess) return bail(hip_fail(e, "pool"));
  s->pool.init(s->pool_mem.as<char>(), k.hbm_budget_bytes);
  // slot table: the item list holds every running request's source tiles
  s->items_cap = std::max<int64_t>(1024, (int64_t)(k.hbm_budget_bytes / (24 * (uint64_t)kTile)));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align256(off);
    off = o + bytes;
    return o;
  };
  s->o_pargs = take(sizeof(PassArgs) * k.max_slots);
  s->o_sargs = take(sizeof(SolveArgs) * k.max_slots);
  s->o_items = take(sizeof(uint2) * (size_t)s->items_cap);
  s->o_states = take(sizeof(IterState) * k.max_slots);
  s->table_bytes = align256(off);
  if ((e = s->table.ensure(s->table_bytes)) != hipSuccess) return bail(hip_fail(e, "table"));
  if ((e = hipMemset(s->table.p, 0, s->table_bytes)) != hipSuccess) return bail(hip_fail(e, "memset"));
  if ((e = hipHostMalloc(&s->host_table, s->table_bytes, hipHostMallocDefault)) != hipSuccess)
    return bail(hip_fail(e, "hipHostMalloc"));
  if (const char* f = getenv("ICP_FAULT_INJECT")) {
    s->fault_on = true;
    s->fault_tag = strtoull(f, nullptr, 10);
  }
  if (const char* f = getenv("ICP_FAULT_INJECT_STEP")) s->fault_step = strtoll(f, nullptr, 10);
  if ((rc = build_graph(s)) != 0) return bail(rc);
  if (k.background_thread) s->worker = std::thread(worker_loop, s);
  *out = s;
  return ICP_SUCCESS;
}

int icp_server_submit(icp_server_t* s, const icp_request_t* q, uint64_t* ticket) {
  const int64_t t0 = now_ns();
  if (!s || !q || !ticket) return fail(ICP_E_INVALID_ARG, "server / request / ticket is NULL");
  const bool plane = s->cfg.variant == ICP_POINT_TO_PLANE;
  int rc;
  if (q->host_memory) {
    if (!q->src_xyz || !q->tgt_xyz || q->n_src < 1 || q->n_tgt < 1)
      return fail(ICP_E_INVALID_ARG, "null cloud or point count < 1");
    if (q->n_src > (int64_t)INT32_MAX || q->n_tgt > (int64_t)INT32_MAX)
      return fail(ICP_E_TOO_LARGE, "more than 2^31-1 points");
    if (plane && !q->tgt_normals) return fail(ICP_E_INVALID_ARG, "tgt_normals is NULL (point-to-plane)");
    if ((rc = check_pose(q->T_init, "T_init")) != 0) return rc;
  } else if ((rc = check_common(q->src_xyz, q->n_src, q->tgt_xyz, q->tgt_normals, q->n_tgt, q->T_init,
                                1.0, s->cfg.variant, s->cfg.precision, true)) != 0) {
    return rc;
  }
  if ((rc = check_iteration(0, q->rel_tol)) != 0) return rc;
  if (!(q->spacing >= 0.0) || !std::isfinite(q->spacing)) return fail(ICP_E_INVALID_ARG, "spacing must be finite and >= 0");
  if (q->reserved != 0) return fail(ICP_E_INVALID_ARG, "reserved must be 0");
  for (int l = 0; l < s->cfg.n_levels; ++l)
    if (s->cfg.corr_dist[l] == 0.0 && !(s->cfg.corr_factor * std::max(s->cfg.voxel[l], q->spacing) > 0.0))
      return fail(ICP_E_INVALID_ARG, "level without corr_dist needs voxel > 0 or spacing > 0");
  Req* r = new Req();
  r->n_src = q->n_src;
  r->n_tgt = q->n_tgt;
  for (int k = 0; k < 16; ++k) r->T[k] = q->T_init[k];
  r->rel_tol = q->rel_tol;
  r->spacing = q->spacing;
  r->tag = q->user_tag;
  r->t_submit = t0;
  r->in_bytes = input_bytes(r->n_src, r->n_tgt);
  if (r->in_bytes > s->pool.cap) {
    delete r;
    return fail(ICP_E_TOO_LARGE, "request inputs exceed the server's memory budget");
  }
  bool on_device;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->broken) {
      delete r;
      return fail(ICP_E_DEVICE, "server stopped after a device error");
    }
    on_device = alloc_inputs(s, r);
  }
  DeviceGuard dg(s->ctx->device);
  const hipMemcpyKind kind = q->host_memory ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  hipError_t e = hipSuccess;
  // the copy starts after the work that produces the inputs (submit blocks
  // until its copy is done anyway)
  if (!q->host_memory && q->stream) e = hipStreamSynchronize(static_cast<hipStream_t>(q->stream));
  if (e != hipSuccess) {
  } else if (on_device) {
    e = hipMemcpyAsync(r->src, q->src_xyz, 12 * (size_t)r->n_src, kind, s->copy_stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->tgt, q->tgt_xyz, 12 * (size_t)r->n_tgt, kind, s->copy_stream);
    if (e == hipSuccess && plane)
      e = hipMemcpyAsync(r->tgt_n, q->tgt_normals, 12 * (size_t)r->n_tgt, kind, s->copy_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
  } else {
    // the pool is full for now: keep a host copy until admission
    r->h_src.resize(3 * (size_t)r->n_src);
    r->h_tgt.resize(3 * (size_t)r->n_tgt);
    if (plane) r->h_tn.resize(3 * (size_t)r->n_tgt);
    const hipMemcpyKind hk = q->host_memory ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    e = hipMemcpy(r->h_src.data(), q->src_xyz, 12 * (size_t)r->n_src, hk);
    if (e == hipSuccess) e = hipMemcpy(r->h_tgt.data(), q->tgt_xyz, 12 * (size_t)r->n_tgt, hk);
    if (e == hipSuccess && plane) e = hipMemcpy(r->h_tn.data(), q->tgt_normals, 12 * (size_t)r->n_tgt, hk);
  }
  std::lock_guard<std::mutex> g(s->mu);
  if (e != hipSuccess) {
    if (r->src) s->pool.release(r->src, r->in_bytes);
    delete r;
    return hip_fail(e, "copy request");
  }
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->pending[r->ticket] = 1;
  s->queue.push_back(r);
  s->cv_work.notify_one();
  return ICP_SUCCESS;
}

int icp_server_step(icp_server_t* s, int32_t* n_busy) {
  if (!s) return fail(ICP_E_INVALID_ARG, "server is NULL");
  if (s->cfg.background_thread) {
    if (n_busy) {
      std::lock_guard<std::mutex> g(s->mu);
      *n_busy = (int32_t)(s->queue.size() + s->active.size());
    }
    return ICP_SUCCESS;
  }
  return server_step(s, n_busy);
}

int icp_server_poll(icp_server_t* s, icp_completion_t* out, int32_t cap, int32_t* n_out) {
  if (!s || !n_out || (cap > 0 && !out)) return fail(ICP_E_INVALID_ARG, "bad poll arguments");
  std::lock_guard<std::mutex> g(s->mu);
  int32_t n = 0;
  while (n < cap && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = n;
  return ICP_SUCCESS;
}

int icp_server_wait(icp_server_t* s, uint64_t ticket, icp_completion_t* out) {
  if (!s || !out) return fail(ICP_E_INVALID_ARG, "server / out is NULL");
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (auto it = s->done.begin(); it != s->done.end(); ++it)
        if (it->ticket == ticket) {
          *out = *it;
          s->done.erase(it);
          return ICP_SUCCESS;
        }
      if (!s->pending.count(ticket)) return fail(ICP_E_NOT_FOUND, "unknown or already delivered ticket");
      if (s->broken) return fail(ICP_E_DEVICE, "server stopped after a device error");
      if (s->cfg.background_thread) {
        s->cv_done.wait_for(lk, std::chrono::milliseconds(50));
        continue;
      }
    }
    int rc = server_step(s, nullptr);
    if (rc) return rc;
  }
}

int icp_server_destroy(icp_server_t* s) {
  if (!s) return ICP_SUCCESS;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  {
    std::lock_guard<std::mutex> step_lock(s->step_mu);
    std::lock_guard<std::mutex> g(s->mu);
    for (Req* r : s->queue) complete(s, r, ICP_E_CANCELLED, nullptr);
    s->queue.clear();
    for (Req* r : s->active) complete(s, r, ICP_E_CANCELLED, nullptr);
    s->active.clear();
  }
  server_free(s);
  delete s;
  return ICP_SUCCESS;
}

}  // extern "C"
