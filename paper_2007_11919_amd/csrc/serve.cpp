// Serving: continuous batching of embed requests over resident models.
//
// A worker thread owns one HIP stream and a ring of step slots.  Each step
// takes row tiles (BM rows) from the admitted requests of one precision,
// oldest request first, writes the tile table into the slot's pinned
// buffer and replays the slot's captured graph: a copy of the table to the
// device followed by the persistent fused embed kernel.  While up to
// `kSlots` steps are on the device the worker keeps admitting queued
// requests (by slot count and bytes), so new work overlaps running work.
// A request completes when the step holding its last tile completes.
//
// The kernel runs exactly the per-tile code of mds_embed, so a row gives the
// same bits alone and in any mix.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mds_internal.h"

namespace mds {
const Model* model_of(const mds_model* h);
}  // namespace mds

using namespace mds;

namespace {

constexpr int kSlots = 3;          // steps that may be in flight at once
constexpr int kModes = 3;          // FP32, split BF16, split FP16
constexpr int kRbc = kEmbedClasses;  // kernel classes: r <= 16, <= 32, <= 64, two wide split
constexpr int kGraphs = kModes * kRbc;
constexpr int kMaxModels = 1024;
constexpr int kDefaultTiles = 2048;

int mode_index(int mode) { return mode == MODE_F32 ? 0 : (mode == MODE_BF16 ? 1 : 2); }
int mode_of_index(int i) { return i == 0 ? MODE_F32 : (i == 1 ? MODE_BF16 : MODE_F16); }

struct Request {
  int32_t model = 0;
  int mode = MODE_F32;
  int rbc = 0;
  const void* x = nullptr;
  void* y = nullptr;
  int64_t n = 0, ldx = 0, ldy = 0;
  int64_t bytes = 0;
  int64_t ntiles = 0, next_tile = 0, tiles_done = 0;
  int32_t state = 0;  // 0 queued, 1 admitted, 2 done
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct StepHeader {
  int32_t nwork;
  int32_t pad[15];  // keeps the tile table 64-byte aligned
};

struct Slot {
  char* host = nullptr;   // pinned: StepHeader + TileWork[cap]
  char* dev = nullptr;    // device copy
  hipEvent_t done = nullptr;
  hipGraphExec_t exec[kGraphs] = {};
  hipGraph_t graph[kGraphs] = {};
  bool busy = false;
  std::vector<std::pair<int64_t, int64_t>> parts;  // (ticket, tiles in this step)
  int64_t rows = 0;
};

}  // namespace

struct mds_server {
  int64_t budget = 0;
  int64_t bytes_in_use = 0;
  int32_t max_slots = 1;
  int32_t tiles_cap = kDefaultTiles;
  int grid = 0;
  hipStream_t stream = nullptr;
  int dev = 0;
  EmbedModelView* views_dev[kModes] = {nullptr, nullptr, nullptr};
  std::vector<const Model*> models;
  Slot slots[kSlots];
  int next_slot = 0;

  std::mutex mu;
  std::condition_variable cv_work;  // worker waits for submissions
  std::condition_variable cv_done;  // waiters wait for completions
  std::deque<int64_t> queue;
  std::vector<int64_t> active;  // admitted, tiles left to schedule (oldest first)
  std::unordered_map<int64_t, Request> reqs;
  int64_t next_ticket = 1;
  int64_t n_admitted_live = 0;  // admitted and not done
  mds_serve_stats_t stats{};
  bool stop = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  hipError_t worker_error = hipSuccess;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

size_t slot_bytes(int cap) { return sizeof(StepHeader) + sizeof(TileWork) * (size_t)cap; }

// Retire the oldest busy slot (blocking on its event).
void retire(mds_server* s, Slot& sl) {
  hipError_t e = hipEventSynchronize(sl.done);
  std::lock_guard<std::mutex> lk(s->mu);
  if (e != hipSuccess && s->worker_error == hipSuccess) s->worker_error = e;
  const double t = s->now();
  for (auto& pr : sl.parts) {
    auto it = s->reqs.find(pr.first);
    if (it == s->reqs.end()) continue;
    Request& rq = it->second;
    rq.tiles_done += pr.second;
    if (rq.tiles_done >= rq.ntiles && rq.state != 2) {
      rq.state = 2;
      rq.t_done = t;
      s->bytes_in_use -= rq.bytes;
      s->n_admitted_live -= 1;
      s->stats.completed += 1;
      s->stats.points += rq.n;
    }
  }
  sl.parts.clear();
  sl.busy = false;
  s->cv_done.notify_all();
}

// Admit queued requests while slots and bytes allow (caller holds the lock).
void admit_locked(mds_server* s) {
  const double t = s->now();
  while (!s->queue.empty()) {
    Request& rq = s->reqs[s->queue.front()];
    if (s->n_admitted_live >= s->max_slots) break;
    if (s->bytes_in_use + rq.bytes > s->budget) break;
    rq.state = 1;
    rq.t_admit = t;
    s->bytes_in_use += rq.bytes;
    s->n_admitted_live += 1;
    s->stats.admitted += 1;
    if (rq.n == 0) {  // nothing to compute
      rq.state = 2;
      rq.t_done = t;
      s->bytes_in_use -= rq.bytes;
      s->n_admitted_live -= 1;
      s->stats.completed += 1;
    } else {
      s->active.push_back(s->queue.front());
    }
    s->queue.pop_front();
  }
}

// Fill slot `sl` with tiles of one precision and column-block class, taken
// from the oldest request onward (caller holds the lock).  Returns false if
// there is nothing to run.
bool build_step_locked(mds_server* s, Slot& sl, int* graph_out) {
  if (s->active.empty()) return false;
  const int mode = s->reqs[s->active.front()].mode;
  const int rbc = s->reqs[s->active.front()].rbc;
  StepHeader* hdr = reinterpret_cast<StepHeader*>(sl.host);
  TileWork* tw = reinterpret_cast<TileWork*>(sl.host + sizeof(StepHeader));
  int nw = 0;
  sl.parts.clear();
  sl.rows = 0;
  for (size_t a = 0; a < s->active.size() && nw < s->tiles_cap; ++a) {
    Request& rq = s->reqs[s->active[a]];
    if (rq.mode != mode || rq.rbc != rbc) continue;
    int64_t took = 0;
    while (rq.next_tile < rq.ntiles && nw < s->tiles_cap) {
      const int64_t row0 = rq.next_tile * BM;
      TileWork& w = tw[nw++];
      w.x = rq.x;
      w.y = rq.y;
      w.ldx = rq.ldx;
      w.ldy = rq.ldy;
      w.row0 = row0;
      w.nrows = (int32_t)std::min<int64_t>(BM, rq.n - row0);
      w.model = rq.model;
      rq.next_tile += 1;
      took += 1;
      sl.rows += w.nrows;
    }
    if (took) sl.parts.emplace_back(s->active[a], took);
  }
  // drop fully scheduled requests from the active list
  s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                 [s](int64_t t) {
                                   const Request& rq = s->reqs[t];
                                   return rq.next_tile >= rq.ntiles;
                                 }),
                  s->active.end());
  hdr->nwork = nw;
  *graph_out = mode_index(mode) * kRbc + rbc;
  s->stats.steps += 1;
  s->stats.tiles += nw;
  return nw > 0;
}

void worker_main(mds_server* s) {
  (void)hipSetDevice(s->dev);
  for (;;) {
    // retire the slot we are about to reuse
    Slot& sl = s->slots[s->next_slot];
    if (sl.busy) retire(s, sl);
    int gi = 0;
    bool have = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      admit_locked(s);
      have = build_step_locked(s, sl, &gi);
      if (!have) {
        // nothing new to launch: retire in-flight steps, then sleep
        bool any_busy = false;
        for (auto& o : s->slots) any_busy |= o.busy;
        if (!any_busy) {
          if (s->stop && s->queue.empty() && s->active.empty()) return;
          s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
          continue;
        }
      }
    }
    if (!have) {
      // wait for the oldest busy step to free memory / slots
      for (int k = 1; k <= kSlots; ++k) {
        Slot& o = s->slots[(s->next_slot + k) % kSlots];
        if (o.busy) {
          retire(s, o);
          break;
        }
      }
      continue;
    }
    hipError_t e = hipGraphLaunch(sl.exec[gi], s->stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, s->stream);
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->worker_error == hipSuccess) s->worker_error = e;
    }
    sl.busy = true;
    s->next_slot = (s->next_slot + 1) % kSlots;
  }
}

mds_status capture_graphs(mds_server* s) {
  for (int mi = 0; mi < kModes; ++mi)
    for (int rbc = 0; rbc < kRbc; ++rbc) {
      if (mode_of_index(mi) == MODE_F32 && rbc == kWideHiClass) continue;  // no such launch
      mds_status st = prepare_embed_worklist(mode_of_index(mi), rbc);
      if (st != MDS_OK) return st;
    }
  for (int k = 0; k < kSlots; ++k) {
    Slot& sl = s->slots[k];
    for (int gi = 0; gi < kGraphs; ++gi) {
      const int mi = gi / kRbc, rbc = gi % kRbc;
      if (mode_of_index(mi) == MODE_F32 && rbc == kWideHiClass) continue;
      MDS_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipMemcpyAsync(sl.dev, sl.host, slot_bytes(s->tiles_cap), hipMemcpyHostToDevice,
                                    s->stream);
      mds_status st = MDS_OK;
      if (e == hipSuccess) {
        const StepHeader* hdr = reinterpret_cast<const StepHeader*>(sl.dev);
        const TileWork* tw = reinterpret_cast<const TileWork*>(sl.dev + sizeof(StepHeader));
        st = launch_embed_worklist(mode_of_index(mi), rbc, s->views_dev[mi], tw, &hdr->nwork, 0,
                                   s->stream);
      }
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(s->stream, &g);
      if (e != hipSuccess) return hip_fail(e, "capture memcpy");
      if (st != MDS_OK) return st;
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      sl.graph[gi] = g;
      MDS_HIP(hipGraphInstantiate(&sl.exec[gi], g, nullptr, nullptr, 0));
    }
  }
  return MDS_OK;
}

void destroy_server(mds_server* s) {
  for (auto& sl : s->slots) {
    for (int gi = 0; gi < kGraphs; ++gi) {
      if (sl.exec[gi]) (void)hipGraphExecDestroy(sl.exec[gi]);
      if (sl.graph[gi]) (void)hipGraphDestroy(sl.graph[gi]);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
  }
  for (auto* v : s->views_dev)
    if (v) (void)hipFree(v);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

mds_status mds_serve_create(int64_t budget_bytes, int32_t max_slots, int32_t tiles_per_step,
                            mds_server** out) {
  if (!out) return set_error(MDS_ERR_INVALID_ARG, "out is NULL");
  if (budget_bytes <= 0) return set_error(MDS_ERR_INVALID_ARG, "budget_bytes must be > 0");
  if (max_slots < 1 || max_slots > 65536) return set_error(MDS_ERR_INVALID_ARG, "max_slots out of range");
  if (tiles_per_step < 0 || tiles_per_step > (1 << 20))
    return set_error(MDS_ERR_INVALID_ARG, "tiles_per_step out of range");
  mds_server* s = new (std::nothrow) mds_server();
  if (!s) return set_error(MDS_ERR_OOM, "host allocation failed");
  s->budget = budget_bytes;
  s->max_slots = max_slots;
  s->tiles_cap = tiles_per_step ? tiles_per_step : kDefaultTiles;
  s->stats.budget_bytes = budget_bytes;
  hipError_t e = hipGetDevice(&s->dev);
  int ncu = 256;
  hipDeviceProp_t prop;
  if (e == hipSuccess && hipGetDeviceProperties(&prop, s->dev) == hipSuccess && prop.multiProcessorCount > 0)
    ncu = prop.multiProcessorCount;
  (void)ncu;
  mds_status st = MDS_OK;
  do {
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess) {
      st = hip_fail(e, "hipStreamCreate");
      break;
    }
    for (int mi = 0; mi < kModes && st == MDS_OK; ++mi) {
      if ((e = hipMalloc(&s->views_dev[mi], sizeof(EmbedModelView) * kMaxModels)) != hipSuccess)
        st = hip_fail(e, "hipMalloc(views)");
    }
    if (st != MDS_OK) break;
    for (auto& sl : s->slots) {
      if ((e = hipHostMalloc(reinterpret_cast<void**>(&sl.host), slot_bytes(s->tiles_cap),
                             hipHostMallocDefault)) != hipSuccess) {
        st = hip_fail(e, "hipHostMalloc(step table)");
        break;
      }
      reinterpret_cast<StepHeader*>(sl.host)->nwork = 0;
      if ((e = hipMalloc(reinterpret_cast<void**>(&sl.dev), slot_bytes(s->tiles_cap))) != hipSuccess) {
        st = hip_fail(e, "hipMalloc(step table)");
        break;
      }
      if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) {
        st = hip_fail(e, "hipEventCreate");
        break;
      }
    }
    if (st != MDS_OK) break;
    st = capture_graphs(s);
  } while (false);
  if (st != MDS_OK) {
    destroy_server(s);
    return st;
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return MDS_OK;
}

mds_status mds_serve_add_model(mds_server* s, const mds_model* h, int32_t* model_id) {
  if (!s || !h || !model_id) return set_error(MDS_ERR_INVALID_ARG, "NULL argument");
  const Model* m = model_of(h);
  std::lock_guard<std::mutex> lk(s->mu);
  if ((int)s->models.size() >= kMaxModels) return set_error(MDS_ERR_BUDGET, "too many models");
  if (m->rb > embed_max_rb()) return set_error(MDS_ERR_INVALID_ARG, "model r too large for serving");
  if (!m->vectors) return set_error(MDS_ERR_INVALID_ARG, "serving needs a model fitted on data rows");
  if (s->bytes_in_use + m->bytes > s->budget)
    return set_error(MDS_ERR_BUDGET, "model does not fit in the byte budget");
  const int id = (int)s->models.size();
  for (int mi = 0; mi < kModes; ++mi) {
    EmbedModelView v = m->view(mode_of_index(mi));
    MDS_HIP(hipMemcpy(s->views_dev[mi] + id, &v, sizeof(v), hipMemcpyHostToDevice));
  }
  s->models.push_back(m);
  s->bytes_in_use += m->bytes;
  s->stats.bytes_in_use = s->bytes_in_use;
  *model_id = id;
  return MDS_OK;
}

mds_status mds_serve_submit(mds_server* s, int32_t model_id, const void* X, int32_t dt, int64_t n_pts,
                            int64_t ldx, int32_t prec, void* Y, int64_t ldy, int64_t* ticket) {
  if (!s || !ticket) return set_error(MDS_ERR_INVALID_ARG, "NULL argument");
  // the serving kernels read X and write Y as float
  if (dt != MDS_F32) return set_error(MDS_ERR_INVALID_ARG, "serving takes float32 rows (MDS_F32)");
  int mode;
  switch (prec) {
    case MDS_PREC_FP32: mode = MODE_F32; break;
    case MDS_PREC_SPLIT_BF16: mode = MODE_BF16; break;
    case MDS_PREC_SPLIT_FP16: mode = MODE_F16; break;
    default: return set_error(MDS_ERR_INVALID_ARG, "serving takes FP32 or split precisions");
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (model_id < 0 || model_id >= (int32_t)s->models.size())
    return set_error(MDS_ERR_NOT_FOUND, "unknown model id");
  const Model* m = s->models[model_id];
  if (n_pts < 0) return set_error(MDS_ERR_INVALID_ARG, "n_pts < 0");
  if (n_pts > 0 && (!X || !Y)) return set_error(MDS_ERR_INVALID_ARG, "X or Y is NULL");
  if (ldx < m->p || ldy < m->r) return set_error(MDS_ERR_INVALID_ARG, "ldx < p or ldy < r");
  Request rq;
  rq.model = model_id;
  rq.mode = mode;
  rq.rbc = embed_class(mode, m->p, m->rb, m->l_pad, mode == MODE_BF16 ? m->bf_lo_zero : m->h_lo_zero);
  rq.x = X;
  rq.y = Y;
  rq.n = n_pts;
  rq.ldx = ldx;
  rq.ldy = ldy;
  rq.bytes = 4 * n_pts * (m->p + m->r);
  int64_t model_bytes = 0;
  for (const Model* mm : s->models) model_bytes += mm->bytes;
  if (rq.bytes > s->budget - model_bytes)
    return set_error(MDS_ERR_BUDGET, "request larger than the budget left after the models");
  rq.ntiles = (n_pts + BM - 1) / BM;
  rq.t_submit = s->now();
  const int64_t t = s->next_ticket++;
  s->reqs.emplace(t, rq);
  s->queue.push_back(t);
  s->stats.submitted += 1;
  *ticket = t;
  s->cv_work.notify_one();
  return MDS_OK;
}

mds_status mds_serve_poll(mds_server* s, int64_t ticket, int32_t* state, double* t_submit,
                          double* t_admit, double* t_done) {
  if (!s) return set_error(MDS_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(MDS_ERR_NOT_FOUND, "unknown ticket");
  if (s->worker_error != hipSuccess) return hip_fail(s->worker_error, "serving step");
  if (state) *state = it->second.state;
  if (t_submit) *t_submit = it->second.t_submit;
  if (t_admit) *t_admit = it->second.t_admit;
  if (t_done) *t_done = it->second.t_done;
  return MDS_OK;
}

mds_status mds_serve_wait(mds_server* s, int64_t ticket, double timeout_s) {
  if (!s) return set_error(MDS_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(MDS_ERR_NOT_FOUND, "unknown ticket");
  auto pred = [&] { return s->reqs[ticket].state == 2 || s->worker_error != hipSuccess; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    return set_error(MDS_ERR_STATE, "timed out waiting for the ticket");
  }
  if (s->worker_error != hipSuccess) return hip_fail(s->worker_error, "serving step");
  return MDS_OK;
}

mds_status mds_serve_stats(mds_server* s, mds_serve_stats_t* out) {
  if (!s || !out) return set_error(MDS_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->queued = (int64_t)s->queue.size();
  out->in_flight = s->n_admitted_live;
  out->bytes_in_use = s->bytes_in_use;
  out->budget_bytes = s->budget;
  return MDS_OK;
}

double mds_serve_now(mds_server* s) { return s ? s->now() : 0.0; }

void mds_serve_destroy(mds_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipStreamSynchronize(s->stream);
  destroy_server(s);
}

}  // extern "C"
