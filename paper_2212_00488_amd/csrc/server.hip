// Serving runtime of the integer path: a persistent worker thread takes
// stereo frames of mixed shapes as they are submitted, keeps per-(shape,
// batch size, slot) device buffers, plans and captured HIP graphs resident,
// admits frames in arrival order while a slot (a stream of its own) is free
// and the cost-volume budget of the frames in flight allows, merging the
// oldest pending frame with later pending frames of its shape into one
// batched launch, and returns each result with its submit / admit / done
// times.  Frames in different slots overlap on the device; no two in-flight
// launches share scratch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "context.h"
#include "pipeline.h"
#include "stereo.h"

using namespace stereo_host;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  const uint8_t* left;
  const uint8_t* right;
  int16_t* out;
  int W, H, Dmax;
  uint64_t tag;
  size_t volume;  // X * Y * D * 4 bytes: the admission measure
  bool direct = false;  // out is page-locked: the map is copied into it directly
  Clock::time_point t_submit, t_admit;
};

// Resident state of one shape and batch size nb on one slot: device inputs
// and outputs of nb frames, pinned staging of the outputs, the plan and the
// captured graph of the path over the nb pairs.
struct Exec {
  int nb = 1;
  uint8_t* d_left = nullptr;   // [nb][H][W][3]
  uint8_t* d_right = nullptr;  // [nb][H][W][3]
  int16_t* d_out = nullptr;    // [nb][H][W]
  int16_t* h_out = nullptr;    // pinned [nb][H][W]
  Plan* plan = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

constexpr int kServeMaxBatch = 8;  // frames of one launch (stereo_disparity_batch's pairs)

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<Request> reqs;  // the frames of the launch in flight
  Exec* ex = nullptr;
  std::map<std::tuple<int, int, int, int>, Exec*> execs;  // (W, H, Dmax, nb)
};

}  // namespace

struct stereo_server {
  stereo_server_config cfg{};
  stereo_params params{};
  stereo_ctx* ctx = nullptr;
  std::vector<Slot> slots;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> incoming;          // guarded by mu
  std::deque<stereo_server_result> done; // guarded by mu
  std::deque<Request> pending;           // worker only
  size_t inflight = 0;                   // worker only
  int max_batch = 1;                     // frames of one shape merged into a launch
  bool stop = false;                     // guarded by mu
  std::string err;                       // guarded by mu (errors of the worker)
  std::thread worker;
};

namespace {

double ms_since(const stereo_server* s, Clock::time_point t) {
  return std::chrono::duration<double, std::milli>(t - s->t0).count();
}

// Frees an Exec and its plan (the slot's work with it has completed).
void free_exec(stereo_ctx* c, Exec* e) {
  if (!e) return;
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  if (e->d_left) (void)hipFree(e->d_left);
  if (e->d_right) (void)hipFree(e->d_right);
  if (e->d_out) (void)hipFree(e->d_out);
  if (e->h_out) (void)hipHostFree(e->h_out);
  if (e->plan) {
    if (e->graph) --e->plan->pins;
    drop_plan(c, e->plan);
  }
  delete e;
}

// Builds the resident state of (W, H, Dmax) for batches of nb frames on
// slot i: buffers, a plan of its own and a graph captured from the path's
// launch sequence over the nb pairs on the slot's stream.
int make_exec(stereo_server* s, int i, int W, int H, int Dmax, int nb, Exec** out) {
  Slot& sl = s->slots[i];
  stereo_ctx* c = s->ctx;
  Exec* e = new Exec();
  e->nb = nb;
  const size_t img = (size_t)W * H * 3, omap = (size_t)W * H * 2;
  hipError_t he = hipMalloc(&e->d_left, nb * img);
  if (he == hipSuccess) he = hipMalloc(&e->d_right, nb * img);
  if (he == hipSuccess) he = hipMalloc(&e->d_out, nb * omap);
  if (he == hipSuccess)
    he = hipHostMalloc(reinterpret_cast<void**>(&e->h_out), nb * omap, hipHostMallocDefault);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    free_exec(c, e);
    return fail(c, STEREO_ENOMEM, "server buffers for %d x %dx%d: %s", nb, W, H,
                hipGetErrorString(he));
  }
  // the plan's owner key is unique per (slot, batch size): each Exec has its own
  const void* owner = reinterpret_cast<const char*>(&sl) + nb;
  int rc = get_plan(c, W, H, Dmax, s->params, nb, owner, sl.stream, &e->plan);
  if (rc) {
    e->plan = nullptr;
    free_exec(c, e);
    return rc;
  }
  stereo_dev::PairPtrs pp{};
  for (int k = 0; k < nb; ++k) {
    pp.left[k] = e->d_left + k * img;
    pp.right[k] = e->d_right + k * img;
    pp.out[k] = e->d_out + k * (size_t)W * H;
  }
  he = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
  if (he == hipSuccess) {
    rc = run(c, *e->plan, pp, nb, false, false, sl.stream);
    hipError_t ee = hipStreamEndCapture(sl.stream, &e->graph);
    if (!rc && ee != hipSuccess) rc = fail(c, STEREO_EHIP, "capture: %s", hipGetErrorString(ee));
  } else {
    rc = fail(c, STEREO_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(he));
  }
  if (!rc) {
    he = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
    if (he != hipSuccess) rc = fail(c, STEREO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(he));
  }
  // the graph launches into the plan's memory: the plan must outlive it, so
  // it is pinned against eviction
  if (e->graph) ++e->plan->pins;
  if (rc) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(sl.stream);  // the plan's set-up was enqueued there
    free_exec(c, e);
    return rc;
  }
  *out = e;
  return 0;
}

void post(stereo_server* s, const Request& r, int status, int slot, int batch,
          Clock::time_point t_done) {
  stereo_server_result res{};
  res.tag = r.tag;
  res.status = status;
  res.slot = slot;
  res.batch = batch;
  res.t_submit_ms = ms_since(s, r.t_submit);
  res.t_admit_ms = status ? res.t_submit_ms : ms_since(s, r.t_admit);
  res.t_done_ms = ms_since(s, t_done);
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->done.push_back(res);
  }
  s->cv_done.notify_all();
}

// Starts the frames of `batch` (one shape, at most kServeMaxBatch) on free
// slot i as one launch; returns 0 or an error code (the frames are then
// answered with that status).
int start(stereo_server* s, int i, std::vector<Request>& batch) {
  Slot& sl = s->slots[i];
  const Request& r0 = batch.front();
  const int nb = (int)batch.size();
  auto key = std::make_tuple(r0.W, r0.H, r0.Dmax, nb);
  auto it = sl.execs.find(key);
  Exec* e = nullptr;
  if (it == sl.execs.end()) {
    int rc = make_exec(s, i, r0.W, r0.H, r0.Dmax, nb, &e);
    // out of device memory: free the resident state (graphs, buffers, plans)
    // of idle slots, this one first, and try again
    for (int k = 0; rc == STEREO_ENOMEM && k < (int)s->slots.size(); ++k) {
      Slot& q = s->slots[(i + k) % s->slots.size()];
      if (q.busy || q.execs.empty()) continue;
      (void)hipStreamSynchronize(q.stream);
      for (auto& kv : q.execs) free_exec(s->ctx, kv.second);
      q.execs.clear();
      rc = make_exec(s, i, r0.W, r0.H, r0.Dmax, nb, &e);
    }
    if (rc) return rc;
    sl.execs[key] = e;
  } else {
    e = it->second;
  }
  const size_t img = (size_t)r0.W * r0.H * 3, omap = (size_t)r0.W * r0.H * 2;
  hipError_t he = hipSuccess;
  for (int k = 0; k < nb && he == hipSuccess; ++k) {
    he = hipMemcpyAsync(e->d_left + k * img, batch[k].left, img, hipMemcpyHostToDevice, sl.stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(e->d_right + k * img, batch[k].right, img, hipMemcpyHostToDevice,
                          sl.stream);
  }
  if (he == hipSuccess) he = hipGraphLaunch(e->exec, sl.stream);
  // a page-locked output buffer takes its map by DMA; pageable memory goes
  // through the slot's pinned staging and a host copy on completion
  for (int k = 0; k < nb && he == hipSuccess; ++k) {
    Request& r = batch[k];
    hipPointerAttribute_t at{};
    r.direct = hipPointerGetAttributes(&at, r.out) == hipSuccess && at.type == hipMemoryTypeHost;
    (void)hipGetLastError();  // the query fails for pageable memory; not an error here
    he = hipMemcpyAsync(r.direct ? (void*)r.out : (void*)(e->h_out + k * (size_t)r.W * r.H),
                        e->d_out + k * (size_t)r.W * r.H, omap, hipMemcpyDeviceToHost, sl.stream);
  }
  if (he == hipSuccess) he = hipEventRecord(sl.done, sl.stream);
  if (he != hipSuccess) return fail(s->ctx, STEREO_EHIP, "enqueue: %s", hipGetErrorString(he));
  const Clock::time_point now = Clock::now();
  for (Request& r : batch) r.t_admit = now;
  sl.busy = true;
  sl.reqs = batch;
  sl.ex = e;
  return 0;
}

// Largest power of two <= n (batch sizes 1, 2, 4, 8 keep the resident graphs
// per shape and slot few).
int pow2_floor(int n) {
  int b = 1;
  while (2 * b <= n) b *= 2;
  return b;
}

void worker_main(stereo_server* s) {
  (void)hipSetDevice(s->cfg.device);
  for (;;) {
    {
      std::unique_lock<std::mutex> g(s->mu);
      bool any_busy = false;
      for (const Slot& sl : s->slots) any_busy |= sl.busy;
      if (s->incoming.empty() && s->pending.empty() && !any_busy) {
        if (s->stop) return;
        s->cv_work.wait(g, [&] { return s->stop || !s->incoming.empty(); });
        if (s->stop && s->incoming.empty()) return;
      }
      while (!s->incoming.empty()) {
        s->pending.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
    }
    bool progressed = false;
    // completions
    for (int i = 0; i < (int)s->slots.size(); ++i) {
      Slot& sl = s->slots[i];
      if (!sl.busy) continue;
      hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      int status = 0;
      if (q != hipSuccess) {
        status = STEREO_EHIP;
        std::lock_guard<std::mutex> g(s->mu);
        s->err = hipGetErrorString(q);
      }
      const Clock::time_point now = Clock::now();
      const int nb = (int)sl.reqs.size();
      for (int k = 0; k < nb; ++k) {
        const Request& r = sl.reqs[k];
        const size_t px = (size_t)r.W * r.H;
        if (!status && !r.direct) std::memcpy(r.out, sl.ex->h_out + k * px, px * 2);
        s->inflight -= r.volume;
        post(s, r, status, i, nb, now);
      }
      sl.busy = false;
      sl.reqs.clear();
      progressed = true;
    }
    // admission in arrival order: the oldest pending frame goes to a free
    // slot when the budget has room (a frame alone in flight is always
    // admitted), together with the next pending frames of its shape that the
    // budget also admits, up to max_batch, as one batched launch
    while (!s->pending.empty()) {
      const Request& head = s->pending.front();
      int free_slot = -1;
      for (int i = 0; i < (int)s->slots.size() && free_slot < 0; ++i)
        if (!s->slots[i].busy) free_slot = i;
      if (free_slot < 0) break;
      const uint64_t budget = s->cfg.mem_budget;
      if (budget && s->inflight > 0 && s->inflight + head.volume > budget) break;
      std::vector<size_t> pick{0};
      size_t vol = head.volume;
      for (size_t k = 1; k < s->pending.size() && (int)pick.size() < s->max_batch; ++k) {
        const Request& r = s->pending[k];
        if (r.W != head.W || r.H != head.H || r.Dmax != head.Dmax) continue;
        if (budget && s->inflight + vol + r.volume > budget) break;
        pick.push_back(k);
        vol += r.volume;
      }
      pick.resize(pow2_floor((int)pick.size()));
      std::vector<Request> batch;
      vol = 0;
      for (size_t k : pick) {
        batch.push_back(s->pending[k]);
        vol += s->pending[k].volume;
      }
      for (size_t n = pick.size(); n-- > 0;) s->pending.erase(s->pending.begin() + pick[n]);
      int rc = start(s, free_slot, batch);
      if (rc) {
        {
          std::lock_guard<std::mutex> g(s->mu);
          s->err = s->ctx->err;
        }
        for (const Request& r : batch) post(s, r, rc, -1, (int)batch.size(), Clock::now());
      } else {
        s->inflight += vol;
      }
      progressed = true;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

void stereo_server_default_config(stereo_server_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->size = sizeof(stereo_server_config);
  cfg->device = 0;
  cfg->slots = 4;
  cfg->mem_budget = 0;
  stereo_default_params(&cfg->params);
  cfg->max_batch = kServeMaxBatch;
}

int stereo_server_create(stereo_server** out, const stereo_server_config* cfg) {
  if (!out || !cfg) return STEREO_EINVAL;
  *out = nullptr;
  if (cfg->size != sizeof(stereo_server_config) || cfg->slots < 1 || cfg->slots > 16 ||
      cfg->max_batch < 1 || cfg->max_batch > kServeMaxBatch)
    return STEREO_EINVAL;
  stereo_ctx* c = nullptr;
  int rc = stereo_create(&c, cfg->device, 0);
  if (rc) return rc;
  stereo_params p;
  rc = common_checks(c, 2, 2, 1, &cfg->params, &p);
  if (rc) {
    stereo_destroy(c);
    return rc;
  }
  stereo_server* s = new stereo_server();
  s->cfg = *cfg;
  s->max_batch = cfg->max_batch;
  s->params = p;
  s->params.flags = 0;
  s->ctx = c;
  s->slots.resize(cfg->slots);
  for (Slot& sl : s->slots) {
    // default-priority streams and events without timing
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      for (Slot& q : s->slots) {
        if (q.stream) (void)hipStreamDestroy(q.stream);
        if (q.done) (void)hipEventDestroy(q.done);
      }
      stereo_destroy(c);
      delete s;
      return STEREO_EHIP;
    }
  }
  s->t0 = Clock::now();
  s->worker = std::thread(worker_main, s);
  *out = s;
  return 0;
}

int stereo_server_submit(stereo_server* s, const uint8_t* left, const uint8_t* right, int W, int H,
                         int Dmax, int16_t* out, uint64_t tag) {
  if (!s) return STEREO_EINVAL;
  if (!left || !right || !out) return STEREO_EINVAL;
  if (W < 2 || H < 2 || W > STEREO_MAX_SIDE || H > STEREO_MAX_SIDE || Dmax < 1 || Dmax > W ||
      Dmax > STEREO_MAX_DMAX)
    return STEREO_EINVAL;
  Request r{};
  r.left = left;
  r.right = right;
  r.out = out;
  r.W = W;
  r.H = H;
  r.Dmax = Dmax;
  r.tag = tag;
  r.volume = (size_t)((W + 1) / 2) * ((H + 1) / 2) * ((Dmax + 1) / 2) * 4;
  r.t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return STEREO_EINVAL;
    s->incoming.push_back(r);
  }
  s->cv_work.notify_one();
  return 0;
}

int stereo_server_poll(stereo_server* s, stereo_server_result* res, int max, int timeout_ms) {
  if (!s || !res || max < 1) return STEREO_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  if (s->done.empty() && timeout_ms > 0)
    s->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), [&] { return !s->done.empty(); });
  int n = 0;
  while (n < max && !s->done.empty()) {
    res[n++] = s->done.front();
    s->done.pop_front();
  }
  return n;
}

const char* stereo_server_last_error(stereo_server* s) {
  if (!s) return "null server";
  std::lock_guard<std::mutex> g(s->mu);
  thread_local std::string copy;
  copy = s->err;
  return copy.c_str();
}

void stereo_server_destroy(stereo_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->cfg.device);
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    for (auto& kv : sl.execs) free_exec(s->ctx, kv.second);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  stereo_destroy(s->ctx);
  delete s;
}

}  // extern "C"
