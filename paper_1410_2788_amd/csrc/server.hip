// Request loop of the NPB library: molecules of different sizes arrive at
// any time and are solved with continuous batching.  A request is admitted
// (arrival order) as soon as a workspace for it fits into a free region of
// the device arena the server owns and fewer than max_batch requests are
// active; it joins the running launches at the next tick boundary (a few
// pseudo-time steps), and it leaves, reporting its result and returning its
// arena region, as soon as its own last step is done, while the others keep
// stepping.  Each result equals the single solve of the same request bit for
// bit: every run of every request is swept with the arithmetic of its
// single solve, only the launches are shared.
//
// One worker thread per server drives the device through its own contexts
// and stream; submit / poll / stats may be called from any thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "npb.h"
#include "npb_internal.h"

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// pseudo-time steps per tick: the granularity at which requests join
constexpr int kTickSteps = 4;

struct Request {
  std::vector<double> xyz, q, radius;  // copies taken at submit
  npb_molecule mol{};
  npb_grid grid{};
  npb_params params{};
  size_t ws_bytes = 0;
  size_t ws_off = 0;
  double t_submit = 0.0, t_done = 0.0;
  bool done = false;
  npb_status status = NPB_OK;
  npb_result res{};
};

// First-fit allocator of 256-byte aligned regions of the arena; freed
// regions merge with free neighbours.
struct Arena {
  std::map<size_t, size_t> free;  // offset -> bytes
  void reset(size_t bytes) {
    free.clear();
    free[0] = bytes;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t noff = it->first + bytes;
      free.erase(it);
      if (rest) free[noff] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    auto it = free.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

}  // namespace

struct npb_server {
  int device = 0;
  npb_ctx* tuned = nullptr;  // launch shapes the engines copy
  hipStream_t stream = nullptr;
  unsigned char* arena = nullptr;
  size_t arena_bytes = 0;
  int max_batch = 0;
  size_t max_queue = 0;

  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;  // node-based: references stay valid
  std::vector<double> latency_s;               // submit -> done, since the last reset
  npb_server_stats st{};
  Arena free_regions;
  int active = 0;
  std::thread worker;

  void run();
};

void npb_server::run() {
  (void)hipSetDevice(device);
  // one engine per precision, created on first use
  std::unique_ptr<npb::RollingEngine> eng[3];
  std::vector<npb::RollingDone> done;
  std::vector<Request*> admitted;
  double busy_from = -1.0;
  for (;;) {
    admitted.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      if (active == 0) {
        if (busy_from >= 0.0) {
          st.busy_ms += (now_s() - busy_from) * 1e3;
          busy_from = -1.0;
        }
        cv.wait(lk, [&] { return stop || !queue.empty(); });
        if (stop && queue.empty()) return;
      }
      // admission in arrival order: while a region of the arena holds the
      // request's workspace and fewer than max_batch requests are active
      while (!queue.empty() && active < max_batch) {
        Request& r = reqs.at(queue.front());
        size_t off = 0;
        if (!free_regions.alloc(r.ws_bytes, &off)) break;
        r.ws_off = off;
        admitted.push_back(&r);
        queue.pop_front();
        active += 1;
      }
    }
    if (busy_from < 0.0) busy_from = now_s();
    for (Request* r : admitted) {
      const int prec = r->params.precision;
      npb_status s = NPB_OK;
      if (!eng[prec]) {
        npb::RollingEngine* e = nullptr;
        s = npb::rolling_create(tuned, prec, stream, max_batch, &e);
        eng[prec].reset(e);
      }
      if (s == NPB_OK)
        s = eng[prec]->add(reinterpret_cast<uint64_t>(r), &r->mol, &r->grid, &r->params,
                           arena + r->ws_off, r->ws_bytes);
      if (s != NPB_OK) {
        std::lock_guard<std::mutex> lk(mu);
        r->status = s;
        r->done = true;
        r->t_done = now_s();
        latency_s.push_back(r->t_done - r->t_submit);
        st.failed += 1;
        free_regions.release(r->ws_off, r->ws_bytes);
        active -= 1;
      }
    }
    // one tick of every engine with problems; then whatever has finished
    done.clear();
    bool stepping = false;
    for (auto& e : eng) {
      if (!e || e->active() == 0) continue;
      const npb_status ts = e->tick(kTickSteps);
      // a failed enqueue ends every request of this engine with its status
      if (ts != NPB_OK) e->abort_all(ts, done);
      stepping = stepping || e->stepping() > 0;
      std::lock_guard<std::mutex> lk(mu);
      st.batches += 1;
    }
    for (auto& e : eng) {
      if (!e) continue;
      // nothing left to enqueue: wait for the device before polling
      if (!stepping && e->active() > 0) (void)e->drain();
      e->poll(done);
    }
    if (!done.empty()) {
      std::lock_guard<std::mutex> lk(mu);
      const double t = now_s();
      for (const npb::RollingDone& d : done) {
        Request& r = *reinterpret_cast<Request*>(d.id);
        r.res = d.res;
        r.status = d.status;
        r.t_done = t;
        r.done = true;
        latency_s.push_back(t - r.t_submit);
        if (r.status == NPB_OK)
          st.completed += 1;
        else
          st.failed += 1;
        free_regions.release(r.ws_off, r.ws_bytes);
        active -= 1;
      }
    }
  }
}

extern "C" {

npb_status npb_server_create(npb_ctx* ctx, size_t hbm_budget, int max_batch, int max_queue,
                             npb_server** out) {
  if (!ctx || !out || hbm_budget < 256 || max_batch < 1 || max_queue < 1) return NPB_EINVAL;
  *out = nullptr;
  const int device = npb::ctx_device(ctx);
  npb_server* sv = new (std::nothrow) npb_server();
  if (!sv) return NPB_ENOMEM;
  sv->device = device;
  sv->max_batch = max_batch;
  sv->max_queue = (size_t)max_queue;
  npb_status s = npb_ctx_create(device, &sv->tuned);
  if (s != NPB_OK) {
    delete sv;
    return s;
  }
  npb::copy_tuning(ctx, sv->tuned);
  if (hipSetDevice(device) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
    npb_ctx_destroy(sv->tuned);
    delete sv;
    return NPB_EDEVICE;
  }
  if (hipMalloc(reinterpret_cast<void**>(&sv->arena), hbm_budget) != hipSuccess) {
    (void)hipStreamDestroy(sv->stream);
    npb_ctx_destroy(sv->tuned);
    delete sv;
    return NPB_ENOMEM;
  }
  sv->arena_bytes = hbm_budget;
  sv->free_regions.reset(hbm_budget & ~size_t(255));
  try {
    sv->worker = std::thread([sv] { sv->run(); });
  } catch (...) {
    (void)hipFree(sv->arena);
    (void)hipStreamDestroy(sv->stream);
    npb_ctx_destroy(sv->tuned);
    delete sv;
    return NPB_ENOMEM;
  }
  *out = sv;
  return NPB_OK;
}

npb_status npb_submit(npb_server* sv, const npb_molecule* mol, const npb_grid* grid,
                      const npb_params* params, uint64_t* ticket) {
  if (!sv || !mol || !grid || !params || !ticket) return NPB_EINVAL;
  size_t bytes = 0;
  const npb_status s = npb_workspace_bytes(mol, grid, params, &bytes);  // validates
  if (s != NPB_OK) return s;
  if (align256(bytes) > (sv->arena_bytes & ~size_t(255))) return NPB_EBUSY;  // never fits
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop) return NPB_EINVAL;
  if (sv->queue.size() >= sv->max_queue) {
    sv->st.refused += 1;
    return NPB_EBUSY;
  }
  const uint64_t t = sv->next_ticket++;
  Request& r = sv->reqs[t];
  const int na = mol->n_atoms;
  r.xyz.assign(mol->xyz, mol->xyz + 3 * (size_t)na);
  r.q.assign(mol->q, mol->q + na);
  r.radius.assign(mol->radius, mol->radius + na);
  r.mol.n_atoms = na;
  r.mol.xyz = r.xyz.data();
  r.mol.q = r.q.data();
  r.mol.radius = r.radius.data();
  r.grid = *grid;
  r.params = *params;
  r.ws_bytes = bytes;
  r.t_submit = now_s();
  sv->queue.push_back(t);
  sv->st.submitted += 1;
  *ticket = t;
  sv->cv.notify_one();
  return NPB_OK;
}

npb_status npb_poll(npb_server* sv, uint64_t ticket, npb_result* out, int* done) {
  if (!sv || !out || !done) return NPB_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return NPB_EINVAL;
  if (!it->second.done) {
    *done = 0;
    return NPB_OK;
  }
  *done = 1;
  *out = it->second.res;
  const npb_status s = it->second.status;
  sv->reqs.erase(it);
  return s;
}

npb_status npb_server_get_stats(npb_server* sv, npb_server_stats* out) {
  if (!sv || !out) return NPB_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->st;
  out->queued = (int64_t)sv->queue.size();
  std::vector<double> l = sv->latency_s;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      const size_t k = (size_t)std::min<double>(l.size() - 1, std::ceil(p * l.size()) - 1);
      return l[k] * 1e3;
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
  }
  return NPB_OK;
}

npb_status npb_server_reset_stats(npb_server* sv) {
  if (!sv) return NPB_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  const int64_t queued = sv->st.queued;
  sv->st = npb_server_stats{};
  sv->st.queued = queued;
  sv->latency_s.clear();
  return NPB_OK;
}

void npb_server_destroy(npb_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->device);
  (void)hipStreamSynchronize(sv->stream);
  (void)hipFree(sv->arena);
  (void)hipStreamDestroy(sv->stream);
  npb_ctx_destroy(sv->tuned);
  delete sv;
}

}  // extern "C"
