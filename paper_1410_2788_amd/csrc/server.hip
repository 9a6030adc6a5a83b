// Request loop of the NPB library: molecules of different sizes arrive at
// any time, are admitted by their HBM footprint into a device arena the
// server owns, and are solved together by npb_solve_batch.  Batching is
// continuous: when a batch finishes, the next one is formed from whatever
// is waiting, in arrival order, up to the arena size and the batch limit.
//
// One worker thread per server drives the device through its own context
// and stream; submit / poll / stats may be called from any thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
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

struct Request {
  std::vector<double> xyz, q, radius;  // copies taken at submit
  npb_molecule mol{};
  npb_grid grid{};
  npb_params params{};
  size_t ws_bytes = 0;
  double t_submit = 0.0, t_done = 0.0;
  bool done = false;
  npb_status status = NPB_OK;
  npb_result res{};
};

}  // namespace

struct npb_server {
  int device = 0;
  npb_ctx* ctx = nullptr;  // the worker's own
  hipStream_t stream = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  int max_batch = 0;
  size_t max_queue = 0;

  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;  // node-based: references stay valid
  std::vector<double> latency_s;               // submit -> done, completed requests
  npb_server_stats st{};
  std::thread worker;

  void run();
};

void npb_server::run() {
  (void)hipSetDevice(device);
  std::vector<npb_molecule> mols;
  std::vector<npb_grid> grids;
  std::vector<npb_params> params;
  std::vector<void*> ws;
  std::vector<size_t> wsb;
  std::vector<npb_result> out;
  std::vector<Request*> batch;
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop && queue.empty()) return;
      // admission: arrival order, while the workspaces fit the arena
      size_t used = 0;
      int prec = -1;
      while (!queue.empty() && (int)batch.size() < max_batch) {
        Request& r = reqs.at(queue.front());
        const size_t need = align256(r.ws_bytes);
        if (used + need > arena_bytes) break;
        if (prec >= 0 && r.params.precision != prec) break;
        prec = r.params.precision;
        used += need;
        batch.push_back(&r);
        queue.pop_front();
      }
    }
    const int n = (int)batch.size();
    mols.resize(n);
    grids.resize(n);
    params.resize(n);
    ws.resize(n);
    wsb.resize(n);
    out.assign(n, npb_result{});
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
      mols[i] = batch[i]->mol;
      grids[i] = batch[i]->grid;
      params[i] = batch[i]->params;
      ws[i] = static_cast<unsigned char*>(arena) + off;
      wsb[i] = batch[i]->ws_bytes;
      off += align256(batch[i]->ws_bytes);
    }
    const double t0 = now_s();
    const npb_status s = npb_solve_batch(ctx, n, mols.data(), grids.data(), params.data(),
                                         ws.data(), wsb.data(), nullptr, stream, out.data());
    const double t1 = now_s();
    std::lock_guard<std::mutex> lk(mu);
    st.batches += 1;
    st.busy_ms += (t1 - t0) * 1e3;
    for (int i = 0; i < n; ++i) {
      Request& r = *batch[i];
      r.res = out[i];
      // a batch-level failure fails every request of it; after the solves
      // each request carries its own outcome
      if (s == NPB_OK || s == NPB_EDIVERGED || s == NPB_ERANGE)
        r.status = !out[i].finite ? NPB_EDIVERGED : NPB_OK;
      else
        r.status = s;
      r.t_done = t1;
      r.done = true;
      latency_s.push_back(t1 - r.t_submit);
      if (r.status == NPB_OK)
        st.completed += 1;
      else
        st.failed += 1;
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
  npb_status s = npb_ctx_create(device, &sv->ctx);
  if (s != NPB_OK) {
    delete sv;
    return s;
  }
  // batches differ from one to the next: direct launches, no graph capture
  (void)npb_ctx_set_graph(sv->ctx, 0);
  npb::copy_tuning(ctx, sv->ctx);
  if (hipSetDevice(device) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
    npb_ctx_destroy(sv->ctx);
    delete sv;
    return NPB_EDEVICE;
  }
  if (hipMalloc(&sv->arena, hbm_budget) != hipSuccess) {
    (void)hipStreamDestroy(sv->stream);
    npb_ctx_destroy(sv->ctx);
    delete sv;
    return NPB_ENOMEM;
  }
  sv->arena_bytes = hbm_budget;
  try {
    sv->worker = std::thread([sv] { sv->run(); });
  } catch (...) {
    (void)hipFree(sv->arena);
    (void)hipStreamDestroy(sv->stream);
    npb_ctx_destroy(sv->ctx);
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
  if (align256(bytes) > sv->arena_bytes) return NPB_EBUSY;  // can never be admitted
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
  npb_ctx_destroy(sv->ctx);
  delete sv;
}

}  // extern "C"
