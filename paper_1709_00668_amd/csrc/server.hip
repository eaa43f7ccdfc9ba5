// Serving loop for many resident tensors: updates of uneven batches (dense
// slices or COO nonzeros) arrive as requests; up to `slots` of them run at
// once, each on its own HIP stream driven by its own host thread, so the
// kernels of different updates overlap on the GPU.  Requests are admitted in
// arrival order as slots, staging memory and HBM budget free up: a request
// waits while its tensor has an update in flight (updates of one tensor apply
// in arrival order), and a request whose batch does not fit the free staging
// memory, or whose working set does not fit what the running requests leave
// of the HBM budget, lets later requests of other tensors go first
// (continuous batching at request granularity).  Each admitted batch is
// copied into the server's own device staging pool, so the caller's buffer is
// free once the request has started.
//
// Every update runs the same code and launch shapes as a direct
// sbt_update_batch_* call, and the kernels are deterministic, so a tensor's
// results do not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sambaten.h"
#include "internal.hpp"

namespace {

// first-fit sub-allocator over the staging pool (offsets aligned to 256 B)
class Pool {
 public:
  static size_t round(size_t n) { return (n + 255) / 256 * 256; }
  void init(size_t size) {
    size = size / 256 * 256;
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
  }
  bool alloc(size_t n, size_t* off) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

struct Request {
  uint64_t ticket;
  sbt_tensor* t;
  const void* Y;               // dense batch, or
  const void* coo[4];          // COO batch: i, j, k, v (nnz each)
  int64_t nnz = -1;            // COO entries (-1: dense)
  int64_t K_new;
  size_t bytes;                // staged batch
  size_t need = 0;             // working set charged against the HBM budget
  int state = 0;  // 0 queued, 1 running, 2 done
  sbt_status result = SBT_OK;
  double t_submit = 0, t_start = 0, t_done = 0;
};

}  // namespace

struct sbt_server {
  int slots = 0;
  void* pool_mem = nullptr;
  Pool pool;
  size_t budget = 0;     // HBM budget for the running requests' working sets (0: none)
  size_t charged = 0;    // working sets of the running requests
  std::mutex mu;
  std::condition_variable cv;        // work available / state changed
  std::deque<uint64_t> queue;        // queued tickets in arrival order
  std::unordered_map<uint64_t, Request> reqs;
  std::set<const sbt_tensor*> busy;  // tensors with an update in flight
  uint64_t next_ticket = 1;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // working set of a request: its tensor's update workspace as it stands
  // (COO summaries grow to fit their first updates) and its staged batch
  static size_t working_set(const Request& r) {
    return sbt::update_workspace_bytes(r.t) + Pool::round(r.bytes);
  }

  // first admissible request in arrival order, with its staging offset
  bool pick(uint64_t* ticket, size_t* off) {
    std::set<const sbt_tensor*> blocked;  // keep each tensor's order
    for (auto it = queue.begin(); it != queue.end();) {
      Request& r = reqs[*it];
      if (busy.count(r.t) || blocked.count(r.t)) {
        blocked.insert(r.t);
        ++it;
        continue;
      }
      // (the tensor is idle here: its workspace does not change under us)
      const size_t need = working_set(r);
      if (budget && need > budget) {
        // could never run, even alone: it fails, and its tensor's later
        // requests go on
        r.result = SBT_E_NOMEM;
        r.state = 2;
        r.t_start = r.t_done = now();
        sbt::server_lease(r.t, -1);
        it = queue.erase(it);
        cv.notify_all();
        continue;
      }
      if ((!budget || charged + need <= budget) && pool.alloc(r.bytes, off)) {
        r.need = need;
        charged += need;
        *ticket = *it;
        queue.erase(it);
        return true;
      }
      blocked.insert(r.t);
      ++it;
    }
    return false;
  }

  void work() {
    hipStream_t st = nullptr;
    const bool ok_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
      uint64_t ticket = 0;
      size_t off = 0;
      Request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || pick(&ticket, &off); });
        if (stop && !ticket) break;
        r = &reqs[ticket];
        busy.insert(r->t);
        r->state = 1;
        r->t_start = now();
        ++running;
      }
      sbt_status res = SBT_OK;
      if (!ok_stream) {
        res = SBT_E_DEVICE;
      } else {
        char* stage = (char*)pool_mem + off;
        if (r->nnz < 0) {
          if (hipMemcpyAsync(stage, r->Y, r->bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            res = SBT_E_DEVICE;
          else
            res = sbt::server_update_dense(r->t, stage, r->K_new, st);
        } else {
          // the four arrays back to back, each 256-byte aligned
          const size_t part = Pool::round((size_t)r->nnz * 4);
          for (int q = 0; q < 4 && res == SBT_OK; ++q)
            if (r->nnz > 0 && hipMemcpyAsync(stage + q * part, r->coo[q], (size_t)r->nnz * 4,
                                             hipMemcpyDeviceToDevice, st) != hipSuccess)
              res = SBT_E_DEVICE;
          if (res == SBT_OK)
            res = sbt::server_update_coo(r->t, (const int32_t*)stage,
                                         (const int32_t*)(stage + part),
                                         (const int32_t*)(stage + 2 * part),
                                         (const float*)(stage + 3 * part), r->nnz, r->K_new, st);
        }
        // the update returns after its own synchronisation; the staging copy is done
        if (hipStreamSynchronize(st) != hipSuccess && res == SBT_OK) res = SBT_E_DEVICE;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        pool.release(off, r->bytes);
        charged -= r->need;
        busy.erase(r->t);
        sbt::server_lease(r->t, -1);
        r->result = res;
        r->t_done = now();
        r->state = 2;
        --running;
      }
      cv.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
  }
};

extern "C" {

sbt_status sbt_server_create(int32_t slots, int64_t staging_bytes, int64_t hbm_budget_bytes,
                             sbt_server** out) {
  if (!out || slots < 1 || slots > 32 || staging_bytes < 256 || hbm_budget_bytes < 0)
    return SBT_E_INVALID;
  sbt_server* s = new (std::nothrow) sbt_server();
  if (!s) return SBT_E_NOMEM;
  if (hipMalloc(&s->pool_mem, (size_t)staging_bytes) != hipSuccess) {
    delete s;
    return SBT_E_NOMEM;
  }
  s->pool.init((size_t)staging_bytes);
  s->budget = (size_t)hbm_budget_bytes;
  s->slots = slots;
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < slots; ++i) s->workers.emplace_back([s] { s->work(); });
  *out = s;
  return SBT_OK;
}

}  // extern "C"

namespace {
sbt_status enqueue(sbt_server* s, Request& r, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(s->mu);
  // requests that could never be admitted (the working set is checked at
  // admission, when the tensor is idle)
  if (Pool::round(r.bytes) > s->pool.size()) return SBT_E_NOMEM;
  if (s->budget && Pool::round(r.bytes) > s->budget) return SBT_E_NOMEM;
  r.ticket = s->next_ticket++;
  r.t_submit = s->now();
  s->reqs[r.ticket] = r;
  s->queue.push_back(r.ticket);
  sbt::server_lease(r.t, +1);
  *ticket = r.ticket;
  s->cv.notify_all();
  return SBT_OK;
}
}  // namespace

extern "C" {

sbt_status sbt_server_submit_dense(sbt_server* s, sbt_tensor* t, const void* Y_dev,
                                   int64_t K_new, uint64_t* ticket) {
  if (!s || !t || !Y_dev || !ticket) return SBT_E_INVALID;
  const size_t esz = sbt::store_elem_bytes(t);
  if (esz == 0) return SBT_E_STATE;
  int64_t I = 0, J = 0, K = 0;
  int32_t R = 0;
  sbt_get_shape(t, &I, &J, &K, &R);
  if (K_new < 1) return SBT_E_SHAPE;
  Request r;
  r.t = t;
  r.Y = Y_dev;
  r.K_new = K_new;
  r.bytes = (size_t)I * (size_t)J * (size_t)K_new * esz;
  return enqueue(s, r, ticket);
}

sbt_status sbt_server_submit_coo(sbt_server* s, sbt_tensor* t, const int32_t* i_dev,
                                 const int32_t* j_dev, const int32_t* k_dev, const float* v_dev,
                                 int64_t nnz, int64_t K_new, uint64_t* ticket) {
  if (!s || !t || !ticket || nnz < 0 || (nnz > 0 && (!i_dev || !j_dev || !k_dev || !v_dev)))
    return SBT_E_INVALID;
  if (!sbt::is_coo(t)) return SBT_E_STATE;
  if (K_new < 1) return SBT_E_SHAPE;
  Request r;
  r.t = t;
  r.Y = nullptr;
  r.coo[0] = i_dev;
  r.coo[1] = j_dev;
  r.coo[2] = k_dev;
  r.coo[3] = v_dev;
  r.nnz = nnz;
  r.K_new = K_new;
  r.bytes = 4 * Pool::round((size_t)nnz * 4);
  return enqueue(s, r, ticket);
}

sbt_status sbt_server_poll(sbt_server* s, uint64_t ticket, int32_t* state, sbt_status* result,
                           double* t_submit, double* t_start, double* t_done) {
  if (!s) return SBT_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return SBT_E_INVALID;
  const Request& r = it->second;
  if (state) *state = r.state;
  if (result) *result = r.result;
  if (t_submit) *t_submit = r.t_submit;
  if (t_start) *t_start = r.t_start;
  if (t_done) *t_done = r.t_done;
  return SBT_OK;
}

sbt_status sbt_server_drain(sbt_server* s) {
  if (!s) return SBT_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
  return SBT_OK;
}

void sbt_server_destroy(sbt_server* s) {
  if (!s) return;
  sbt_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& w : s->workers) w.join();
  (void)hipFree(s->pool_mem);
  delete s;
}

}  // extern "C"
