// Continuous-batching solve server (one GPU).
//
// Requests arrive with (dim, degree, level, rhs, tolerance, solve mode).  A
// request is admitted, in arrival order, as soon as a slot is free and its
// device footprint fits the remaining memory budget; idle hierarchies of
// finished requests are cached per (dim, degree, level, mode) and handed to
// later requests of the same shape, and evicted (least recently used first)
// when a new shape needs their memory.  Requests of the same (dim, degree,
// solve mode) form a group with one HIP stream; different groups overlap on
// the device.  A tick enqueues the set-up of newly admitted requests and one CG
// iteration for every active request, waits once for all streams, launches the
// true residual of converged requests, then preconditions every group (new
// requests included) with one batched V-cycle whose smoother colour passes are
// packed into one launch per (level, colour) across the group's requests
// (levels may differ); converged requests are retired once their true residual,
// queued ahead of the preconditioners, is done.  Each
// request runs exactly the arithmetic of a stand-alone vps_pcg_solve with the
// same deterministic kernels, so its result does not depend on the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "vps.h"
#include "problem.hpp"

namespace {

struct Slot {
  vps::Problem* prob = nullptr;
  hipStream_t stream = nullptr;
  size_t bytes = 0;
  std::tuple<int, int, int, int> key;
};

struct Request {
  long long id = 0;
  int dim = 0, k = 0, level = 0, mode = 0, maxit = 0;
  double rtol = 0;
  const double* b = nullptr;
  double* x = nullptr;
  size_t bytes = 0;
  Slot slot;
  vps::CgState cs;
  bool admitted = false, done = false;
  vps_solve_stats_t stats{};
};

unsigned flags_for(int mode) {
  return mode == VPS_SOLVE_MIXED ? VPS_FLAG_FP32_HIERARCHY : VPS_FLAG_FP64_HIERARCHY;
}

// Host threads that issue the launches of different request groups at once: each group has its
// own stream and is handled by one thread, so the order of every stream's work is the order of a
// single-threaded tick (and so are the results); only the host time of issuing overlaps.
class LaunchPool {
 public:
  explicit LaunchPool(int workers) {
    for (int i = 0; i < workers; ++i) threads_.emplace_back([this] { loop(); });
  }
  ~LaunchPool() {
    {
      std::lock_guard<std::mutex> l(m_);
      stop_ = true;
    }
    wake_.notify_all();
    for (std::thread& t : threads_) t.join();
  }
  // f(0) .. f(n-1), spread over the workers and the calling thread; returns when all have run
  void run(int n, const std::function<void(int)>& f) {
    if (threads_.empty() || n <= 1) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> l(m_);
      job_ = &f;
      n_ = n;
      next_ = 0;
      done_ = 0;
      device_ = dev;
      ++gen_;
    }
    wake_.notify_all();
    work();
    std::unique_lock<std::mutex> l(m_);
    finished_.wait(l, [this] { return done_ == n_; });
    job_ = nullptr;
  }

 private:
  void work() {
    for (;;) {
      int i;
      const std::function<void(int)>* f;
      {
        std::lock_guard<std::mutex> l(m_);
        if (!job_ || next_ >= n_) return;
        i = next_++;
        f = job_;
      }
      (*f)(i);
      std::lock_guard<std::mutex> l(m_);
      if (++done_ == n_) finished_.notify_all();
    }
  }
  void loop() {
    unsigned seen = 0;
    for (;;) {
      int dev;
      {
        std::unique_lock<std::mutex> l(m_);
        wake_.wait(l, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        dev = device_;
      }
      if (hipSetDevice(dev) != hipSuccess) (void)hipGetLastError();  // the caller's device
      work();
    }
  }
  std::vector<std::thread> threads_;
  std::mutex m_;
  std::condition_variable wake_, finished_;
  const std::function<void(int)>* job_ = nullptr;
  int n_ = 0, next_ = 0, done_ = 0, device_ = 0;
  unsigned gen_ = 0;
  bool stop_ = false;
};

}  // namespace

struct vps_server {
  size_t budget = 0;
  int max_active = 1;
  long long next_id = 1;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<long long, Request*> all;
  std::list<Slot> idle;  // cached hierarchies, most recently used at the front
  std::deque<long long> completed;  // finished tickets not yet reported by vps_server_completed
  size_t in_use = 0, cached = 0;
  std::map<std::tuple<int, int, int>, hipStream_t> streams;  // per (dim, degree, mode)
  std::map<std::tuple<int, int, int>, hipEvent_t> end_events;  // per stream: true residuals done
  LaunchPool* pool = nullptr;
};

namespace {

int sfail(int code, const std::string& m) {
  vps::set_last_error(m);
  return code;
}

void free_slot(Slot& s) {
  delete s.prob;  // synchronises the problem's (group) stream
  s.prob = nullptr;
  s.stream = nullptr;
}

hipStream_t group_stream(vps_server* S, int dim, int k, int mode) {
  auto key = std::make_tuple(dim, k, mode);
  auto it = S->streams.find(key);
  if (it != S->streams.end()) return it->second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  S->streams[key] = st;
  return st;
}

// Try to give request r a hierarchy.  Returns 1 on success, 0 if it must wait, <0 on error.
int acquire(vps_server* S, Request* r) {
  auto key = std::make_tuple(r->dim, r->k, r->level, r->mode);
  for (auto it = S->idle.begin(); it != S->idle.end(); ++it) {
    if (it->key == key) {
      r->slot = *it;
      S->cached -= it->bytes;
      S->in_use += it->bytes;
      S->idle.erase(it);
      return 1;
    }
  }
  while (S->in_use + S->cached + r->bytes > S->budget && !S->idle.empty()) {
    Slot victim = S->idle.back();
    S->idle.pop_back();
    S->cached -= victim.bytes;
    free_slot(victim);
  }
  if (S->in_use + S->cached + r->bytes > S->budget) return 0;
  Slot s;
  s.key = key;
  s.bytes = r->bytes;
  s.stream = group_stream(S, r->dim, r->k, r->mode);
  if (!s.stream) return sfail(VPS_EHIP, "hipStreamCreate failed");
  vps::Status st = vps::create_problem(r->dim, r->k, r->level, flags_for(r->mode), s.stream, &s.prob);
  if (st.code) return sfail(st.code, st.msg);
  S->in_use += s.bytes;
  r->slot = s;
  return 1;
}

void release(vps_server* S, Request* r) {
  S->in_use -= r->slot.bytes;
  S->cached += r->slot.bytes;
  S->idle.push_front(r->slot);
  r->slot = Slot();
}

void finish(vps_server* S, Request* r) {
  r->done = true;
  S->completed.push_back(r->id);
  r->stats.iterations = r->cs.stats.iterations;
  r->stats.rel_residual = r->cs.stats.rel_residual;
  r->stats.true_rel_residual = r->cs.stats.true_rel_residual;
  r->stats.status = r->cs.stats.status;
}

}  // namespace

extern "C" {

int vps_server_create(size_t hbm_budget_bytes, int max_active, void* hip_stream, vps_server** out) {
  (void)hip_stream;
  if (!out || max_active < 1 || hbm_budget_bytes == 0) return sfail(VPS_EINVAL, "bad server arguments");
  vps_server* s = new vps_server();
  s->budget = hbm_budget_bytes;
  s->max_active = max_active;
  const unsigned hw = std::thread::hardware_concurrency();
#ifndef VPS_SERVER_THREADS
#define VPS_SERVER_THREADS 7u
#endif
  const int workers = hw > 2 ? (int)std::min(hw - 1, (unsigned)VPS_SERVER_THREADS) : 0;  // plus the calling thread
  s->pool = new LaunchPool(workers);
  *out = s;
  return VPS_OK;
}

int vps_server_submit(vps_server* s, int dim, int degree, int level, const double* b_dev, double* x_dev, double rtol,
                      int solve_mode, int maxit, long long* ticket) {
  if (!s || !b_dev || !x_dev || !ticket) return sfail(VPS_EINVAL, "null argument");
  if (solve_mode != VPS_SOLVE_FP64 && solve_mode != VPS_SOLVE_MIXED) return sfail(VPS_EINVAL, "bad solve mode");
  if (!(rtol > 0) || maxit < 1) return sfail(VPS_EINVAL, "rtol must be > 0 and maxit >= 1");
  size_t bytes = 0;
  if (int e = vps_footprint_bytes(dim, degree, level, flags_for(solve_mode), &bytes)) return sfail(e, vps_last_error());
  if (bytes > s->budget) return sfail(VPS_EBUSY, "request footprint exceeds the server memory budget");
  Request* r = new Request();
  r->id = s->next_id++;
  r->dim = dim;
  r->k = degree;
  r->level = level;
  r->mode = solve_mode;
  r->maxit = maxit;
  r->rtol = rtol;
  r->b = b_dev;
  r->x = x_dev;
  r->bytes = bytes;
  s->queue.push_back(r);
  s->all[r->id] = r;
  *ticket = r->id;
  return VPS_OK;
}

int vps_server_step(vps_server* s, int* n_active, int* n_queued) {
  if (!s) return sfail(VPS_EINVAL, "null server");
  using Key = std::tuple<int, int, int>;
  auto key_of = [](const Request* r) { return std::make_tuple(r->dim, r->k, r->mode); };
  // Run fn(request) for each list of `lists` on the launch pool (one list per stream).
  auto on_pool = [&](std::vector<std::vector<Request*>*>& lists, const std::function<vps::Status(Request*)>& fn) {
    std::vector<vps::Status> res(lists.size());
    s->pool->run((int)lists.size(), [&](int i) {
      for (Request* r : *lists[i]) {
        res[i] = fn(r);
        if (res[i].code) return;
      }
    });
    for (const vps::Status& st : res)
      if (st.code) return st;
    return vps::Status::ok();
  };
  // admit in arrival order; the rhs check of a new request waits for this tick's synchronisation
  std::vector<Request*> begun;
  while (!s->queue.empty() && (int)(s->active.size() + begun.size()) < s->max_active) {
    Request* r = s->queue.front();
    int got = acquire(s, r);
    if (got < 0) return got;
    if (got == 0) break;
    s->queue.pop_front();
    r->admitted = true;
    vps::Status st = vps::pcg_begin_launch(r->slot.prob, r->mode, r->b, r->x, &r->cs);
    if (st.code) return sfail(st.code, st.msg);
    begun.push_back(r);
  }
  // one CG iteration for every active request (groups overlap on their streams; each group's
  // launches are issued by one host thread)
  {
    std::map<Key, std::vector<Request*>> by_stream;
    for (Request* r : s->active) by_stream[key_of(r)].push_back(r);
    std::vector<std::vector<Request*>*> lists;
    for (auto& kv : by_stream) lists.push_back(&kv.second);
    vps::Status st = on_pool(lists, [](Request* r) {
      return vps::pcg_iterate_launch(r->slot.prob, r->mode, r->x, &r->cs);
    });
    if (st.code) return sfail(st.code, st.msg);
  }
  for (auto& kv : s->streams)
    if (hipStreamSynchronize(kv.second) != hipSuccess) return sfail(VPS_EHIP, "stream synchronize failed");
  // a request whose CG has ended launches its true residual (read back once this tick's
  // preconditioners are issued) or, with nothing to compute, is finished now
  std::vector<Request*> ending;
  auto end_request = [&](Request* r) -> vps::Status {
    bool pending = false;
    vps::Status st = vps::pcg_end_launch(r->slot.prob, r->b, r->x, &r->cs, &pending);
    if (st.code) return st;
    if (pending) {
      ending.push_back(r);
    } else {
      finish(s, r);
      release(s, r);
    }
    return vps::Status::ok();
  };
  std::vector<Request*> still;
  std::map<Key, std::vector<Request*>> groups;
  for (Request* r : s->active) {
    vps::Status st = vps::pcg_decide(r->slot.prob, r->mode, r->rtol, r->maxit, &r->cs);
    if (st.code) return sfail(st.code, st.msg);
    if (r->cs.done) {
      st = end_request(r);
      if (st.code) return sfail(st.code, st.msg);
    } else {
      still.push_back(r);
      groups[key_of(r)].push_back(r);
    }
  }
  std::vector<Request*> newcomers;
  for (Request* r : begun) {
    vps::Status st = vps::pcg_begin_check(r->slot.prob, &r->cs);
    if (st.code) return sfail(st.code, st.msg);
    if (r->cs.done) {
      st = end_request(r);
      if (st.code) return sfail(st.code, st.msg);
    } else {
      newcomers.push_back(r);
      groups[key_of(r)].push_back(r);
    }
  }
  // mark the end of the true-residual work on each stream that has some: the host waits for these
  // marks, not for the preconditioners queued behind them
  std::vector<hipEvent_t> marks;
  {
    std::set<Key> keys;
    for (Request* r : ending) keys.insert(key_of(r));
    for (const Key& k : keys) {
      hipEvent_t& ev = s->end_events[k];
      if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
        return sfail(VPS_EHIP, "hipEventCreate failed");
      }
      if (hipEventRecord(ev, s->streams[k]) != hipSuccess) return sfail(VPS_EHIP, "hipEventRecord failed");
      marks.push_back(ev);
    }
  }
  // preconditioner: one batched V-cycle per group, colour passes packed across its requests (new
  // requests take their first application with the others); groups issue from parallel threads
  {
    std::vector<std::pair<const Key, std::vector<Request*>>*> glist;
    for (auto& kv : groups) glist.push_back(&kv);
    std::vector<vps::Status> res(glist.size());
    s->pool->run((int)glist.size(), [&](int i) {
      std::vector<vps::Problem*> ps;
      for (Request* r : glist[i]->second) ps.push_back(r->slot.prob);
      res[i] = vps::precondition_group(ps.data(), (int)ps.size(), std::get<2>(glist[i]->first));
      if (res[i].code) return;
      for (Request* r : glist[i]->second) {
        const bool fresh = r->cs.it == 0;  // first application: p = z
        res[i] = fresh ? vps::pcg_begin_after_precond(r->slot.prob, r->mode)
                       : vps::pcg_after_precond(r->slot.prob, r->mode);
        if (res[i].code) return;
      }
    });
    for (const vps::Status& st : res)
      if (st.code) return sfail(st.code, st.msg);
  }
  for (hipEvent_t ev : marks)
    if (hipEventSynchronize(ev) != hipSuccess) return sfail(VPS_EHIP, "event synchronize failed");
  for (Request* r : ending) {
    vps::pcg_end_finish(r->slot.prob, &r->cs);
    finish(s, r);
    release(s, r);
  }
  still.insert(still.end(), newcomers.begin(), newcomers.end());
  s->active.swap(still);
  if (n_active) *n_active = (int)s->active.size();
  if (n_queued) *n_queued = (int)s->queue.size();
  return VPS_OK;
}

int vps_server_poll(vps_server* s, long long ticket, int* done, vps_solve_stats_t* stats) {
  if (!s || !done) return sfail(VPS_EINVAL, "null argument");
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return sfail(VPS_EINVAL, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  if (it->second->done && stats) *stats = it->second->stats;
  return VPS_OK;
}

int vps_server_completed(vps_server* s, long long* tickets, int cap, int* n) {
  if (!s || !n || cap < 0 || (cap > 0 && !tickets)) return sfail(VPS_EINVAL, "bad arguments");
  int k = 0;
  while (k < cap && !s->completed.empty()) {
    tickets[k++] = s->completed.front();
    s->completed.pop_front();
  }
  *n = k;
  return VPS_OK;
}

int vps_server_memory(vps_server* s, size_t* in_use, size_t* cached) {
  if (!s) return sfail(VPS_EINVAL, "null server");
  if (in_use) *in_use = s->in_use;
  if (cached) *cached = s->cached;
  return VPS_OK;
}

int vps_server_destroy(vps_server* s) {
  if (!s) return VPS_OK;
  delete s->pool;
  for (auto& kv : s->streams) (void)hipStreamSynchronize(kv.second);
  for (Request* r : s->active) free_slot(r->slot);
  for (Slot& sl : s->idle) free_slot(sl);
  for (auto& kv : s->end_events)
    if (kv.second) (void)hipEventDestroy(kv.second);
  for (auto& kv : s->streams) (void)hipStreamDestroy(kv.second);
  for (auto& kv : s->all) delete kv.second;
  delete s;
  return VPS_OK;
}

}  // extern "C"
