// Continuous-batching solve server (one GPU).
//
// Requests arrive with (dim, degree, level, rhs, tolerance, solve mode).  The
// caller's stream (given at creation) is marked at submit, and the request's
// first device work waits for that mark, so a rhs written on the caller's
// stream just before submit is read complete.  A request is admitted, in arrival order, as soon as a slot is free and its
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
//
// A request whose launches fail ends with that error in its status and gives
// its hierarchy back; the other requests and the server's accounting carry on.
// Only a failed wait on a group stream (the device itself is in error) ends
// every active request of the tick.
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
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
  int inject = -1;             // test hook: the stage whose launch is made to fail
  bool admitted = false, done = false;
  vps_solve_stats_t stats{};
};

// Stages at which vps_server_inject_fault can make a request's launch fail.
enum { kStageAdmit = 0, kStageIterate = 1, kStagePrecondition = 2 };

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
  hipStream_t caller = nullptr;  // the caller's stream: request inputs are ready on it at submit
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
  // evict (least recently used first) only if that can make room: otherwise the request waits for
  // active requests to finish and the cache stays
  if (S->in_use + r->bytes > S->budget) return 0;
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

void drop_ready(Request* r) {
  if (r->ready) (void)hipEventDestroy(r->ready);
  r->ready = nullptr;
}

// End request r with error `code` (its status) and give its hierarchy back to the cache: the
// hierarchy holds no state a later request relies on (every solve starts by filling its vectors).
void fail_request(vps_server* S, Request* r, int code, const std::string& msg) {
  vps::set_last_error(msg);
  r->cs.done = true;
  r->cs.stats.status = code;
  drop_ready(r);
  finish(S, r);
  if (r->slot.prob) release(S, r);
}

// The test hook: a launch of request r at `stage` reports an error instead of running.
vps::Status injected(const Request* r, int stage) {
  if (r->inject == stage) return vps::Status{VPS_EHIP, "fault injected by vps_server_inject_fault"};
  return vps::Status::ok();
}

}  // namespace

extern "C" {

int vps_server_create(size_t hbm_budget_bytes, int max_active, void* hip_stream, vps_server** out) {
  if (!out || max_active < 1 || hbm_budget_bytes == 0) return sfail(VPS_EINVAL, "bad server arguments");
  vps_server* s = new vps_server();
  s->caller = static_cast<hipStream_t>(hip_stream);
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
  // mark the caller's stream: the request's first device work waits for what is queued there now
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return sfail(VPS_EHIP, "hipEventCreate failed");
  }
  if (hipEventRecord(ready, s->caller) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(ready);
    return sfail(VPS_EHIP, "hipEventRecord on the caller's stream failed");
  }
  Request* r = new Request();
  r->ready = ready;
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
  // Run fn(request) for each list of `lists` on the launch pool (one list per stream); a request
  // whose fn fails is recorded in `failed` (the others of its list still run).
  using Failure = std::pair<Request*, vps::Status>;
  auto on_pool = [&](std::vector<std::vector<Request*>*>& lists, const std::function<vps::Status(Request*)>& fn,
                     std::vector<Failure>* failed) {
    std::vector<std::vector<Failure>> res(lists.size());
    s->pool->run((int)lists.size(), [&](int i) {
      for (Request* r : *lists[i]) {
        vps::Status st = fn(r);
        if (st.code) res[i].push_back(Failure(r, st));
      }
    });
    for (auto& v : res) failed->insert(failed->end(), v.begin(), v.end());
  };
  // admit in arrival order; the rhs check of a new request waits for this tick's synchronisation
  std::vector<Request*> begun;
  while (!s->queue.empty() && (int)(s->active.size() + begun.size()) < s->max_active) {
    Request* r = s->queue.front();
    int got = acquire(s, r);
    if (got == 0) break;
    s->queue.pop_front();
    r->admitted = true;
    if (got < 0) {
      fail_request(s, r, got, vps_last_error());
      continue;
    }
    vps::Status st = injected(r, kStageAdmit);
    if (!st.code && hipStreamWaitEvent(r->slot.stream, r->ready, 0) != hipSuccess) {
      (void)hipGetLastError();
      st = vps::Status{VPS_EHIP, "hipStreamWaitEvent on the submit mark failed"};
    }
    if (!st.code) st = vps::pcg_begin_launch(r->slot.prob, r->mode, r->b, r->x, &r->cs);
    if (st.code) {
      fail_request(s, r, st.code, st.msg);
      continue;
    }
    drop_ready(r);  // released once the wait queued above has passed
    begun.push_back(r);
  }
  // one CG iteration for every active request (groups overlap on their streams; each group's
  // launches are issued by one host thread)
  std::set<Request*> gone;  // requests that ended with an error this tick
  {
    std::map<Key, std::vector<Request*>> by_stream;
    for (Request* r : s->active) by_stream[key_of(r)].push_back(r);
    std::vector<std::vector<Request*>*> lists;
    for (auto& kv : by_stream) lists.push_back(&kv.second);
    std::vector<Failure> failed;
    on_pool(lists, [](Request* r) {
      vps::Status st = injected(r, kStageIterate);
      return st.code ? st : vps::pcg_iterate_launch(r->slot.prob, r->mode, r->x, &r->cs);
    }, &failed);
    for (Failure& f : failed) {
      fail_request(s, f.first, f.second.code, f.second.msg);
      gone.insert(f.first);
    }
  }
  bool device_error = false;
  for (auto& kv : s->streams)
    if (hipStreamSynchronize(kv.second) != hipSuccess) device_error = true;
  if (device_error) {
    // the device is in error: every request in flight ends with it, the queue stays
    (void)hipGetLastError();
    for (Request* r : s->active)
      if (!gone.count(r)) fail_request(s, r, VPS_EHIP, "stream synchronize failed");
    for (Request* r : begun) fail_request(s, r, VPS_EHIP, "stream synchronize failed");
    s->active.clear();
    if (n_active) *n_active = 0;
    if (n_queued) *n_queued = (int)s->queue.size();
    return sfail(VPS_EHIP, "stream synchronize failed");
  }
  // a request whose CG has ended launches its true residual (read back once this tick's
  // preconditioners are issued) or, with nothing to compute, is finished now
  std::vector<Request*> ending;
  auto end_request = [&](Request* r) {
    bool pending = false;
    vps::Status st = vps::pcg_end_launch(r->slot.prob, r->b, r->x, &r->cs, &pending);
    if (st.code) {
      fail_request(s, r, st.code, st.msg);
    } else if (pending) {
      ending.push_back(r);
    } else {
      finish(s, r);
      release(s, r);
    }
  };
  std::vector<Request*> still;
  std::map<Key, std::vector<Request*>> groups;
  for (Request* r : s->active) {
    if (gone.count(r)) continue;
    vps::Status st = vps::pcg_decide(r->slot.prob, r->mode, r->rtol, r->maxit, &r->cs);
    if (st.code) {
      fail_request(s, r, st.code, st.msg);
    } else if (r->cs.done) {
      end_request(r);
    } else {
      still.push_back(r);
      groups[key_of(r)].push_back(r);
    }
  }
  std::vector<Request*> newcomers;
  for (Request* r : begun) {
    vps::Status st = vps::pcg_begin_check(r->slot.prob, &r->cs);
    if (st.code) {
      fail_request(s, r, st.code, st.msg);
    } else if (r->cs.done) {
      end_request(r);
    } else {
      newcomers.push_back(r);
      groups[key_of(r)].push_back(r);
    }
  }
  // mark the end of the true-residual work on each stream that has some: the host waits for these
  // marks, not for the preconditioners queued behind them
  std::vector<std::pair<hipEvent_t, Key>> marks;
  {
    std::set<Key> keys;
    for (Request* r : ending) keys.insert(key_of(r));
    for (const Key& k : keys) {
      hipEvent_t& ev = s->end_events[k];
      bool ok = ev || hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      if (!ok) ev = nullptr;
      ok = ok && hipEventRecord(ev, s->streams[k]) == hipSuccess;
      if (ok) {
        marks.push_back(std::make_pair(ev, k));
      } else {
        // the true residual of these requests cannot be waited for: they end with the error
        (void)hipGetLastError();
        std::vector<Request*> keep;
        for (Request* r : ending) {
          if (key_of(r) == k)
            fail_request(s, r, VPS_EHIP, "hipEventRecord failed");
          else
            keep.push_back(r);
        }
        ending.swap(keep);
      }
    }
  }
  // preconditioner: one batched V-cycle per group, colour passes packed across its requests (new
  // requests take their first application with the others); groups issue from parallel threads.
  // A failure ends every request of its group (their V-cycles share launches).
  {
    std::vector<std::pair<const Key, std::vector<Request*>>*> glist;
    for (auto& kv : groups) glist.push_back(&kv);
    std::vector<vps::Status> res(glist.size());
    s->pool->run((int)glist.size(), [&](int i) {
      std::vector<vps::Problem*> ps;
      for (Request* r : glist[i]->second) {
        res[i] = injected(r, kStagePrecondition);
        if (res[i].code) return;
        ps.push_back(r->slot.prob);
      }
      res[i] = vps::precondition_group(ps.data(), (int)ps.size(), std::get<2>(glist[i]->first));
      if (res[i].code) return;
      for (Request* r : glist[i]->second) {
        const bool fresh = r->cs.it == 0;  // first application: p = z
        res[i] = fresh ? vps::pcg_begin_after_precond(r->slot.prob, r->mode)
                       : vps::pcg_after_precond(r->slot.prob, r->mode);
        if (res[i].code) return;
      }
    });
    for (size_t i = 0; i < glist.size(); ++i) {
      if (!res[i].code) continue;
      for (Request* r : glist[i]->second) {
        fail_request(s, r, res[i].code, res[i].msg);
        gone.insert(r);
      }
    }
  }
  for (auto& mk : marks) {
    if (hipEventSynchronize(mk.first) == hipSuccess) continue;
    (void)hipGetLastError();
    std::vector<Request*> keep;
    for (Request* r : ending) {
      if (key_of(r) == mk.second)
        fail_request(s, r, VPS_EHIP, "event synchronize failed");
      else
        keep.push_back(r);
    }
    ending.swap(keep);
  }
  for (Request* r : ending) {
    vps::pcg_end_finish(r->slot.prob, &r->cs);
    finish(s, r);
    release(s, r);
  }
  std::vector<Request*> next;
  for (Request* r : still)
    if (!gone.count(r)) next.push_back(r);
  for (Request* r : newcomers)
    if (!gone.count(r)) next.push_back(r);
  s->active.swap(next);
  if (n_active) *n_active = (int)s->active.size();
  if (n_queued) *n_queued = (int)s->queue.size();
  return VPS_OK;
}

int vps_server_inject_fault(vps_server* s, long long ticket, int stage) {
  if (!s) return sfail(VPS_EINVAL, "null server");
  if (stage < kStageAdmit || stage > kStagePrecondition) return sfail(VPS_EINVAL, "bad stage");
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return sfail(VPS_EINVAL, "unknown ticket");
  if (it->second->done) return sfail(VPS_EINVAL, "request already finished");
  it->second->inject = stage;
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
  for (auto& kv : s->all) {
    drop_ready(kv.second);
    delete kv.second;
  }
  delete s;
  return VPS_OK;
}

}  // extern "C"
