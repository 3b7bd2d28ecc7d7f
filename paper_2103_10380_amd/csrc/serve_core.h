// Continuous-batching scheduler of the render server (host only, no HIP).
//
// Requests wait in a FIFO queue. Before every step the scheduler admits
// queued requests in order while their output fits the arena and fewer than
// max_inflight are running (a request that does not fit blocks the ones behind
// it, so admission stays FIFO). A step then takes up to step_tiles 8x8 tiles
// from the running requests, an equal share each; requests that are only
// partly covered continue in the next step, and requests admitted meanwhile
// join it.
// An Executor runs each step (the GPU executor launches one persistent kernel
// per storage-format group; tests use a fake one). Two steps are in flight at a time: step i+1 is
// planned and launched before the scheduler waits for step i, so the device
// gets the next step without waiting for the host. A request completes when
// every step holding its tiles has finished.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace fnr_serve {

enum Status { kOk = 0, kInval = -1, kNoMem = -2, kDevice = -3, kBusy = -4, kCanceled = -5,
              kShutdown = -6, kTimedOut = -7 };

// First-fit allocator over [0, size) with coalescing; 256-byte granules.
class Arena {
 public:
  explicit Arena(uint64_t size) : size_(size) {
    if (size_) free_[0] = size_;
  }
  static uint64_t round(uint64_t n) { return (n + 255) & ~uint64_t(255); }
  bool alloc(uint64_t n, uint64_t *off) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = round(n);
    used_ -= n;
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
  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }

 private:
  uint64_t size_, used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

enum class RState { Queued, Running, Done, Canceled, Failed };

struct Request {
  uint64_t ticket = 0;
  int scene = 0;
  float K[9], c2w[12];
  int H = 0, W = 0, N = 0;
  float near_ = 0, far_ = 0, eps = 0;
  int tiles = 0, next_tile = 0;
  uint64_t bytes = 0, off = 0;
  int pending = 0;  // launched steps holding tiles of this request, not yet waited for
  bool has_arena = false, cancel_requested = false, failed = false;
  RState st = RState::Queued;
  Status err = kOk;
  std::chrono::steady_clock::time_point t_submit, t_done;
};

struct Segment {
  Request *req;
  int first, count;  // tiles [first, first + count) of the request
};

struct Step {
  std::vector<Segment> segs;
  int total_tiles = 0;
};

class Executor {
 public:
  virtual ~Executor() {}
  // Runs every segment of the step to completion; returns kOk or an error.
  virtual Status run(const Step &step, uint64_t arena_base_unused) = 0;
  // Asynchronous form, slots 0 and 1 used alternately: launch a step, wait for
  // it later (the step object stays alive until then). The default runs the
  // step at launch.
  virtual Status launch(const Step &step, int slot) {
    done_[slot & 1] = run(step, 0);
    return kOk;
  }
  virtual Status wait(int slot) { return done_[slot & 1]; }

 private:
  Status done_[2] = {kOk, kOk};
};

struct Config {
  uint64_t arena_bytes = 0;
  int max_inflight = 16;
  int queue_cap = 4096;
  // about 16M rays: when the server is loaded a step holds many requests, so
  // the gap before each step's launches (graph replay with its table copy) is
  // amortised; a lone request of up to 1920x1080 (32,400 tiles) is one step
  int step_tiles = 1 << 18;
};

class Core {
 public:
  Core(const Config &cfg, Executor *ex) : cfg_(cfg), arena_(cfg.arena_bytes), ex_(ex) {
    worker_ = std::thread([this] { loop(); });
  }
  ~Core() { shutdown(); }

  Status submit(std::unique_ptr<Request> r, uint64_t *ticket) {
    std::unique_lock<std::mutex> g(mu_);
    if (stopping_) return kShutdown;
    if (Arena::round(r->bytes) > arena_.size()) return kNoMem;
    if ((int)queue_.size() >= cfg_.queue_cap) return kBusy;
    r->ticket = ++last_ticket_;
    r->t_submit = std::chrono::steady_clock::now();
    r->tiles = ((r->W + 7) / 8) * ((r->H + 7) / 8);
    *ticket = r->ticket;
    Request *raw = r.get();
    all_[raw->ticket] = std::move(r);
    queue_.push_back(raw);
    cv_work_.notify_all();
    return kOk;
  }

  // Waits for a ticket; on kOk returns the arena offset and the latency.
  Status wait(uint64_t ticket, int64_t timeout_us, uint64_t *off, double *latency_ms) {
    std::unique_lock<std::mutex> g(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return kInval;
    Request *r = it->second.get();
    auto done = [&] { return r->st == RState::Done || r->st == RState::Canceled ||
                             r->st == RState::Failed; };
    if (timeout_us < 0) {
      cv_done_.wait(g, done);
    } else if (!cv_done_.wait_until(g, deadline(timeout_us), done)) {
      return kTimedOut;
    }
    if (r->st == RState::Canceled) return kCanceled;
    if (r->st == RState::Failed) return r->err;
    if (off) *off = r->off;
    if (latency_ms)
      *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    return kOk;
  }

  Status release(uint64_t ticket) {
    std::unique_lock<std::mutex> g(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return kInval;
    Request *r = it->second.get();
    if (r->st == RState::Queued || r->st == RState::Running) return kBusy;
    if (r->has_arena) arena_.release(r->off, r->bytes);
    all_.erase(it);
    cv_work_.notify_all();  // memory came back: admission may proceed
    return kOk;
  }

  Status cancel(uint64_t ticket) {
    std::unique_lock<std::mutex> g(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return kInval;
    Request *r = it->second.get();
    if (r->st == RState::Queued) {
      queue_.erase(std::find(queue_.begin(), queue_.end(), r));
      finish(r, RState::Canceled, kCanceled);
    } else if (r->st == RState::Running) {
      r->cancel_requested = true;  // retired at the next step boundary
    }
    return kOk;
  }

  void stats(uint64_t *steps, uint64_t *completed, uint64_t *max_batch) {
    std::unique_lock<std::mutex> g(mu_);
    if (steps) *steps = steps_;
    if (completed) *completed = completed_;
    if (max_batch) *max_batch = max_batch_;
  }

  uint64_t arena_used() {
    std::unique_lock<std::mutex> g(mu_);
    return arena_.used();
  }

  // Cancels queued requests, lets running ones finish, stops the worker.
  void shutdown() {
    {
      std::unique_lock<std::mutex> g(mu_);
      if (!stopping_) {
        stopping_ = true;
        for (Request *r : queue_) finish(r, RState::Canceled, kShutdown);
        queue_.clear();
      }
      cv_work_.notify_all();
    }
    if (worker_.joinable()) worker_.join();
  }

  Request *find(uint64_t ticket) {
    auto it = all_.find(ticket);
    return it == all_.end() ? nullptr : it->second.get();
  }
  std::mutex &mutex() { return mu_; }

 private:
  // Timed waits use the system clock, whose wait primitive sanitizers model.
  static std::chrono::system_clock::time_point deadline(int64_t us) {
    return std::chrono::system_clock::now() + std::chrono::microseconds(us);
  }

  void finish(Request *r, RState st, Status err) {
    r->st = st;
    r->err = err;
    r->t_done = std::chrono::steady_clock::now();
    if ((st == RState::Canceled || st == RState::Failed) && r->has_arena) {
      arena_.release(r->off, r->bytes);
      r->has_arena = false;
    }
    if (st == RState::Done) ++completed_;
    cv_done_.notify_all();
  }

  void admit() {
    while (!queue_.empty() && (int)running_.size() < cfg_.max_inflight) {
      Request *r = queue_.front();
      if (!arena_.alloc(r->bytes, &r->off)) break;  // FIFO: the head waits for memory
      r->has_arena = true;
      r->st = RState::Running;
      queue_.pop_front();
      running_.push_back(r);
    }
  }

  // Every running request gets an equal share of the step's tile budget (so a
  // small request that joins behind a large one finishes within a step or
  // two); budget a request cannot use goes to the others in admission order.
  void plan(Step *s) {
    s->segs.clear();
    s->total_tiles = 0;
    std::vector<Request *> act;
    for (Request *r : running_)
      if (!r->cancel_requested && !r->failed && r->next_tile < r->tiles) act.push_back(r);
    if (act.empty()) return;
    std::vector<int> take(act.size(), 0);
    int budget = cfg_.step_tiles;
    const int share = std::max(1, budget / (int)act.size());
    for (size_t j = 0; j < act.size() && budget > 0; ++j) {
      take[j] = std::min({share, act[j]->tiles - act[j]->next_tile, budget});
      budget -= take[j];
    }
    for (size_t j = 0; j < act.size() && budget > 0; ++j) {
      const int more = std::min(budget, act[j]->tiles - act[j]->next_tile - take[j]);
      take[j] += more;
      budget -= more;
    }
    for (size_t j = 0; j < act.size(); ++j) {
      if (take[j] <= 0) continue;
      s->segs.push_back(Segment{act[j], act[j]->next_tile, take[j]});
      s->total_tiles += take[j];
    }
  }

  // Retires running requests that are done, cancelled or failed and have no
  // tiles in a launched step.
  void retire() {
    for (auto it = running_.begin(); it != running_.end();) {
      Request *r = *it;
      if (r->pending > 0) {
        ++it;
      } else if (r->failed) {
        finish(r, RState::Failed, r->err);
        it = running_.erase(it);
      } else if (r->cancel_requested) {
        finish(r, RState::Canceled, kCanceled);
        it = running_.erase(it);
      } else if (r->next_tile >= r->tiles) {
        finish(r, RState::Done, kOk);
        it = running_.erase(it);
      } else {
        ++it;
      }
    }
  }

  // A launched step has finished (or failed): its requests have one step less
  // in flight.
  void step_done(const Step &s, Status st) {
    for (const Segment &sg : s.segs) {
      Request *r = sg.req;
      --r->pending;
      if (st != kOk && !r->failed) {
        r->failed = true;
        r->err = st;
      }
    }
  }

  void loop() {
    std::unique_lock<std::mutex> g(mu_);
    Step steps[2];
    bool inflight[2] = {false, false};
    int cur = 0;
    for (;;) {
      const int prev = cur ^ 1;
      if (!inflight[prev])
        cv_work_.wait(g, [&] { return stopping_ || !running_.empty() || !queue_.empty(); });
      if (stopping_ && running_.empty() && !inflight[prev]) break;
      admit();
      retire();
      plan(&steps[cur]);
      bool launched = false;
      if (!steps[cur].segs.empty()) {
        for (const Segment &sg : steps[cur].segs) {
          sg.req->next_tile += sg.count;
          ++sg.req->pending;
        }
        ++steps_;
        max_batch_ = std::max<uint64_t>(max_batch_, steps[cur].segs.size());
        g.unlock();
        const Status st = ex_->launch(steps[cur], cur);
        g.lock();
        if (st != kOk) {
          step_done(steps[cur], st);
        } else {
          inflight[cur] = true;
          launched = true;
        }
      }
      if (inflight[prev]) {
        g.unlock();
        const Status st = ex_->wait(prev);
        g.lock();
        inflight[prev] = false;
        step_done(steps[prev], st);
        retire();
      } else if (!launched) {
        retire();
        if (running_.empty() && !queue_.empty() && !stopping_) {
          // nothing fits until results are released
          cv_work_.wait_until(g, deadline(5000));
        }
        continue;
      }
      if (launched) cur ^= 1;
    }
  }

  Config cfg_;
  Arena arena_;
  Executor *ex_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Request *> queue_;
  std::vector<Request *> running_;
  std::map<uint64_t, std::unique_ptr<Request>> all_;
  uint64_t last_ticket_ = 0, steps_ = 0, completed_ = 0, max_batch_ = 0;
  bool stopping_ = false;
  std::thread worker_;
};

}  // namespace fnr_serve
