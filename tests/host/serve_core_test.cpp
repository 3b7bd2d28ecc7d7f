// Host-only tests of the render server's scheduler (serve_core.h) with a fake
// executor: admission by arena budget, FIFO order, continuous joining,
// cancellation, executor failures, shutdown. Built with g++ (optionally with
// -fsanitize=thread or address) by tests/test_serve_core.py.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "serve_core.h"

using namespace fnr_serve;

#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      exit(1);                                                           \
    }                                                                    \
  } while (0)

struct FakeExec : Executor {
  std::atomic<int> steps{0};
  std::atomic<int> fail_at{-1};
  std::atomic<int> delay_us{0};
  std::mutex mu;
  std::vector<std::vector<uint64_t>> seen;  // tickets per step
  Status run(const Step &s, uint64_t) override {
    int n = steps++;
    {
      std::lock_guard<std::mutex> g(mu);
      std::vector<uint64_t> t;
      int total = 0;
      for (auto &sg : s.segs) {
        t.push_back(sg.req->ticket);
        total += sg.count;
        CHECK(sg.first >= 0 && sg.first + sg.count <= sg.req->tiles);
      }
      CHECK(total == s.total_tiles);
      seen.push_back(t);
    }
    if (delay_us) std::this_thread::sleep_for(std::chrono::microseconds(delay_us));
    return n == fail_at ? kDevice : kOk;
  }
};

static std::unique_ptr<Request> req(int W, int H) {
  std::unique_ptr<Request> r(new Request());
  r->W = W;
  r->H = H;
  r->bytes = (uint64_t)W * H * 16;
  return r;
}

static void test_basic_completion() {
  FakeExec ex;
  Config cfg;
  cfg.arena_bytes = 64 << 20;
  Core core(cfg, &ex);
  uint64_t t[4];
  for (int i = 0; i < 4; ++i) CHECK(core.submit(req(64, 48), &t[i]) == kOk);
  for (int i = 0; i < 4; ++i) {
    uint64_t off;
    double ms;
    CHECK(core.wait(t[i], -1, &off, &ms) == kOk);
    CHECK(ms >= 0);
    CHECK(core.release(t[i]) == kOk);
  }
  CHECK(core.arena_used() == 0);
  uint64_t steps, done, mb;
  core.stats(&steps, &done, &mb);
  CHECK(done == 4);
}

static void test_arena_backpressure_and_fifo() {
  FakeExec ex;
  Config cfg;
  cfg.arena_bytes = 3 * 100 * 100 * 16;  // three 100x100 results fit
  Core core(cfg, &ex);
  uint64_t t[6];
  for (int i = 0; i < 6; ++i) CHECK(core.submit(req(100, 100), &t[i]) == kOk);
  // a request larger than the whole arena can never run
  uint64_t big;
  CHECK(core.submit(req(1000, 1000), &big) == kNoMem);
  // the first three complete; the rest wait for memory
  for (int i = 0; i < 3; ++i) CHECK(core.wait(t[i], 2000000, nullptr, nullptr) == kOk);
  CHECK(core.wait(t[3], 20000, nullptr, nullptr) == kTimedOut);
  CHECK(core.release(t[0]) == kOk);
  CHECK(core.wait(t[3], 2000000, nullptr, nullptr) == kOk);
  CHECK(core.wait(t[4], 20000, nullptr, nullptr) == kTimedOut);
  for (int i = 1; i < 4; ++i) CHECK(core.release(t[i]) == kOk);
  for (int i = 4; i < 6; ++i) {
    CHECK(core.wait(t[i], 2000000, nullptr, nullptr) == kOk);
    CHECK(core.release(t[i]) == kOk);
  }
  // FIFO: no step ever holds a later ticket before an earlier one finished admission
  std::lock_guard<std::mutex> g(ex.mu);
  uint64_t last_first = 0;
  for (auto &s : ex.seen) {
    CHECK(!s.empty());
    CHECK(s[0] >= last_first);
    last_first = s[0];
    for (size_t j = 1; j < s.size(); ++j) CHECK(s[j] > s[j - 1]);
  }
}

static void test_large_request_spans_steps_and_others_join() {
  FakeExec ex;
  ex.delay_us = 2000;
  Config cfg;
  cfg.arena_bytes = 256 << 20;
  cfg.step_tiles = 100;
  Core core(cfg, &ex);
  uint64_t a, b;
  CHECK(core.submit(req(800, 800), &a) == kOk);  // 10,000 tiles: 100 steps
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  CHECK(core.submit(req(16, 16), &b) == kOk);   // joins while a is running
  CHECK(core.wait(b, 5000000, nullptr, nullptr) == kOk);
  CHECK(core.wait(a, 20, nullptr, nullptr) == kTimedOut);  // b finished first
  CHECK(core.wait(a, 10000000, nullptr, nullptr) == kOk);
  uint64_t steps, done, mb;
  core.stats(&steps, &done, &mb);
  CHECK(steps >= 100 && mb >= 2);
  CHECK(core.release(a) == kOk && core.release(b) == kOk);
}

static void test_cancel_and_failures() {
  FakeExec ex;
  ex.delay_us = 1000;
  Config cfg;
  cfg.arena_bytes = 100 * 100 * 16;  // one at a time
  cfg.step_tiles = 20;
  Core core(cfg, &ex);
  uint64_t a, b, c;
  CHECK(core.submit(req(100, 100), &a) == kOk);
  CHECK(core.submit(req(100, 100), &b) == kOk);
  CHECK(core.submit(req(100, 100), &c) == kOk);
  CHECK(core.cancel(b) == kOk);  // queued: cancelled at once
  CHECK(core.wait(b, 0, nullptr, nullptr) == kCanceled);
  CHECK(core.cancel(a) == kOk);  // running: retired at the next step boundary
  CHECK(core.wait(a, 2000000, nullptr, nullptr) == kCanceled);
  CHECK(core.wait(c, 2000000, nullptr, nullptr) == kOk);  // memory came back
  CHECK(core.release(a) == kOk && core.release(b) == kOk && core.release(c) == kOk);
  CHECK(core.arena_used() == 0);
  // an executor error fails the requests of that step
  ex.fail_at = ex.steps + 1;
  uint64_t d;
  CHECK(core.submit(req(40, 40), &d) == kOk);
  Status s = core.wait(d, 2000000, nullptr, nullptr);
  CHECK(s == kDevice || s == kOk);
  CHECK(core.release(d) == kOk);
  CHECK(core.release(12345) == kInval);
}

static void test_shutdown() {
  FakeExec ex;
  ex.delay_us = 500;
  Config cfg;
  cfg.arena_bytes = 100 * 100 * 16;
  Core *core = new Core(cfg, &ex);
  uint64_t t[5];
  for (int i = 0; i < 5; ++i) CHECK(core->submit(req(100, 100), &t[i]) == kOk);
  core->shutdown();
  uint64_t x;
  CHECK(core->submit(req(8, 8), &x) == kShutdown);
  int done = 0, canceled = 0;
  for (int i = 0; i < 5; ++i) {
    Status s = core->wait(t[i], 0, nullptr, nullptr);
    done += s == kOk;
    canceled += s == kCanceled;
  }
  CHECK(done + canceled == 5 && canceled >= 3);
  delete core;
}

static void test_concurrent_clients() {
  FakeExec ex;
  Config cfg;
  cfg.arena_bytes = 8 * 64 * 64 * 16;
  cfg.max_inflight = 4;
  Core core(cfg, &ex);
  std::vector<std::thread> th;
  std::atomic<int> ok{0};
  for (int c = 0; c < 8; ++c)
    th.emplace_back([&] {
      for (int i = 0; i < 50; ++i) {
        uint64_t t;
        Status s;
        while ((s = core.submit(req(64, 64), &t)) == kBusy) std::this_thread::yield();
        CHECK(s == kOk);
        CHECK(core.wait(t, -1, nullptr, nullptr) == kOk);
        CHECK(core.release(t) == kOk);
        ++ok;
      }
    });
  for (auto &t : th) t.join();
  CHECK(ok == 400);
  CHECK(core.arena_used() == 0);
}

int main() {
  test_basic_completion();
  test_arena_backpressure_and_fifo();
  test_large_request_spans_steps_and_others_join();
  test_cancel_and_failures();
  test_shutdown();
  test_concurrent_clients();
  printf("serve_core: all tests passed\n");
  return 0;
}
