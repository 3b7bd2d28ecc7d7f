// Render server: the C ABI over the continuous-batching scheduler
// (serve_core.h) with a GPU executor. Every step is one persistent launch of
// k_render_step per (storage format, lookup, component class) group over the
// tile ranges of that group's scheduled requests, whatever their scene; each
// group's launch and the copy of its descriptor table are captured once into a
// HIP graph and replayed each step on the group's own stream.
#include <string.h>

#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <vector>

#include "fastnerf.h"
#include "fastnerf_internal.h"
#include "fastnerf_kernels.h"
#include "serve_core.h"

using namespace fnr;
namespace fs = fnr_serve;

namespace {

#define HIP_CHECK(call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #call);    \
  } while (0)

// Device image of a step: header {tiles, views} then the views.
struct StepHeader {
  int total;
  int nviews;
  int pad[2];
};

class GpuExecutor : public fs::Executor {
 public:
  GpuExecutor() {}
  ~GpuExecutor() override { free_all(); }

  fastnerf_status init(const std::vector<fastnerf_cache_s *> &scenes, int max_views,
                       uint8_t *arena) {
    scenes_ = scenes;
    max_views_ = max_views;
    arena_ = arena;
    std::vector<DevCache> dc;
    for (auto *c : scenes) dc.push_back(dev_cache(c));
    HIP_CHECK(hipMalloc(&caches_, sizeof(DevCache) * dc.size()));
    HIP_CHECK(hipMemcpy(caches_, dc.data(), sizeof(DevCache) * dc.size(), hipMemcpyHostToDevice));
    table_bytes_ = sizeof(StepHeader) + sizeof(DevView) * (size_t)max_views;
    int cus = 1;
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    cus_ = cus < 1 ? 1 : cus;
    return FASTNERF_OK;
  }

  fs::Status run(const fs::Step &step, uint64_t) override {
    const fs::Status st = launch(step, 0);
    return st == fs::kOk ? wait(0) : st;
  }

  // Enqueues the step's launches with the descriptor tables of slot `slot`
  // (0 or 1: the scheduler alternates them and waits for a slot before it
  // reuses it, so the pinned table of a step in flight is never rewritten).
  // Each group runs on its own stream, so one group's tail overlaps the other
  // groups' work; a group's steps stay in order on its stream.
  fs::Status launch(const fs::Step &step, int slot) override {
    slot &= 1;
    // one launch per (format, interpolation, component-count) group present
    std::map<int, std::vector<const fs::Segment *>> groups;
    for (const auto &sg : step.segs) {
      const fastnerf_cache_s *c = scenes_[sg.req->scene];
      groups[group_key(c)].push_back(&sg);
    }
    std::vector<Group *> &launched = launched_[slot];
    launched.clear();
    // on a failure the step's requests are failed and their memory may be
    // reused: the groups already launched finish first
    auto fail = [&launched]() {
      for (Group *x : launched) (void)hipStreamSynchronize(x->stream);
      launched.clear();
      return fs::kDevice;
    };
    for (auto &kv : groups) {
      Group *g = nullptr;
      if (group(kv.first, &g) != FASTNERF_OK) return fail();
      StepHeader *hh = reinterpret_cast<StepHeader *>(g->h_table[slot]);
      DevView *hv = reinterpret_cast<DevView *>(g->h_table[slot] + sizeof(StepHeader));
      int tb = 0, n = 0;
      std::set<int> used;
      for (const fs::Segment *sg : kv.second) {
        const fs::Request *r = sg->req;
        fastnerf_cache_s *c = scenes_[r->scene];
        make_view(c, r->K, r->c2w, r->H, r->W, r->near_, r->far_,
                  reinterpret_cast<float *>(arena_ + r->off), tb, hv + n);
        hv[n].tile_offset = sg->first;
        hv[n].scene = r->scene;
        hv[n].N = r->N;
        hv[n].lim = eps_limit(r->eps);
        tb += sg->count;
        ++n;
        used.insert(r->scene);
      }
      hh->total = tb;
      hh->nviews = n;
      launched.push_back(g);
      if (hipGraphLaunch(g->exec[slot], g->stream) != hipSuccess) return fail();
      // each scene's last use, once per step (a marker per request segment had
      // put up to max_inflight packets between the step's kernels)
      for (int sc : used)
        if (hipEventRecord(scenes_[sc]->last_use, g->stream) != hipSuccess) return fail();
      if (hipEventRecord(g->done[slot], g->stream) != hipSuccess) return fail();
    }
    return fs::kOk;
  }

  // Waits for every group of the slot's step, also after one of them failed.
  fs::Status wait(int slot) override {
    fs::Status st = fs::kOk;
    for (Group *g : launched_[slot & 1])
      if (hipEventSynchronize(g->done[slot & 1]) != hipSuccess) st = fs::kDevice;
    return st;
  }

 private:
  // Per group: its stream, a pinned descriptor table, a captured graph (table
  // copy, then the step kernel) and an end-of-launch event for each of the two
  // slots; the device table and the queue counters are shared by the slots,
  // since the group's steps run in order on its stream.
  struct Group {
    hipStream_t stream = nullptr;
    hipEvent_t done[2] = {nullptr, nullptr};    // end of the group's last launch in each slot
    uint8_t *h_table[2] = {nullptr, nullptr};  // pinned
    uint8_t *d_table = nullptr;
    unsigned *counter = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
  };

  // (storage format, interpolation, component-count class): each has its own
  // step kernel (the class fixes the record layout)
  static int group_key(const fastnerf_cache_s *c) {
    return (int)c->desc.storage * 8 + (c->desc.pos_interp == FASTNERF_LINEAR ? 4 : 0) +
           maxd_class(c->desc.D) / 8;
  }

  fastnerf_status group(int key, Group **out) {
    auto it = groups_.find(key);
    if (it != groups_.end()) {
      *out = it->second.get();
      return FASTNERF_OK;
    }
    std::unique_ptr<Group> g(new Group());
    const fastnerf_status st = build_group(key, g.get());
    if (st != FASTNERF_OK) {
      destroy_group(g.get());
      return st;
    }
    *out = g.get();
    groups_[key] = std::move(g);
    return FASTNERF_OK;
  }

  fastnerf_status build_group(int key, Group *g) {
    HIP_CHECK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
      HIP_CHECK(hipEventCreateWithFlags(&g->done[k], hipEventDisableTiming));
      HIP_CHECK(hipHostMalloc(&g->h_table[k], table_bytes_, hipHostMallocDefault));
      memset(g->h_table[k], 0, table_bytes_);
    }
    HIP_CHECK(hipMalloc(&g->d_table, table_bytes_));
    HIP_CHECK(hipMalloc(&g->counter, kQueueCounters * sizeof(unsigned)));
    // cleared on the group's stream, ahead of every launch of its graphs
    HIP_CHECK(hipMemsetAsync(g->counter, 0, kQueueCounters * sizeof(unsigned), g->stream));
    const int fmt = key >> 3;
    const bool lin = key & 4;
    const int D = (key & 3) == 0 ? 4 : ((key & 3) == 1 ? 8 : 16);
    const int grid = cus_ * render_step_occupancy(fmt, lin, D);
    RenderArgs a;
    memset(&a, 0, sizeof a);
    a.views = reinterpret_cast<const DevView *>(g->d_table + sizeof(StepHeader));
    a.dyn_total = reinterpret_cast<const int *>(g->d_table);
    a.caches = caches_;
    a.counter = g->counter;
    a.nwaves = (unsigned)grid * (kBlock / kWave);
    for (int k = 0; k < 2; ++k) {
      HIP_CHECK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipMemcpyAsync(g->d_table, g->h_table[k], table_bytes_,
                                    hipMemcpyHostToDevice, g->stream);
      if (e == hipSuccess) e = launch_render_step(fmt, lin, D, a, grid, g->stream);
      hipError_t e2 = hipStreamEndCapture(g->stream, &g->graph[k]);
      if (e != hipSuccess) return hip_fail(e, "step capture");
      if (e2 != hipSuccess) return hip_fail(e2, "end capture");
      HIP_CHECK(hipGraphInstantiate(&g->exec[k], g->graph[k], nullptr, nullptr, 0));
    }
    return FASTNERF_OK;
  }

  static void destroy_group(Group *g) {
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (int k = 0; k < 2; ++k) {
      if (g->exec[k]) (void)hipGraphExecDestroy(g->exec[k]);
      if (g->graph[k]) (void)hipGraphDestroy(g->graph[k]);
      if (g->h_table[k]) (void)hipHostFree(g->h_table[k]);
      if (g->done[k]) (void)hipEventDestroy(g->done[k]);
    }
    if (g->d_table) (void)hipFree(g->d_table);
    if (g->counter) (void)hipFree(g->counter);
    if (g->stream) (void)hipStreamDestroy(g->stream);
  }

  void free_all() {
    for (auto &kv : groups_) destroy_group(kv.second.get());
    groups_.clear();
    if (caches_) (void)hipFree(caches_);
    caches_ = nullptr;
  }

  std::vector<fastnerf_cache_s *> scenes_;
  int max_views_ = 0, cus_ = 1;
  size_t table_bytes_ = 0;
  uint8_t *arena_ = nullptr;
  DevCache *caches_ = nullptr;
  std::map<int, std::unique_ptr<Group>> groups_;
  std::vector<Group *> launched_[2];  // groups launched in each slot's last step
};

}  // namespace

struct fastnerf_server_s {
  std::vector<fastnerf_cache_s *> scenes;
  uint8_t *arena = nullptr;
  GpuExecutor exec;
  std::unique_ptr<fs::Core> core;
};

static fastnerf_status from_core(fs::Status s, const char *what) {
  if (s == fs::kOk) return FASTNERF_OK;
  return fail((fastnerf_status)s, "%s", what);
}

extern "C" fastnerf_status fastnerf_server_create(const fastnerf_cache *scenes, int32_t nscenes,
                                                  uint64_t arena_bytes, int32_t max_inflight,
                                                  fastnerf_server *out) {
  if (!scenes || nscenes < 1 || !out) return fail(FASTNERF_EINVAL, "no scenes or null out");
  if (max_inflight < 1 || max_inflight > 4096)
    return fail(FASTNERF_EINVAL, "max_inflight = %d outside [1, 4096]", max_inflight);
  if (arena_bytes == 0) {
    // admission by the device's free memory: the arena takes a quarter of
    // what is free now (the scenes are resident already)
    size_t free_b = 0, total_b = 0;
    const hipError_t me = hipMemGetInfo(&free_b, &total_b);
    if (me != hipSuccess) return hip_fail(me, "free device memory");
    arena_bytes = (uint64_t)(free_b / 4) & ~(uint64_t)255;
  }
  if (arena_bytes < 256) return fail(FASTNERF_EINVAL, "arena too small");
  for (int i = 0; i < nscenes; ++i)
    if (!scenes[i] || !scenes[i]->finalized)
      return fail(FASTNERF_EINVAL, "scene %d is null or not finalized", i);
  std::unique_ptr<fastnerf_server_s> s(new (std::nothrow) fastnerf_server_s());
  if (!s) return fail(FASTNERF_ENOMEM, "host allocation");
  s->scenes.assign(scenes, scenes + nscenes);
  hipError_t e = hipMalloc(&s->arena, arena_bytes);
  if (e != hipSuccess) return hip_fail(e, "arena");
  fastnerf_status st = s->exec.init(s->scenes, max_inflight, s->arena);
  if (st != FASTNERF_OK) {
    (void)hipFree(s->arena);
    return st;
  }
  fs::Config cfg;
  cfg.arena_bytes = arena_bytes;
  cfg.max_inflight = max_inflight;
  s->core.reset(new fs::Core(cfg, &s->exec));
  *out = s.release();
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_serve_submit(fastnerf_server s, int32_t scene,
                                                 const float K[9], const float c2w[12],
                                                 int32_t H, int32_t W, float near_, float far_,
                                                 int32_t N, float eps, uint64_t *ticket) {
  if (!s || !ticket) return fail(FASTNERF_EINVAL, "null server or ticket");
  if (scene < 0 || scene >= (int)s->scenes.size())
    return fail(FASTNERF_EINVAL, "scene %d out of range", scene);
  static const float dummy = 0.0f;
  fastnerf_status st = check_view(K, c2w, H, W, near_, far_, &dummy);
  if (st == FASTNERF_OK) st = check_render_params(N, eps);
  if (st == FASTNERF_OK && N == 0)
    st = fail(FASTNERF_EINVAL, "serving renders N >= 1 samples per ray");
  if (st != FASTNERF_OK) return st;
  std::unique_ptr<fs::Request> r(new fs::Request());
  r->scene = scene;
  memcpy(r->K, K, sizeof r->K);
  memcpy(r->c2w, c2w, sizeof r->c2w);
  r->H = H;
  r->W = W;
  r->near_ = near_;
  r->far_ = far_;
  r->N = N;
  r->eps = eps;
  r->bytes = (uint64_t)H * W * 4 * sizeof(float);
  return from_core(s->core->submit(std::move(r), ticket), "submit");
}

extern "C" fastnerf_status fastnerf_serve_wait(fastnerf_server s, uint64_t ticket,
                                               int64_t timeout_us, const float **out_device,
                                               double *latency_ms) {
  if (!s) return fail(FASTNERF_EINVAL, "null server");
  uint64_t off = 0;
  fs::Status r = s->core->wait(ticket, timeout_us, &off, latency_ms);
  if (r == fs::kOk && out_device) *out_device = reinterpret_cast<const float *>(s->arena + off);
  return from_core(r, "wait");
}

extern "C" fastnerf_status fastnerf_serve_release(fastnerf_server s, uint64_t ticket) {
  if (!s) return fail(FASTNERF_EINVAL, "null server");
  return from_core(s->core->release(ticket), "release");
}

extern "C" fastnerf_status fastnerf_serve_cancel(fastnerf_server s, uint64_t ticket) {
  if (!s) return fail(FASTNERF_EINVAL, "null server");
  return from_core(s->core->cancel(ticket), "cancel");
}

extern "C" fastnerf_status fastnerf_server_stats(fastnerf_server s, uint64_t *steps,
                                                 uint64_t *completed, uint64_t *max_batch) {
  if (!s) return fail(FASTNERF_EINVAL, "null server");
  s->core->stats(steps, completed, max_batch);
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_server_destroy(fastnerf_server s) {
  if (!s) return fail(FASTNERF_EINVAL, "null server");
  s->core->shutdown();
  s->core.reset();
  s->exec.~GpuExecutor();
  new (&s->exec) GpuExecutor();
  if (s->arena) (void)hipFree(s->arena);
  delete s;
  return FASTNERF_OK;
}
