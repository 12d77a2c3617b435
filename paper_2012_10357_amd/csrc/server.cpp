// Continuous-batching render server.
//
// The paper's engine renders one scene per dispatch (Sec. 2.2.3).  For
// serving many users, requests of different scenes and resolutions arrive
// over time; this server keeps scenes and their BVHs resident, admits queued
// requests in arrival order while their output buffers fit an HBM budget,
// and launches every admitted request together as one persistent-kernel
// batch on a free stream -- while earlier batches are still running, so the
// tail of one batch overlaps the start of the next.  A request completes
// when its own pixels are done, not when its launch ends: the kernel counts
// each request's finished jobs on the device and sets a flag in pinned host
// memory once they are all done, which the scheduler thread polls (with the
// request's shadow and bounce ray counts beside it).
//
// The scheduler core is independent of HIP: it talks to an Executor, so the
// same admission, batching and accounting logic also runs against a
// simulated executor (no device) for host-side testing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>

#include "host_common.h"

namespace pr {
pr_status launch_prepared(const std::vector<ReqDev>& reqs, const std::vector<pr_scene*>& scenes,
                          uint32_t total_jobs, int step_budget, int compact, bool use_graph,
                          unsigned long long* counts_dev, hipStream_t stream, hipEvent_t done_evt,
                          unsigned long long* track_dev, DoneRec* done_host);
pr_status add_request(std::vector<ReqDev>& reqs, std::vector<pr_scene*>& scenes, pr_scene* s,
                      const pr_camera* cam, const pr_render_opts* o, uint32_t w, uint32_t h, float* rgb,
                      float* t, int32_t* inst, uint32_t tile_w_override, uint32_t& total_jobs,
                      bool check_ptrs);
int budget_for(const pr_scene* s, const pr_render_opts* o, uint32_t override_budget);
int compact_for(const pr_scene* s, const pr_render_opts* o, uint32_t override_pct);
}  // namespace pr

using namespace pr;

namespace {

using Clock = std::chrono::steady_clock;
double now_s() {
  return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing, 256-byte granules.
class PoolAlloc {
 public:
  explicit PoolAlloc(uint64_t size) : size_(size) { free_[0] = size; }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = (bytes + 255) & ~uint64_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        uint64_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        live_[*off] = bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off) {
    auto l = live_.find(off);
    if (l == live_.end()) return;
    uint64_t bytes = l->second;
    live_.erase(l);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  uint64_t size() const { return size_; }

 private:
  uint64_t size_, used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;
  std::map<uint64_t, uint64_t> live_;
};

struct Ticket {
  uint64_t id = 0;
  pr_request req{};
  uint64_t bytes = 0, off = 0;
  // several samples per pixel: colour accumulators and sample counters,
  // carved right after the outputs
  unsigned long long* sample_acc = nullptr;
  uint32_t* sample_cnt = nullptr;
  double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
  uint64_t rays_shadow = 0, rays_bounce = 0;
  int state = 0;  // 0 queued, 1 admitted, 2 launched, 3 done
  pr_status status = PR_OK;
  int slot = -1;
};

// What the scheduler needs from a device.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual pr_status init(uint64_t pool_bytes, uint32_t slots, uint32_t max_batch) = 0;
  virtual char* pool_base() = 0;
  // launch the given admitted tickets on slot; outputs already carved
  virtual pr_status launch(int slot, std::vector<Ticket*>& batch) = 0;
  virtual bool done(int slot) = 0;   // has the slot's last launch completed?
  // has request i of the slot's running launch completed?  (its ray counts)
  virtual bool request_done(int slot, size_t i, uint64_t* rays_shadow, uint64_t* rays_bounce) = 0;
  virtual void shutdown() = 0;
};

class HipExecutor : public Executor {
 public:
  explicit HipExecutor(int dev, bool graph) : dev_(dev), graph_(graph) {}
  pr_status init(uint64_t pool_bytes, uint32_t slots, uint32_t max_batch) override {
    hipError_t e = hipSetDevice(dev_);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((e = hipMalloc((void**)&pool_, pool_bytes)) != hipSuccess) return hip_fail(e, "hipMalloc(pool)");
    max_batch_ = max_batch;
    streams_.resize(slots);
    events_.resize(slots);
    track_.assign(slots, nullptr);
    done_.assign(slots, nullptr);
    for (uint32_t i = 0; i < slots; ++i) {
      if ((e = hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
      if ((e = hipEventCreateWithFlags(&events_[i], hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
      // per slot: device job and ray counters, host-visible completion records
      if ((e = hipMalloc((void**)&track_[i], (size_t)max_batch * 3 * sizeof(unsigned long long))) != hipSuccess)
        return hip_fail(e, "hipMalloc(request counters)");
      if ((e = hipHostMalloc((void**)&done_[i], (size_t)max_batch * sizeof(DoneRec), hipHostMallocDefault)) !=
          hipSuccess)
        return hip_fail(e, "hipHostMalloc(completion records)");
      std::memset(done_[i], 0, (size_t)max_batch * sizeof(DoneRec));
    }
    return PR_OK;
  }
  char* pool_base() override { return pool_; }
  pr_status launch(int slot, std::vector<Ticket*>& batch) override {
    const hipError_t de = hipSetDevice(dev_);
    if (de != hipSuccess) return hip_fail(de, "hipSetDevice");
    std::vector<ReqDev> reqs;
    std::vector<pr_scene*> scenes;
    uint32_t total = 0;
    for (Ticket* t : batch) {
      pr_status st = add_request(reqs, scenes, t->req.scene, &t->req.cam, &t->req.opts, t->req.width,
                                 t->req.height, t->req.out_rgb, t->req.out_t, t->req.out_inst, 0, total,
                                 false);
      if (st != PR_OK) return st;
      if (t->sample_acc) {
        // pool memory is reused: accumulators and counters must start at zero
        const size_t bytes = (size_t)((char*)(t->sample_cnt + (size_t)t->req.width * t->req.height) -
                                      (char*)t->sample_acc);
        hipError_t e = hipMemsetAsync(t->sample_acc, 0, bytes, streams_[slot]);
        if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(sample accumulators)");
        reqs.back().sample_acc = t->sample_acc;
        reqs.back().sample_cnt = t->sample_cnt;
      }
    }
    // the slot's previous launch has completed: reset its records and counters
    const size_t n = batch.size();
    for (size_t i = 0; i < n; ++i) __atomic_store_n(&done_[slot][i].done, 0u, __ATOMIC_RELAXED);
    hipError_t e = hipMemsetAsync(track_[slot], 0, n * 3 * sizeof(unsigned long long), streams_[slot]);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(request counters)");
    int budget = budget_for(scenes[0], nullptr, 0);
    return launch_prepared(reqs, scenes, total, budget, compact_for(scenes[0], nullptr, 0), graph_, nullptr,
                           streams_[slot], events_[slot], track_[slot], done_[slot]);
  }
  bool done(int slot) override { return hipEventQuery(events_[slot]) != hipErrorNotReady; }
  bool request_done(int slot, size_t i, uint64_t* sh, uint64_t* bo) override {
    const DoneRec& r = done_[slot][i];
    if (__atomic_load_n(&r.done, __ATOMIC_ACQUIRE) == 0u) return false;
    *sh = r.rays_shadow;
    *bo = r.rays_bounce;
    return true;
  }
  void shutdown() override {
    for (auto s : streams_) (void)hipStreamSynchronize(s);
    for (auto e : events_) (void)hipEventDestroy(e);
    for (auto s : streams_) (void)hipStreamDestroy(s);
    for (auto t : track_)
      if (t) (void)hipFree(t);
    for (auto d : done_)
      if (d) (void)hipHostFree(d);
    streams_.clear();
    events_.clear();
    track_.clear();
    done_.clear();
    if (pool_) (void)hipFree(pool_);
    pool_ = nullptr;
  }

 private:
  int dev_;
  bool graph_;
  char* pool_ = nullptr;
  uint32_t max_batch_ = 0;
  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> events_;
  std::vector<unsigned long long*> track_;
  std::vector<DoneRec*> done_;
};

// Simulated device: a launch completes after a time proportional to the
// pixels it renders; no memory is touched.  For host-side tests.
class SimExecutor : public Executor {
 public:
  explicit SimExecutor(uint32_t us_per_mpix) : us_per_mpix_(us_per_mpix) {}
  pr_status init(uint64_t, uint32_t slots, uint32_t) override {
    busy_until_.assign(slots, 0.0);
    return PR_OK;
  }
  char* pool_base() override { return reinterpret_cast<char*>(uintptr_t(1) << 40); }
  pr_status launch(int slot, std::vector<Ticket*>& batch) override {
    double px = 0;
    for (Ticket* t : batch) px += (double)t->req.width * t->req.height * t->req.opts.spp;
    busy_until_[slot] = now_s() + 20e-6 + px * 1e-6 * us_per_mpix_ * 1e-6;
    return PR_OK;
  }
  bool done(int slot) override { return now_s() >= busy_until_[slot]; }
  // a simulated launch completes all its requests together
  bool request_done(int, size_t, uint64_t*, uint64_t*) override { return false; }
  void shutdown() override {}

 private:
  uint32_t us_per_mpix_;
  std::vector<double> busy_until_;
};

}  // namespace

struct pr_server {
  pr_server_opts opts{};
  std::unique_ptr<Executor> exec;
  std::unique_ptr<PoolAlloc> pool;
  std::vector<pr_scene*> scenes;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<Ticket*> waiting;                     // FIFO, not yet admitted
  std::vector<Ticket*> admitted;                   // carved, not yet launched
  // per slot: tickets of its running launch, by request index; an entry is
  // cleared once that request has completed (it may then be released while
  // the launch still runs)
  std::vector<std::vector<Ticket*>> slot_batch;
  std::vector<bool> slot_busy;
  std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread thread;
  pr_server_stats stats{};

  uint64_t footprint(const pr_request& r) const {
    uint64_t px = (uint64_t)r.width * r.height;
    auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    uint64_t b = up(px * 12) + up(px * 4) + up(px * 4);
    if (r.opts.spp > 1) b += up(px * 24) + up(px * 4);
    return b;
  }

  void carve(Ticket* t) {
    char* base = exec->pool_base() + t->off;
    uint64_t px = (uint64_t)t->req.width * t->req.height;
    auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    t->req.out_rgb = reinterpret_cast<float*>(base);
    t->req.out_t = reinterpret_cast<float*>(base + up(px * 12));
    t->req.out_inst = reinterpret_cast<int32_t*>(base + up(px * 12) + up(px * 4));
    if (t->req.opts.spp > 1) {
      char* sb = base + up(px * 12) + up(px * 4) + up(px * 4);
      t->sample_acc = reinterpret_cast<unsigned long long*>(sb);
      t->sample_cnt = reinterpret_cast<uint32_t*>(sb + up(px * 24));
    }
  }

  void finish(Ticket* tk, double t) {
    tk->t_done = t;
    tk->state = 3;
    ++stats.completed;
  }

  void loop() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      bool progressed = false;
      // 1. completions: requests whose device flag is set, then whole launches
      for (size_t s = 0; s < slot_batch.size(); ++s) {
        if (!slot_busy[s]) continue;
        bool any = false;
        for (size_t i = 0; i < slot_batch[s].size(); ++i) {
          Ticket* tk = slot_batch[s][i];
          if (tk && exec->request_done((int)s, i, &tk->rays_shadow, &tk->rays_bounce)) {
            finish(tk, now_s());
            slot_batch[s][i] = nullptr;
            any = true;
          }
        }
        if (exec->done((int)s)) {
          const double t = now_s();
          for (size_t i = 0; i < slot_batch[s].size(); ++i) {
            Ticket* tk = slot_batch[s][i];
            if (!tk) continue;
            // the launch has ended: its records are final
            (void)exec->request_done((int)s, i, &tk->rays_shadow, &tk->rays_bounce);
            finish(tk, t);
          }
          slot_batch[s].clear();
          slot_busy[s] = false;
          any = true;
        }
        if (any) {
          progressed = true;
          cv_done.notify_all();
        }
      }
      // 2. admission: FIFO while the head fits the pool (no skipping: no starvation)
      while (!waiting.empty()) {
        Ticket* t = waiting.front();
        uint64_t off;
        if (!pool->alloc(t->bytes, &off)) break;
        waiting.pop_front();
        t->off = off;
        carve(t);
        t->t_admit = now_s();
        t->state = 1;
        admitted.push_back(t);
        ++stats.admitted;
        progressed = true;
      }
      stats.pool_bytes_in_use = pool->used();
      stats.pool_bytes_peak = pool->peak();
      // 3. launch everything admitted on a free slot, in batches of max_batch
      while (!admitted.empty()) {
        int free_slot = -1;
        for (size_t s = 0; s < slot_batch.size(); ++s)
          if (!slot_busy[s]) {
            free_slot = (int)s;
            break;
          }
        if (free_slot < 0) break;
        size_t n = std::min<size_t>(admitted.size(), opts.max_batch);
        std::vector<Ticket*> batch(admitted.begin(), admitted.begin() + n);
        admitted.erase(admitted.begin(), admitted.begin() + n);
        // smallest first within the launch: the job queue hands out requests
        // in table order, and each request completes on its own, so the small
        // ones finish early instead of behind a large one
        std::stable_sort(batch.begin(), batch.end(), [](const Ticket* a, const Ticket* b) {
          return (uint64_t)a->req.width * a->req.height * a->req.opts.spp <
                 (uint64_t)b->req.width * b->req.height * b->req.opts.spp;
        });
        double t = now_s();
        pr_status st = exec->launch(free_slot, batch);
        ++stats.launches;
        for (Ticket* tk : batch) {
          tk->t_launch = t;
          tk->slot = free_slot;
          if (st != PR_OK) {
            tk->status = st;
            tk->state = 3;
            tk->t_done = t;
            ++stats.completed;
          } else {
            tk->state = 2;
          }
        }
        if (st == PR_OK) {
          slot_batch[free_slot] = batch;
          slot_busy[free_slot] = true;
        } else {
          cv_done.notify_all();
        }
        progressed = true;
      }
      bool inflight = false;
      for (size_t s = 0; s < slot_busy.size(); ++s) inflight = inflight || slot_busy[s];
      if (stop && waiting.empty() && admitted.empty() && !inflight) break;
      if (!progressed) {
        // poll running launches every 20 us; sleep until a submit otherwise
        if (inflight || !admitted.empty())
          cv_sched.wait_for(lk, std::chrono::microseconds(20));
        else
          cv_sched.wait_for(lk, std::chrono::milliseconds(50));
      }
    }
  }
};

namespace {

pr_status create_server(const pr_server_opts* o, std::unique_ptr<Executor> exec, pr_server** out) {
  if (!o || !out) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  if (o->hbm_budget_bytes < 4096) return set_error(PR_ERR_INVALID_ARG, "hbm_budget_bytes too small");
  if (o->max_inflight < 1 || o->max_inflight > 8) return set_error(PR_ERR_INVALID_ARG, "max_inflight must be 1..8");
  if (o->max_batch < 1 || o->max_batch > 4096) return set_error(PR_ERR_INVALID_ARG, "max_batch must be 1..4096");
  auto* s = new pr_server();
  s->opts = *o;
  s->exec = std::move(exec);
  pr_status st = s->exec->init(o->hbm_budget_bytes, o->max_inflight, o->max_batch);
  if (st != PR_OK) {
    s->exec->shutdown();
    delete s;
    return st;
  }
  s->pool = std::make_unique<PoolAlloc>(o->hbm_budget_bytes);
  s->slot_batch.resize(o->max_inflight);
  s->slot_busy.assign(o->max_inflight, false);
  s->thread = std::thread([s] { s->loop(); });
  *out = s;
  return ok();
}

}  // namespace

extern "C" {

pr_status pr_server_create(const pr_server_opts* o, pr_server** out) {
  try {
    if (!o) return set_error(PR_ERR_INVALID_ARG, "opts is NULL");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || (int)o->device >= n)
      return set_error(PR_ERR_DEVICE, "device %u not available", o->device);
    return create_server(o, std::make_unique<HipExecutor>((int)o->device, o->use_graph != 0), out);
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

pr_status pr_server_create_simulated(const pr_server_opts* o, uint32_t us_per_mpix, pr_server** out) {
  try {
    return create_server(o, std::make_unique<SimExecutor>(us_per_mpix), out);
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

pr_status pr_server_add_scene(pr_server* srv, pr_scene* scene, uint32_t* slot) {
  if (!srv || !scene) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  if (!scene->built) return set_error(PR_ERR_NOT_BUILT, "scene BVH not built");
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->scenes.push_back(scene);
  if (slot) *slot = (uint32_t)srv->scenes.size() - 1;
  return ok();
}

pr_status pr_server_submit(pr_server* srv, const pr_request* req, uint64_t* ticket) {
  try {
    if (!srv || !req || !ticket) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      if (std::find(srv->scenes.begin(), srv->scenes.end(), req->scene) == srv->scenes.end())
        return set_error(PR_ERR_INVALID_ARG, "request scene is not registered with this server");
    }
    // validate everything but the output pointers (the server owns those)
    std::vector<ReqDev> tmp;
    std::vector<pr_scene*> tmps;
    uint32_t total = 0;
    float dummy;
    bool sim = dynamic_cast<SimExecutor*>(srv->exec.get()) != nullptr;
    if (!sim) {
      pr_status st = add_request(tmp, tmps, req->scene, &req->cam, &req->opts, req->width, req->height,
                                 &dummy, nullptr, nullptr, 0, total, false);
      if (st != PR_OK) return st;
    } else if (req->width < 1 || req->height < 1 || req->width > 16384 || req->height > 16384 ||
               req->opts.spp < 1 || req->opts.spp > 64) {
      return set_error(PR_ERR_INVALID_ARG, "bad request size");
    }
    auto t = std::make_unique<Ticket>();
    t->req = *req;
    t->bytes = srv->footprint(*req);
    if (t->bytes > srv->opts.hbm_budget_bytes) {
      std::lock_guard<std::mutex> lk(srv->mu);
      ++srv->stats.rejected;
      return set_error(PR_ERR_OUT_OF_MEMORY, "request needs %llu bytes, budget is %llu",
                       (unsigned long long)t->bytes, (unsigned long long)srv->opts.hbm_budget_bytes);
    }
    t->t_submit = now_s();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return set_error(PR_ERR_BUSY, "server is shutting down");
    t->id = srv->next_ticket++;
    *ticket = t->id;
    srv->waiting.push_back(t.get());
    srv->tickets.emplace(t->id, std::move(t));
    ++srv->stats.submitted;
    srv->cv_sched.notify_one();
    return ok();
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

pr_status pr_server_wait(pr_server* srv, uint64_t ticket, uint32_t timeout_ms, pr_request_result* out) {
  if (!srv || !out) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return set_error(PR_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  Ticket* t = it->second.get();
  bool ok_ = srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [t] { return t->state == 3; });
  if (!ok_) return set_error(PR_ERR_TIMEOUT, "ticket %llu not done after %u ms", (unsigned long long)ticket, timeout_ms);
  out->status = t->status;
  out->rgb = t->req.out_rgb;
  out->t = t->req.out_t;
  out->inst = t->req.out_inst;
  out->width = t->req.width;
  out->height = t->req.height;
  out->t_submit = t->t_submit;
  out->t_admit = t->t_admit;
  out->t_launch = t->t_launch;
  out->t_done = t->t_done;
  out->rays_primary = (uint64_t)t->req.width * t->req.height * t->req.opts.spp;
  out->rays_shadow = t->rays_shadow;
  out->rays_bounce = t->rays_bounce;
  out->user_tag = t->req.user_tag;
  if (t->status != PR_OK) return set_error(t->status, "request failed");
  return ok();
}

pr_status pr_server_release(pr_server* srv, uint64_t ticket) {
  if (!srv) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return set_error(PR_ERR_INVALID_ARG, "unknown ticket");
  Ticket* t = it->second.get();
  if (t->state != 3) return set_error(PR_ERR_BUSY, "ticket still in flight");
  if (t->state >= 1) srv->pool->release(t->off);
  srv->tickets.erase(it);
  srv->stats.pool_bytes_in_use = srv->pool->used();
  srv->cv_sched.notify_one();   // freed memory may admit waiting requests
  return ok();
}

pr_status pr_server_stats_get(pr_server* srv, pr_server_stats* out) {
  if (!srv || !out) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  out->pool_bytes_in_use = srv->pool->used();
  out->pool_bytes_peak = srv->pool->peak();
  return ok();
}

pr_status pr_server_destroy(pr_server* srv) {
  if (!srv) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_sched.notify_one();
  }
  if (srv->thread.joinable()) srv->thread.join();
  srv->exec->shutdown();
  delete srv;
  return ok();
}

}  // extern "C"
