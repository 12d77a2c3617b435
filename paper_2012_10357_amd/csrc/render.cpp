// Render, batch, counting and autotuning entry points.
//
// A frame is one dispatch over all pixels (Sec. 2.2.3: DispatchRays starts
// the ray-generation shader).  Here every launch -- one request or a batch of
// many -- is the same persistent kernel reading a table of requests and
// popping pixel jobs from a device queue; the table and the queue header are
// written by a single host-to-device copy from pinned staging, so a launch is
// (copy, kernel) on the caller's stream and can be captured in a hipGraph.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "host_common.h"

using namespace pr;

namespace pr {

static std::mutex g_ctx_mu;
static std::vector<LaunchCtx*> g_ctx;

LaunchCtx* acquire_ctx(uint32_t n_req) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  for (LaunchCtx* c : g_ctx) {
    if (c->in_use || c->device != dev || c->capacity < n_req) continue;
    if (hipEventQuery(c->done) == hipErrorNotReady) continue;
    c->in_use = true;
    return c;
  }
  auto* c = new LaunchCtx();
  c->capacity = std::max<uint32_t>(n_req, 64);
  c->bytes = sizeof(QueueDev) + (size_t)c->capacity * sizeof(ReqDev);
  c->device = dev;
  if (hipMalloc(&c->dev, c->bytes) != hipSuccess) {
    delete c;
    return nullptr;
  }
  if (hipHostMalloc(&c->host, c->bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(c->dev);
    delete c;
    return nullptr;
  }
  if (hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(c->dev);
    (void)hipHostFree(c->host);
    delete c;
    return nullptr;
  }
  c->in_use = true;
  g_ctx.push_back(c);
  return c;
}

void release_ctx(LaunchCtx* c) {
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  c->in_use = false;
}

}  // namespace pr

namespace {

// Launch parameters per scene size class.  Without an autotuned entry: 8x8
// tiles and bursts of at most 24 march steps (measured best single setting
// over a four-primitive 1080p frame and 1024-instance frames; 64 or more
// steps delay the refills and priority updates that the longest pixels need).
struct Tuned {
  uint32_t tile_w = 8, step_budget = 24;
  uint32_t compact = 0;   // 0 = no regrouping, 1..100 = threshold
};

std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tuned;
bool g_tune_loaded = false;

std::string size_class(const pr_scene* s) {
  // scenes are grouped by instance-count decade and the set of primitive types present
  uint32_t n = s->consts.n_inst;
  int dec = 0;
  while (n >= 10) {
    n /= 10;
    ++dec;
  }
  std::ostringstream os;
  os << "n1e" << dec << "_t" << s->n_types_present;
  return os.str();
}

void load_tune_cache() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("PR_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  // minimal format: {"key": [tile_w, step_budget, compact_pct], ...}
  std::string all((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  size_t p = 0;
  while ((p = all.find('"', p)) != std::string::npos) {
    size_t q = all.find('"', p + 1);
    if (q == std::string::npos) break;
    std::string key = all.substr(p + 1, q - p - 1);
    size_t lb = all.find('[', q), rb = all.find(']', q);
    if (lb == std::string::npos || rb == std::string::npos) break;
    Tuned t;
    if (std::sscanf(all.c_str() + lb, "[%u , %u , %u]", &t.tile_w, &t.step_budget, &t.compact) >= 2 ||
        std::sscanf(all.c_str() + lb, "[%u,%u,%u]", &t.tile_w, &t.step_budget, &t.compact) >= 2) {
      if (t.compact > 100) t.compact = 0;
      g_tuned[key] = t;
    }
    p = rb + 1;
  }
}

void save_tune_cache() {
  const char* path = std::getenv("PR_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream f(path);
  f << "{";
  bool first = true;
  for (auto& kv : g_tuned) {
    f << (first ? "" : ", ") << "\"" << kv.first << "\": [" << kv.second.tile_w << ", "
      << kv.second.step_budget << ", " << kv.second.compact << "]";
    first = false;
  }
  f << "}\n";
}

Tuned tuned_for(const pr_scene* s) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_cache();
  auto it = g_tuned.find(size_class(s));
  return it == g_tuned.end() ? Tuned{} : it->second;
}

pr_status validate_camera(const pr_camera* c) {
  if (!c) return set_error(PR_ERR_INVALID_ARG, "camera is NULL");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c->eye[i]) || !std::isfinite(c->target[i]) || !std::isfinite(c->up[i]))
      return set_error(PR_ERR_INVALID_ARG, "non-finite camera");
  double f[3] = {(double)c->target[0] - c->eye[0], (double)c->target[1] - c->eye[1],
                 (double)c->target[2] - c->eye[2]};
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0)) return set_error(PR_ERR_INVALID_ARG, "camera eye == target");
  double u[3] = {c->up[0], c->up[1], c->up[2]};
  double cx = u[1] * f[2] - u[2] * f[1], cy = u[2] * f[0] - u[0] * f[2], cz = u[0] * f[1] - u[1] * f[0];
  double ul = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (!(std::sqrt(cx * cx + cy * cy + cz * cz) > 1e-6 * fl * ul))
    return set_error(PR_ERR_INVALID_ARG, "camera up is parallel to the view direction");
  if (!(c->vfov_deg > 0 && c->vfov_deg < 180)) return set_error(PR_ERR_INVALID_ARG, "vfov must be in (0, 180)");
  return PR_OK;
}

pr_status validate_opts(const pr_render_opts* o, uint32_t w, uint32_t h) {
  if (!o) return set_error(PR_ERR_INVALID_ARG, "opts is NULL");
  if (w < 1 || h < 1 || w > 16384 || h > 16384)
    return set_error(PR_ERR_INVALID_ARG, "width and height must be in 1..16384");
  if (o->spp < 1 || o->spp > 64) return set_error(PR_ERR_INVALID_ARG, "spp must be in 1..64");
  if (o->max_steps < 1 || o->max_steps > 4096) return set_error(PR_ERR_INVALID_ARG, "max_steps must be in 1..4096");
  if (!(o->eps > 0) || !std::isfinite(o->eps)) return set_error(PR_ERR_INVALID_ARG, "eps must be > 0");
  if (!(o->tmin >= 0) || !(o->tmin < o->tmax) || !std::isfinite(o->tmax))
    return set_error(PR_ERR_INVALID_ARG, "need 0 <= tmin < tmax < inf");
  if (!(o->shadow_offset >= 0) || !std::isfinite(o->shadow_offset))
    return set_error(PR_ERR_INVALID_ARG, "shadow_offset must be >= 0");
  if (!(o->fd_h > 0) || !std::isfinite(o->fd_h)) return set_error(PR_ERR_INVALID_ARG, "fd_h must be > 0");
  if (o->bounces > 1) return set_error(PR_ERR_UNSUPPORTED, "at most one mirror bounce");
  if (o->shadows > 1 || o->jitter > 1) return set_error(PR_ERR_INVALID_ARG, "shadows and jitter are 0 or 1");
  if ((o->tile_w == 0) != (o->tile_h == 0))
    return set_error(PR_ERR_INVALID_ARG, "tile_w and tile_h are both 0 or both set");
  if (o->tile_w && (o->tile_w * o->tile_h != 64 || (64 % o->tile_w) != 0))
    return set_error(PR_ERR_INVALID_ARG, "tile_w * tile_h must be 64");
  if (o->step_budget > 4096) return set_error(PR_ERR_INVALID_ARG, "step_budget must be <= 4096");
  if (o->flags & ~PR_RENDER_NATURAL_ORDER) return set_error(PR_ERR_INVALID_ARG, "unknown render flags");
  if (o->compact_pct > 100 && o->compact_pct != PR_COMPACT_NEVER)
    return set_error(PR_ERR_INVALID_ARG, "compact_pct must be 0, 1..100 or PR_COMPACT_NEVER");
  if (o->reserved != 0) return set_error(PR_ERR_INVALID_ARG, "reserved must be 0");
  return PR_OK;
}

pr_status check_device_ptr(const void* p, size_t bytes, const char* name, int dev) {
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(PR_ERR_INVALID_ARG, "%s is not a device pointer", name);
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return set_error(PR_ERR_INVALID_ARG, "%s is not device memory", name);
  if (a.device != dev) return set_error(PR_ERR_INVALID_ARG, "%s lives on another device", name);
  (void)bytes;
  return PR_OK;
}

// Scheduling hint: the tile rectangle covering the screen projection of the
// iterative fractals' world AABBs.  Their pixels carry the longest sphere-
// tracing chains, which bound a frame's time once the job queue runs dry, so
// the kernel hands these tiles out first.  Left empty (row-major order) for
// scenes with many instances, where the rectangle would cover the screen, for
// boxes reaching behind the camera, and on request.
void first_region(ReqDev& r, const pr_scene* s, const pr_camera* cam, const pr_render_opts* o, uint32_t w,
                  uint32_t h, uint32_t tile_w) {
  r.first_x0 = r.first_y0 = r.first_x1 = r.first_y1 = 0;
  if ((o->flags & PR_RENDER_NATURAL_ORDER) || s->consts.n_inst > 256) return;
  double f[3], up[3], rt[3], u[3], eye[3];
  for (int i = 0; i < 3; ++i) {
    eye[i] = cam->eye[i];
    f[i] = (double)cam->target[i] - cam->eye[i];
    up[i] = cam->up[i];
  }
  auto norm = [](double* v) {
    const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; ++i) v[i] /= l;
  };
  norm(f);
  rt[0] = up[1] * f[2] - up[2] * f[1];
  rt[1] = up[2] * f[0] - up[0] * f[2];
  rt[2] = up[0] * f[1] - up[1] * f[0];
  norm(rt);
  u[0] = f[1] * rt[2] - f[2] * rt[1];
  u[1] = f[2] * rt[0] - f[0] * rt[2];
  u[2] = f[0] * rt[1] - f[1] * rt[0];
  const double sh = std::tan((double)cam->vfov_deg * M_PI / 360.0), aspect = (double)w / h;
  double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  bool any = false;
  for (uint32_t i = 0; i < s->consts.n_inst; ++i) {
    const uint32_t ty = s->host_insts[i].type;
    if (ty != PR_JULIA && ty != PR_MANDELBULB) continue;
    any = true;
    const float* b = &s->world_aabb[6 * (size_t)i];
    for (int c = 0; c < 8; ++c) {
      const double p[3] = {(c & 1) ? b[3] : b[0], (c & 2) ? b[4] : b[1], (c & 4) ? b[5] : b[2]};
      const double v[3] = {p[0] - eye[0], p[1] - eye[1], p[2] - eye[2]};
      const double z = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
      if (!(z > 1e-6)) return;   // reaches behind the camera: keep row-major order
      const double sx = (v[0] * rt[0] + v[1] * rt[1] + v[2] * rt[2]) / z / (sh * aspect);
      const double sy = (v[0] * u[0] + v[1] * u[1] + v[2] * u[2]) / z / sh;
      const double px = (sx + 1.0) * 0.5 * w, py = (1.0 - sy) * 0.5 * h;
      x0 = std::min(x0, px);
      x1 = std::max(x1, px);
      y0 = std::min(y0, py);
      y1 = std::max(y1, py);
    }
  }
  if (!any) return;
  const uint32_t th = 64 / tile_w, tiles_y = (h + th - 1) / th;
  auto clampi = [](double v, uint32_t hi) -> uint32_t {
    return v <= 0.0 ? 0u : (v >= (double)hi ? hi : (uint32_t)v);
  };
  const uint32_t tx0 = clampi(std::floor(x0 / tile_w), r.tiles_x), tx1 = clampi(std::ceil(x1 / tile_w), r.tiles_x);
  const uint32_t ty0 = clampi(std::floor(y0 / th), tiles_y), ty1 = clampi(std::ceil(y1 / th), tiles_y);
  if (tx0 >= tx1 || ty0 >= ty1) return;
  if (tx0 == 0 && ty0 == 0 && tx1 == r.tiles_x && ty1 == tiles_y) return;   // the whole frame
  r.first_x0 = (uint16_t)tx0;
  r.first_y0 = (uint16_t)ty0;
  r.first_x1 = (uint16_t)tx1;
  r.first_y1 = (uint16_t)ty1;
}

void fill_req(ReqDev& r, const pr_scene* s, const pr_camera* cam, const pr_render_opts* o, uint32_t w,
              uint32_t h, uint32_t tile_w, float* rgb, float* t, int32_t* inst, uint32_t job_begin) {
  std::memset(&r, 0, sizeof r);
  {
    // camera basis and pixel mapping, in double, once per request
    double f[3], rt[3];
    for (int i = 0; i < 3; ++i) {
      r.eye[i] = cam->eye[i];
      f[i] = (double)cam->target[i] - cam->eye[i];
    }
    const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (double& v : f) v /= fl;
    const double up[3] = {cam->up[0], cam->up[1], cam->up[2]};
    rt[0] = up[1] * f[2] - up[2] * f[1];
    rt[1] = up[2] * f[0] - up[0] * f[2];
    rt[2] = up[0] * f[1] - up[1] * f[0];
    const double rl = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    for (int i = 0; i < 3; ++i) {
      r.fwd[i] = (float)f[i];
      r.right[i] = (float)(rt[i] / rl);
    }
    const double sh = std::tan((double)cam->vfov_deg * M_PI / 360.0);
    r.pix_kx = (float)(2.0 * sh / h);   // = 2 sh aspect / w
    r.pix_ky = (float)(-2.0 * sh / h);
    r.pix_oy = (float)sh;
  }
  r.width = w;
  r.height = h;
  r.spp = o->spp;
  r.jitter = o->jitter;
  r.max_steps = o->max_steps;
  r.shadows = o->shadows;
  r.bounces = o->bounces;
  r.seed_lo = (uint32_t)(o->seed & 0xffffffffu);
  r.seed_hi = (uint32_t)(o->seed >> 32);
  r.tile_w = tile_w;
  r.eps = o->eps;
  r.tmin = o->tmin;
  r.tmax = o->tmax;
  r.shadow_offset = o->shadow_offset;
  r.fd_h = o->fd_h;
  const uint32_t th = 64 / tile_w;
  r.tiles_x = (w + tile_w - 1) / tile_w;
  const uint32_t tiles_y = (h + th - 1) / th;
  r.job_begin = job_begin;
  r.job_end = job_begin + r.tiles_x * tiles_y * 64 * o->spp;
  r.insts = s->d_insts;
  r.nodes = s->d_nodes;
  r.consts = s->d_consts;
  r.out_rgb = rgb;
  r.out_t = t;
  r.out_inst = inst;
  first_region(r, s, cam, o, w, h, tile_w);
}

int g_blocks_per_cu = 0;

int grid_for(uint32_t total_jobs, int blocks_per_cu = 0) {
  // persistent grid: as many workgroups as can be resident at once
  if (g_blocks_per_cu == 0) g_blocks_per_cu = occupancy_blocks_per_cu();
  int cus = device_cu_count();
  if (cus <= 0) cus = 256;
  long want = (long)cus * (blocks_per_cu > 0 ? blocks_per_cu : g_blocks_per_cu);
  long need = ((long)total_jobs + kBlock - 1) / kBlock;
  return (int)std::max(1L, std::min(want, need));
}

}  // namespace

namespace pr {

// Shared by pr_render, pr_render_batch and the server: copy the request
// table, launch, record the scenes' last-use events.  ``counts_dev`` selects
// the instrumented kernel.
pr_status launch_prepared(const std::vector<ReqDev>& reqs, const std::vector<pr_scene*>& scenes,
                          uint32_t total_jobs, int step_budget, int compact, bool use_graph,
                          unsigned long long* counts_dev, hipStream_t stream, hipEvent_t done_evt,
                          unsigned long long* track_dev, DoneRec* done_host) {
  LaunchCtx* c = acquire_ctx((uint32_t)reqs.size());
  if (!c) return set_error(PR_ERR_OUT_OF_MEMORY, "could not allocate a launch context");
  // fixed-point colour accumulators and sample counters for requests with
  // several samples per pixel (zero at allocation; each launch leaves them zero)
  size_t need_px = 0;
  for (const ReqDev& r : reqs)
    if (r.spp > 1 && !r.sample_acc) need_px += (size_t)r.width * r.height;
  if (need_px > c->sample_px_cap) {
    // grow while the context is idle
    if (c->sample_acc) (void)hipFree(c->sample_acc);
    if (c->sample_cnt) (void)hipFree(c->sample_cnt);
    c->sample_acc = nullptr;
    c->sample_cnt = nullptr;
    c->sample_px_cap = 0;
    if (hipMalloc((void**)&c->sample_acc, need_px * 3 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&c->sample_cnt, need_px * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->sample_acc, 0, need_px * 3 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->sample_cnt, 0, need_px * sizeof(uint32_t)) != hipSuccess) {
      (void)hipGetLastError();
      if (c->sample_acc) (void)hipFree(c->sample_acc);
      if (c->sample_cnt) (void)hipFree(c->sample_cnt);
      c->sample_acc = nullptr;
      c->sample_cnt = nullptr;
      release_ctx(c);
      return set_error(PR_ERR_OUT_OF_MEMORY, "could not allocate %zu bytes of per-sample scratch", need_px * 28);
    }
    c->sample_px_cap = need_px;
  }
  std::vector<ReqDev> table(reqs);
  {
    size_t off = 0;
    for (ReqDev& r : table) {
      if (r.spp > 1 && !r.sample_acc) {
        r.sample_acc = c->sample_acc + off * 3;
        r.sample_cnt = c->sample_cnt + off;
        off += (size_t)r.width * r.height;
      }
    }
  }
  QueueDev q;
  std::memset(&q, 0, sizeof q);
  q.total_jobs = total_jobs;
  q.n_req = (uint32_t)reqs.size();
  bool shared = !scenes.empty();
  // scenes with user estimators run their own build, which does not regroup
  bool user = false;
  for (pr_scene* s : scenes) user = user || (s->n_types_present >> PR_USER_TYPE_BASE) != 0;
  if (user) compact = 0;
  q.compact_pct = (uint32_t)compact;
  q.track = track_dev;
  q.done_recs = done_host;
  for (pr_scene* s : scenes) shared = shared && s == scenes[0];
  // a launch whose two-wide BVH is not all staged in LDS runs the kernel
  // build that traverses the four-wide BVH (same results), when every scene
  // of the launch has one
  bool descend = !user && compact == 0 && counts_dev == nullptr && !(shared && scenes[0]->dnodes.size() <= kLdsNodes);
  for (pr_scene* s : scenes) descend = descend && s->d_nodes4 != nullptr;
  if (shared) {
    // one scene for the whole launch: every workgroup stages its top BVH
    // levels (of the tree its kernel build reads), first instance records
    // and constants in LDS
    if (descend) {
      q.n_stage_nodes = std::min<uint32_t>((uint32_t)scenes[0]->dnodes4.size(), kLdsNodes);
      q.stage_nodes = (const NodeDev*)scenes[0]->d_nodes4;
    } else {
      q.n_stage_nodes = std::min<uint32_t>((uint32_t)scenes[0]->dnodes.size(), kLdsNodes);
      q.stage_nodes = scenes[0]->d_nodes;
    }
    q.n_stage_insts = std::min<uint32_t>(scenes[0]->consts.n_inst, kLdsInsts);
    q.stage_insts = scenes[0]->d_insts;
    q.stage_consts = scenes[0]->d_consts;
  }
  // the requests of a four-wide launch point at their scenes' four-wide trees
  if (descend)
    for (size_t i = 0; i < table.size(); ++i) table[i].nodes = (const NodeDev*)scenes[i]->d_nodes4;
  std::memcpy(c->host, &q, sizeof q);
  std::memcpy((char*)c->host + sizeof(QueueDev), table.data(), table.size() * sizeof(ReqDev));
  const size_t bytes = sizeof(QueueDev) + reqs.size() * sizeof(ReqDev);
  // scenes with user estimators run the kernel built with them
  UserKernels uk;
  if (user) {
    pr_status st = user_kernels(&uk);
    if (st != PR_OK) {
      release_ctx(c);
      return st;
    }
  }
  auto launch = [&](unsigned long long* counts, hipStream_t s, const LaunchCfg& cf) -> int {
    const ReqDev* r0 = (const ReqDev*)((char*)c->dev + sizeof(QueueDev));
    QueueDev* q0 = (QueueDev*)c->dev;
    return user ? launch_trace_user(uk, r0, q0, cf, counts, s)
                : launch_trace(r0, q0, total_jobs, (uint32_t)reqs.size(), cf, counts, s);
  };
  LaunchCfg cfg{step_budget, grid_for(total_jobs, user ? uk.blocks_per_cu : 0), compact, descend};
  hipError_t e;
  bool graphed = false;
  if (use_graph && stream != nullptr && counts_dev == nullptr) {
    const void* kernel_id = user ? uk.plain : nullptr;
    if (!(c->graph && c->graph_bytes == bytes && c->graph_blocks == cfg.grid_blocks &&
          c->graph_budget == step_budget && c->graph_stream == stream && c->graph_kernel == kernel_id &&
          c->graph_compact == compact && c->graph_descend == descend)) {
      if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
      }
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        // a graph missing its copy or kernel would replay as a no-op: any
        // failure while capturing discards it (the plain path runs instead)
        hipError_t ce = hipMemcpyAsync(c->dev, c->host, bytes, hipMemcpyHostToDevice, stream);
        const int le = ce == hipSuccess ? launch(nullptr, stream, cfg) : 1;
        e = hipStreamEndCapture(stream, &g);
        if (e == hipSuccess && (ce != hipSuccess || le != 0)) e = ce != hipSuccess ? ce : hipErrorLaunchFailure;
      }
      if (e == hipSuccess && g) {
        e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
      }
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        c->graph = nullptr;
      } else {
        c->graph_bytes = bytes;
        c->graph_blocks = cfg.grid_blocks;
        c->graph_budget = step_budget;
        c->graph_stream = stream;
        c->graph_kernel = kernel_id;
        c->graph_compact = compact;
        c->graph_descend = descend;
      }
    }
    if (c->graph) {
      e = hipGraphLaunch(c->graph, stream);
      if (e != hipSuccess) {
        release_ctx(c);
        return hip_fail(e, "hipGraphLaunch");
      }
      graphed = true;
    }
  }
  if (!graphed) {
    e = hipMemcpyAsync(c->dev, c->host, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
      release_ctx(c);
      return hip_fail(e, "hipMemcpyAsync(request table)");
    }
    if (launch(counts_dev, stream, cfg) != 0) {
      release_ctx(c);
      return set_error(PR_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
  }
  // the scenes' last-use events guard their buffers against a rebuild while
  // this launch may still read them, so a failed record is an error
  e = hipEventRecord(c->done, stream);
  for (pr_scene* s : scenes)
    if (s->last_use && e == hipSuccess) e = hipEventRecord(s->last_use, stream);
  if (done_evt && e == hipSuccess) e = hipEventRecord(done_evt, stream);
  release_ctx(c);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  return PR_OK;
}

// Validates one request and appends its table entry.
pr_status add_request(std::vector<ReqDev>& reqs, std::vector<pr_scene*>& scenes, pr_scene* s,
                      const pr_camera* cam, const pr_render_opts* o, uint32_t w, uint32_t h, float* rgb,
                      float* t, int32_t* inst, uint32_t tile_w_override, uint32_t& total_jobs,
                      bool check_ptrs) {
  if (!s) return set_error(PR_ERR_INVALID_ARG, "scene is NULL");
  pr_status st = validate_camera(cam);
  if (st != PR_OK) return st;
  if ((st = validate_opts(o, w, h)) != PR_OK) return st;
  if (!s->built || !s->uploaded) return set_error(PR_ERR_NOT_BUILT, "scene BVH not built/uploaded");
  if (!rgb) return set_error(PR_ERR_INVALID_ARG, "out_rgb is NULL");
  if (check_ptrs) {
    if ((st = check_device_ptr(rgb, (size_t)w * h * 12, "out_rgb", s->device)) != PR_OK) return st;
    if (t && (st = check_device_ptr(t, (size_t)w * h * 4, "out_t", s->device)) != PR_OK) return st;
    if (inst && (st = check_device_ptr(inst, (size_t)w * h * 4, "out_inst", s->device)) != PR_OK) return st;
  }
  uint32_t tw = o->tile_w ? o->tile_w : (tile_w_override ? tile_w_override : tuned_for(s).tile_w);
  const uint64_t tiles = (uint64_t)((w + tw - 1) / tw) * ((h + 64 / tw - 1) / (64 / tw));
  if ((uint64_t)total_jobs + tiles * 64ull * o->spp > 0xF0000000ull)
    return set_error(PR_ERR_INVALID_ARG, "too many pixel samples in one launch");
  ReqDev r;
  fill_req(r, s, cam, o, w, h, tw, rgb, t, inst, total_jobs);
  total_jobs = r.job_end;
  reqs.push_back(r);
  scenes.push_back(s);
  return PR_OK;
}

// Persistent grid of the built-in kernel for a launch of total_jobs jobs.
int persistent_grid(uint32_t total_jobs) { return grid_for(total_jobs); }

int budget_for(const pr_scene* s, const pr_render_opts* o, uint32_t override_budget) {
  if (o && o->step_budget) return (int)o->step_budget;
  if (override_budget) return (int)override_budget;
  return (int)tuned_for(s).step_budget;
}

// Regrouping threshold of a launch (0 = none) from an explicit request
// (1..100 or PR_COMPACT_NEVER), else the scene class's tuned choice.
int compact_for(const pr_scene* s, const pr_render_opts* o, uint32_t override_pct) {
  const uint32_t v = (o && o->compact_pct) ? o->compact_pct : override_pct;
  if (v == PR_COMPACT_NEVER) return 0;
  if (v >= 1 && v <= 100) return (int)v;
  return (int)tuned_for(s).compact;
}

}  // namespace pr

extern "C" {

pr_status pr_render(pr_scene* s, const pr_camera* cam, const pr_render_opts* opts, uint32_t w, uint32_t h,
                    float* out_rgb, float* out_t, int32_t* out_inst, void* stream) {
  try {
    std::vector<ReqDev> reqs;
    std::vector<pr_scene*> scenes;
    uint32_t total = 0;
    pr_status st = add_request(reqs, scenes, s, cam, opts, w, h, out_rgb, out_t, out_inst, 0, total, true);
    if (st != PR_OK) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    st = launch_prepared(reqs, scenes, total, budget_for(s, opts, 0), compact_for(s, opts, 0), false, nullptr,
                         (hipStream_t)stream, nullptr, nullptr, nullptr);
    return st == PR_OK ? ok() : st;
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

pr_status pr_launch_shape(uint32_t* compute_units, uint32_t* workgroups_per_cu) {
  if (!compute_units || !workgroups_per_cu) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(PR_ERR_DEVICE, "no HIP device");
  }
  const int cus = device_cu_count();
  if (cus <= 0) return set_error(PR_ERR_DEVICE, "could not query the compute units");
  if (g_blocks_per_cu == 0) g_blocks_per_cu = occupancy_blocks_per_cu();
  *compute_units = (uint32_t)cus;
  *workgroups_per_cu = (uint32_t)g_blocks_per_cu;
  return ok();
}

pr_status pr_render_counts(pr_scene* s, const pr_camera* cam, const pr_render_opts* opts, uint32_t w,
                           uint32_t h, float* out_rgb, uint64_t* counts) {
  try {
    if (!counts) return set_error(PR_ERR_INVALID_ARG, "counts is NULL");
    std::vector<ReqDev> reqs;
    std::vector<pr_scene*> scenes;
    uint32_t total = 0;
    pr_status st = add_request(reqs, scenes, s, cam, opts, w, h, out_rgb, nullptr, nullptr, 0, total, true);
    if (st != PR_OK) return st;
    unsigned long long* d = nullptr;
    hipError_t e = hipMalloc((void**)&d, sizeof(unsigned long long) * kNumCounts);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(counts)");
    e = hipMemset(d, 0, sizeof(unsigned long long) * kNumCounts);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return hip_fail(e, "hipMemset(counts)");
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      st = launch_prepared(reqs, scenes, total, budget_for(s, opts, 0), compact_for(s, opts, 0), false, d,
                           nullptr, nullptr, nullptr, nullptr);
    }
    if (st == PR_OK) {
      e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipMemcpy(counts, d, sizeof(unsigned long long) * kNumCounts, hipMemcpyDeviceToHost);
      if (e != hipSuccess) st = hip_fail(e, "counting render");
    }
    (void)hipFree(d);
    return st == PR_OK ? ok() : st;
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

pr_status pr_render_batch(const pr_request* rq, uint32_t n, const pr_batch_opts* bo, void* stream) {
  try {
    if (!rq || n == 0 || n > 4096) return set_error(PR_ERR_INVALID_ARG, "need 1..4096 requests");
    pr_batch_opts b{0, 0, 0, 0, 0};
    if (bo) b = *bo;
    if ((b.tile_w == 0) != (b.tile_h == 0) || (b.tile_w && b.tile_w * b.tile_h != 64))
      return set_error(PR_ERR_INVALID_ARG, "batch tile must be 0,0 or multiply to 64");
    if (b.compact_pct > 100 && b.compact_pct != PR_COMPACT_NEVER)
      return set_error(PR_ERR_INVALID_ARG, "compact_pct must be 0, 1..100 or PR_COMPACT_NEVER");
    std::vector<ReqDev> reqs;
    std::vector<pr_scene*> scenes;
    reqs.reserve(n);
    uint32_t total = 0;
    for (uint32_t i = 0; i < n; ++i) {
      pr_status st = add_request(reqs, scenes, rq[i].scene, &rq[i].cam, &rq[i].opts, rq[i].width, rq[i].height,
                                 rq[i].out_rgb, rq[i].out_t, rq[i].out_inst, b.tile_w, total, true);
      if (st != PR_OK) {
        std::string m = "request " + std::to_string(i) + ": " + pr_last_error();
        return set_error(st, "%s", m.c_str());
      }
    }
    int budget = b.step_budget ? (int)b.step_budget : budget_for(scenes[0], nullptr, 0);
    pr_status st = launch_prepared(reqs, scenes, total, budget, compact_for(scenes[0], nullptr, b.compact_pct),
                                   b.use_graph != 0, nullptr, (hipStream_t)stream, nullptr, nullptr, nullptr);
    return st == PR_OK ? ok() : st;
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

pr_status pr_autotune(const pr_request* rq, uint32_t n, pr_batch_opts* best_out) {
  try {
    if (!rq || n == 0 || n > 4096) return set_error(PR_ERR_INVALID_ARG, "need 1..4096 requests");
    static const uint32_t tiles[] = {8, 16, 32, 64};
    static const uint32_t budgets[] = {8, 16, 24, 32, 64};
    static const uint32_t compacts[] = {PR_COMPACT_NEVER, 50, 100};
    hipStream_t st_ = nullptr;
    hipError_t e = hipStreamCreate(&st_);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    hipEvent_t a = nullptr, b = nullptr;
    auto cleanup = [&]() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      (void)hipStreamDestroy(st_);
    };
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
      cleanup();
      return hip_fail(e, "hipEventCreate");
    }
    float best_ms = 1e30f;
    pr_batch_opts best{8, 8, 16, 0, PR_COMPACT_NEVER};
    for (uint32_t tw : tiles) {
      for (uint32_t sb : budgets) for (uint32_t cp : compacts) {
        pr_batch_opts o{tw, 64 / tw, sb, 0, cp};
        // warm-up then 3 timed launches, take the minimum
        pr_status s = pr_render_batch(rq, n, &o, st_);
        if (s != PR_OK) {
          cleanup();
          return s;
        }
        float ms_min = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          if ((e = hipEventRecord(a, st_)) != hipSuccess) break;
          if ((s = pr_render_batch(rq, n, &o, st_)) != PR_OK) {
            cleanup();
            return s;
          }
          float ms = 0;
          if ((e = hipEventRecord(b, st_)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess ||
              (e = hipEventElapsedTime(&ms, a, b)) != hipSuccess)
            break;
          ms_min = std::min(ms_min, ms);
        }
        if (e != hipSuccess) {
          cleanup();
          return hip_fail(e, "timing a candidate launch");
        }
        if (ms_min < best_ms) {
          best_ms = ms_min;
          best = o;
        }
      }
    }
    cleanup();
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      load_tune_cache();
      g_tuned[size_class(rq[0].scene)] =
          Tuned{best.tile_w, best.step_budget, best.compact_pct == PR_COMPACT_NEVER ? 0u : best.compact_pct};
      save_tune_cache();
    }
    if (best_out) *best_out = best;
    return ok();
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

}  // extern "C"
