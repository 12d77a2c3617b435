// pr_render_noalloc: one frame like pr_render, with no device allocation.
//
// pr_render keeps its launch table, queue header and the multi-sample
// fixed-point accumulators in launch contexts it allocates on first use.
// Callers that may not allocate device memory (code under HIP graph capture,
// serving loops and harnesses that forbid hipMalloc) use this entry point
// instead: those buffers live in one fixed scratch array per device, held
// from the library's first use on that device until the process ends, and
// the request record reaches the device as a kernel argument (no host
// staging buffer, no copy).  The rendering kernel is pr_render's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "host_common.h"

namespace pr {
pr_status add_request(std::vector<ReqDev>& reqs, std::vector<pr_scene*>& scenes, pr_scene* s,
                      const pr_camera* cam, const pr_render_opts* o, uint32_t w, uint32_t h, float* rgb,
                      float* t, int32_t* inst, uint32_t tile_w_override, uint32_t& total_jobs,
                      bool check_ptrs);
int budget_for(const pr_scene* s, const pr_render_opts* o, uint32_t override_budget);
int compact_for(const pr_scene* s, const pr_render_opts* o, uint32_t override_pct);
int persistent_grid(uint32_t total_jobs);
}  // namespace pr

using namespace pr;

// Layout: [QueueDev | ReqDev] at 0; the per-pixel colour accumulators
// (3 x u64) at kAccOffset, then the per-pixel sample counters (u32).
static __device__ __align__(256) unsigned char scratch[PR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAccOffset = 4096;
static_assert(sizeof(QueueDev) + sizeof(ReqDev) <= kAccOffset, "scratch header");

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// Scratch bytes a request needs: the header, and accumulators and counters
// when it takes several samples per pixel.
size_t scratch_need(uint32_t w, uint32_t h, uint32_t spp) {
  const size_t px = (size_t)w * h;
  return kAccOffset + (spp > 1 ? up256(px * 24) + up256(px * 4) : 0);
}

// The scratch array's device address on each device, from
// hipGetSymbolAddress with that device current (the host-side name of the
// array is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

pr_status scratch_for(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(PR_ERR_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = p;
  }
  *out = (unsigned char*)g_scratch[dev];
  return PR_OK;
}

// The fields of a QueueDev before its cursors, as kernel-argument bytes.
struct QueueHead {
  uint4 w[5];
};
static_assert(sizeof(QueueHead) == offsetof(QueueDev, pad_head), "queue head");

// Writes the launch's queue header and request record into the scratch
// header, sets the queue cursors to zero and clears the accumulator and
// counter words the request uses (one block of 256 threads at least).
__global__ void noalloc_setup(QueueHead qh, ReqDev r, unsigned char* base, uint64_t zero_words16) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < 5) ((uint4*)base)[tid] = qh.w[tid];
  if (tid < sizeof(QueueDev::cursor) / 16)
    ((uint4*)(base + offsetof(QueueDev, cursor)))[tid] = make_uint4(0, 0, 0, 0);
  if (tid == 0) *(ReqDev*)(base + sizeof(QueueDev)) = r;
  uint4* acc = (uint4*)(base + kAccOffset);
  for (uint64_t i = tid; i < zero_words16; i += (uint64_t)gridDim.x * blockDim.x) acc[i] = make_uint4(0, 0, 0, 0);
}

}  // namespace

extern "C" pr_status pr_render_noalloc(pr_scene* s, const pr_camera* cam, const pr_render_opts* opts,
                                       uint32_t w, uint32_t h, float* out_rgb, float* out_t, int32_t* out_inst,
                                       void* stream) {
  try {
    if (!s || !cam || !opts) return set_error(PR_ERR_INVALID_ARG, "scene, camera and opts must be non-NULL");
    if (w < 1 || h < 1 || w > 16384 || h > 16384)
      return set_error(PR_ERR_INVALID_ARG, "width and height must be in 1..16384");
    const size_t need = scratch_need(w, h, opts->spp);
    if (need > (size_t)PR_NOALLOC_SCRATCH_BYTES)
      return set_error(PR_ERR_INVALID_ARG,
                       "%ux%u at %u samples per pixel needs %zu bytes of scratch; the allocation-free path "
                       "holds %zu (at most %zu pixels with several samples)",
                       w, h, opts->spp, need, (size_t)PR_NOALLOC_SCRATCH_BYTES,
                       ((size_t)PR_NOALLOC_SCRATCH_BYTES - kAccOffset - 512) / 28);
    std::vector<ReqDev> reqs;
    std::vector<pr_scene*> scenes;
    uint32_t total = 0;
    pr_status st = add_request(reqs, scenes, s, cam, opts, w, h, out_rgb, out_t, out_inst, 0, total, true);
    if (st != PR_OK) return st;
    if ((s->n_types_present >> PR_USER_TYPE_BASE) != 0)
      return set_error(PR_ERR_UNSUPPORTED, "scenes with user estimators need pr_render (their kernel is "
                                           "built and loaded at run time)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != s->device) return set_error(PR_ERR_INVALID_ARG, "the scene lives on device %d, current is %d", s->device, dev);
    unsigned char* base = nullptr;
    if ((st = scratch_for(dev, &base)) != PR_OK) return st;

    ReqDev r = reqs[0];
    uint64_t zero16 = 0;
    if (r.spp > 1) {
      const size_t px = (size_t)w * h;
      r.sample_acc = (unsigned long long*)(base + kAccOffset);
      r.sample_cnt = (uint32_t*)(base + kAccOffset + up256(px * 24));
      zero16 = (up256(px * 24) + up256(px * 4)) / 16;
    }
    const int compact = compact_for(s, opts, 0);
    QueueDev q;
    std::memset(&q, 0, sizeof q);
    q.total_jobs = total;
    q.n_req = 1;
    q.compact_pct = (uint32_t)compact;
    // one scene: every workgroup stages its top BVH levels, first instance
    // records and constants in LDS, as for pr_render
    // as in pr_render: the four-wide tree for a BVH not all in LDS, staged
    // and pointed at by the request record alike
    const bool descend = compact == 0 && s->dnodes.size() > kLdsNodes && s->d_nodes4 != nullptr;
    if (descend) r.nodes = (const NodeDev*)s->d_nodes4;
    q.n_stage_nodes = std::min<uint32_t>((uint32_t)(descend ? s->dnodes4.size() : s->dnodes.size()), kLdsNodes);
    q.n_stage_insts = std::min<uint32_t>(s->consts.n_inst, kLdsInsts);
    q.stage_nodes = descend ? (const NodeDev*)s->d_nodes4 : s->d_nodes;
    q.stage_insts = s->d_insts;
    q.stage_consts = s->d_consts;

    std::lock_guard<std::mutex> lk(s->mu);
    const uint32_t setup_blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(1024, (zero16 + 255) / 256));
    QueueHead qh;
    std::memcpy(&qh, &q, sizeof qh);
    hipLaunchKernelGGL(noalloc_setup, dim3(setup_blocks), dim3(256), 0, (hipStream_t)stream, qh, r, base, zero16);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "noalloc_setup launch");
    const LaunchCfg cfg{budget_for(s, opts, 0), persistent_grid(total), compact, descend};
    if (launch_trace((const ReqDev*)(base + sizeof(QueueDev)), (QueueDev*)base, total, 1, cfg, nullptr, stream) != 0)
      return set_error(PR_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (s->last_use && (e = hipEventRecord(s->last_use, (hipStream_t)stream)) != hipSuccess)
      return hip_fail(e, "hipEventRecord");
    return ok();
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}
