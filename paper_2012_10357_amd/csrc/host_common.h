// Host-side helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace pr {

pr_status set_error(pr_status st, const char* fmt, ...);
pr_status ok();
pr_status hip_fail(hipError_t e, const char* what);

// A launch context: device memory holding [QueueDev | ReqDev x capacity],
// pinned host staging of the same layout, and an event marking the last
// launch that used it.  Contexts are recycled once their event completes.
struct LaunchCtx {
  void* dev = nullptr;
  void* host = nullptr;       // pinned
  size_t bytes = 0;
  uint32_t capacity = 0;      // requests
  hipEvent_t done = nullptr;
  bool in_use = false;
  int device = -1;
  // per-pixel colour accumulators (3 x u64) and sample counters for
  // multi-sample requests, grown on demand; sample_px_cap pixels
  unsigned long long* sample_acc = nullptr;
  uint32_t* sample_cnt = nullptr;
  size_t sample_px_cap = 0;
  // graph cache for this context
  hipGraphExec_t graph = nullptr;
  size_t graph_bytes = 0;
  int graph_blocks = 0, graph_budget = 0;
  hipStream_t graph_stream = nullptr;
  const void* graph_kernel = nullptr;   // the kernel the graph launches (nullptr: built-in)
  int graph_compact = 0;                // regrouping threshold the graph's kernel runs with
  bool graph_descend = false;           // the graph's kernel is the build for BVHs not all in LDS
};

LaunchCtx* acquire_ctx(uint32_t n_req);
void release_ctx(LaunchCtx* c);

}  // namespace pr

// The scene object behind the opaque handle.
struct pr_scene {
  std::vector<pr::InstDev> host_insts;   // user order
  std::vector<float> host_shade;         // user order: albedo rgb, reflectivity
  std::vector<pr_material> mats;         // the scene's materials (for meshes added later)
  uint32_t n_proc = 0;                   // procedural instances; triangle items follow
  std::vector<float> world_aabb;         // 6 per instance
  std::vector<pr::HostNode> nodes;       // BVH, children adjacent, breadth-first
  std::vector<pr::NodeDev> dnodes;       // device layout: child boxes in the parent
  std::vector<pr::Node4Dev> dnodes4;     // four-wide device layout (empty: none)
  std::vector<uint32_t> order;           // leaf slot -> user instance index
  pr::SceneConstsDev consts{};
  bool built = false;
  bool uploaded = false;
  int device = -1;
  pr::InstDev* d_insts = nullptr;        // leaf order
  pr::NodeDev* d_nodes = nullptr;
  pr::Node4Dev* d_nodes4 = nullptr;
  pr::SceneConstsDev* d_consts = nullptr;
  float* d_shade = nullptr;              // leaf order
  uint64_t device_bytes = 0;
  hipEvent_t last_use = nullptr;         // last launch reading this scene
  std::mutex mu;
  uint32_t n_types_present = 0;          // bit mask of primitive types
};
