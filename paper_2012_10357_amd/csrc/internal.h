// Records shared by the host library and the gfx950 kernels.
//
// The paper keeps per-instance data minimal so that traversal needs few
// resources (Sec. 4.1.1: the local root signature only indexes an instance
// buffer held globally).  Here each instance is one 128-byte record holding
// everything its intersection needs, so a lane loads it once per candidate;
// the material, needed only when a hit is shaded, sits in a separate array.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/procray.h"

namespace pr {

constexpr int kStackDepth = 32;       // BVH traversal stack entries per lane
constexpr int kWave = 64;             // CDNA wavefront width
constexpr int kBlock = 256;           // threads per workgroup (4 waves)
// Bound on the magnitude of a sample colour: scene constants that could
// exceed it are rejected by pr_scene_create and user closest-hit outputs are
// clamped to it, so 32.32 fixed-point sums of up to 64 samples fit 63 bits.
constexpr float kMaxColour = PR_MAX_COLOUR;   // 2^24

// Type tag of a triangle leaf item (not a procedural type).
constexpr uint32_t kTriangle = PR_NUM_TYPES;

// Per-instance record, 32 words.  Local point = Ainv * (world - b).
// A triangle item reuses it in world space: Ainv = (v0, e1 = v1 - v0,
// e2 = v2 - v0), b = unit face normal, lo/hi = its world AABB, type = kTriangle.
struct alignas(16) InstDev {
  float Ainv[9];
  float b[3];
  float lo[3];
  float hi[3];
  float sigma;       // smallest singular value of A: local distance -> world lower bound
  uint32_t type;
  float prm[8];      // kernel-ready parameters, see pack_params(); prm[7] = instance index bits
  float cut[4];      // cutting plane n.p <= d (unit n); n = 0: none
};
static_assert(sizeof(InstDev) == 128, "instance record must stay 128 bytes");

// Host-side BVH node (the exported layout): children adjacent.
struct alignas(16) HostNode {
  float lo[3];
  uint32_t first;    // interior: left child index (right = first + 1); leaf: first instance slot
  float hi[3];
  uint32_t count;    // 0 = interior
};
static_assert(sizeof(HostNode) == 32, "host BVH node must stay 32 bytes");
static_assert(sizeof(HostNode) == sizeof(pr_bvh_node), "exported node layout");

// Device BVH node: an interior node holding both children's boxes, so one
// 64-byte load per visited node gives everything needed to test and order
// its children.  Child k: n == 0 -> interior node c; n >= 1 -> leaf over
// instance slots [c, c + n); n == kNoChild -> absent (single-leaf scenes).
constexpr uint32_t kNoChild = 0xffffffffu;
struct alignas(16) NodeDev {
  float lo0[3];
  uint32_t c0;
  float hi0[3];
  uint32_t n0;
  float lo1[3];
  uint32_t c1;
  float hi1[3];
  uint32_t n1;
};
static_assert(sizeof(NodeDev) == 64, "device BVH node must stay 64 bytes");

// Four-wide BVH node, read by the kernel build for launches whose BVH is not
// all staged in LDS (half the dependent node loads of the two-wide tree).
// The boxes of up to four children are stored as 8-bit grid coordinates,
// child box = org + q * step per axis, on a grid whose cells 1..254 span the
// node's box, each bound rounded outward and widened by one more cell, so a
// decoded box (or a slab distance computed from it in float32) always
// contains the child's box.  ref: kNoRef = no child; bit 31 set = leaf over
// instance slots [first, first + count) as 1 << 31 | (count - 1) << 24 |
// first; else the index of the child node.
constexpr uint32_t kNoRef = 0xffffffffu;
constexpr uint32_t kMaxNodes4 = 8192;   // stack entries (node, child) fit 16 bits
struct alignas(16) Node4Dev {
  float org[3];
  uint32_t ref0;
  float step[3];
  uint32_t ref1;
  uint8_t q[24];     // child c: lo x, y, z and hi x, y, z at q[6c .. 6c + 5]
  uint32_t ref2, ref3;
};
static_assert(sizeof(Node4Dev) == 64, "four-wide BVH node must stay 64 bytes");

struct alignas(16) SceneConstsDev {
  float light[3];
  float ambient;
  float light_rgb[3];
  uint32_t n_inst;
  float background[3];
  uint32_t n_nodes;
  const float* shade;  // per instance slot (BVH leaf order): albedo rgb, reflectivity
  const Node4Dev* nodes4;   // four-wide BVH (null: the scene has none)
};
static_assert(sizeof(SceneConstsDev) == 64, "scene constants");

// One render request as seen by the kernel.  192 bytes.  A job is one
// (pixel, sample); jobs are ordered tile, pixel (Z order in 8x8 tiles), sample.
// The camera arrives as its orthonormal basis and pixel mapping, computed on
// the host in double.
struct alignas(16) ReqDev {
  float eye[3];
  float pix_kx;            // pixel pitch on the image plane at distance 1: 2 tan(vfov / 2) / H
  float fwd[3];            // unit view direction
  uint32_t width;
  float right[3];          // unit image-plane x axis (up x fwd, normalised)
  uint32_t height;
  uint32_t spp, jitter, max_steps, shadows;
  uint32_t bounces, seed_lo, seed_hi, tile_w;
  float eps, tmin, tmax, shadow_offset;
  float fd_h;
  uint32_t tiles_x;
  uint32_t job_begin;      // first global job index of this request
  uint32_t job_end;        // one past the last
  const InstDev* insts;    // instance records, in BVH leaf order
  const NodeDev* nodes;
  const SceneConstsDev* consts;
  float pix_ky, pix_oy;    // -pix_kx and tan(vfov / 2): plane y of pixel row py is (py + jy) pix_ky + pix_oy
  float* out_rgb;
  float* out_t;
  int32_t* out_inst;
  // tiles handed out first, [x0, x1) x [y0, y1) in tile units (empty: row-major order)
  uint16_t first_x0, first_y0, first_x1, first_y1;
  unsigned long long* sample_acc;  // spp > 1: 32.32 fixed-point colour sums (W*H*3), zero between launches
  uint32_t* sample_cnt;            // spp > 1: finished samples per pixel (W*H), zero between launches
};
static_assert(sizeof(ReqDev) == 192, "request record");

// Work queue of one launch.  When every
// request of the launch renders the same scene, that scene's top BVH nodes,
// first instance records and constants are staged in LDS by every workgroup.
// compact_pct > 0 selects the regrouping kernel: a workgroup pools its lanes'
// march queries, sorted by primitive type, whenever fewer than compact_pct %
// of its lanes march or one of its waves marches more than one type.
//
// Jobs are handed out in chunks of 64 consecutive indices.  Chunk c belongs
// to partition c mod kQueueParts, and each partition has its own cursor
// (its chunks in increasing order, counted in jobs past the partition's
// first-round chunks), 256 bytes from the next, so the queue atomics of the
// whole chip spread over kQueueParts addresses instead of contending for one.
// Every wave starts on the chunk numbered like the wave, without an atomic.
constexpr uint32_t kQueueParts = 8;
constexpr uint32_t kCursorWords = 64;
struct alignas(256) QueueDev {
  uint32_t reserved0;
  uint32_t total_jobs;
  uint32_t n_req;
  uint32_t n_stage_nodes;  // 0 = no staging
  uint32_t n_stage_insts;
  uint32_t compact_pct;    // 0: waves march their own lanes; 1..100: regroup threshold
  uint32_t pad1, pad2;
  const NodeDev* stage_nodes;     // global source of the staged scene
  const InstDev* stage_insts;
  const SceneConstsDev* stage_consts;
  // per-request completion tracking (served launches; null otherwise):
  // device counters, 3 per request (jobs done, shadow rays, bounce rays),
  // zero at launch, and host-visible completion records
  unsigned long long* track;
  struct DoneRec* done_recs;
  const void* pad3;
  uint32_t pad_head[44];
  // partition cursors (zero at launch), popped with atomicAdd
  uint32_t cursor[kQueueParts][kCursorWords];
};
static_assert(offsetof(QueueDev, pad_head) == 80, "queue header fields");
static_assert(offsetof(QueueDev, cursor) == 256 && sizeof(QueueDev) == 2304, "queue cursors");

// Completion record of one tracked request, in host-visible (pinned) memory:
// the device writes the request's ray counts and then sets done, once every
// job of the request has finished and its pixels are written.
struct alignas(16) DoneRec {
  unsigned long long rays_shadow;   // shadow rays of primary and bounce hits
  unsigned long long rays_bounce;   // mirror-bounce rays
  uint32_t done;
  uint32_t pad[3];
};
static_assert(sizeof(DoneRec) == 32, "completion record");

constexpr uint32_t kLdsNodes = 128;   // 8 KB: the top seven BVH levels (breadth-first layout)
constexpr uint32_t kLdsInsts = 32;    // 4 KB of instance records
constexpr uint32_t kLdsReqs = 4;      // request records staged per workgroup

// Per-launch counters of the instrumented kernel.
constexpr int kNumCounts = PR_NUM_COUNTS;

struct LaunchCfg {
  int step_budget;   // DE evaluations between refill checks
  int grid_blocks;   // persistent grid size
  int compact_pct;   // 0 = no regrouping (also written to the queue header)
  bool descend;      // the launch's BVH is not all staged in LDS (kernel choice only)
};

}  // namespace pr

// Kernel launch entry points (defined in trace.hip).
namespace pr {
// Run-time build with user estimators (user_de.cpp).
bool user_type_registered(uint32_t type);
struct UserKernels {
  void* plain = nullptr;      // hipFunction_t of pr_trace_user
  void* counting = nullptr;   // hipFunction_t of pr_trace_user_count
  int blocks_per_cu = 1;
};
// Loads (building on first use) the code object for the current registry on
// the current device.  Sets the error message and returns non-OK on failure.
pr_status user_kernels(UserKernels* out);
int launch_trace_user(const UserKernels& k, const ReqDev* reqs_dev, QueueDev* queue_dev, const LaunchCfg& cfg,
                      unsigned long long* counts_dev, void* stream);

int launch_trace(const ReqDev* reqs_dev, QueueDev* queue_dev, uint32_t total_jobs, uint32_t n_req,
                 const LaunchCfg& cfg, unsigned long long* counts_dev, void* stream);
int device_cu_count();
int occupancy_blocks_per_cu();
}  // namespace pr
