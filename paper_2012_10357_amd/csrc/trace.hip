// Persistent ray-tracing kernel for procedural primitives on CDNA4 (gfx950).
//
// What one pixel computes follows the ray-tracing pipeline the paper builds
// on (Sec. 2.2.3): a ray-generation step launches a camera ray through the
// pixel; traversal of the acceleration structure over instanced AABBs finds
// candidate instances; an intersection routine (sphere tracing of the
// primitive's distance estimator in the instance's local space, Sec. 4.1
// "Instance buffer creation") reports hits; the closest hit is shaded
// (Lambert) with a shadow ray whose hit groups are intersection-only
// (listing "Hit group creation"), so any hit occludes; a miss returns the
// background (listing "Ray creation": radiance and shadow miss shaders).
// An optional single mirror bounce per primary hit is shaded the same way.
//
// Execution model (MI355X-native, not the paper's DXR pipeline):
//  - one persistent grid fills the 256 CUs; each lane owns one job, a
//    (pixel, sample), and runs it as a small state machine: traverse ->
//    march -> normal -> shade -> shadow / bounce -> ...;
//  - each loop iteration first refills idle lanes from a device job queue
//    that spans every request of the launch (a wave reserves 64 consecutive
//    jobs per atomic on one of eight partition cursors), then runs the
//    divergent control work, then one pooled FP64 pass over the normal taps
//    the wave's lanes are waiting for, then a burst of up to `step_budget`
//    lock-step FP32 estimator evaluations for all marching lanes (four times
//    that once the queue has no jobs left for the wave); the burst ends
//    early once fewer than an eighth of the busy lanes still march, so
//    finished lanes are re-used without paying a control phase every few
//    steps;
//  - the shadow ray of a primary hit that also bounces is handed to an idle
//    lane of the same wave, so it runs beside the bounce chain;
//  - BVH stacks live in LDS ([depth][lane] layout, conflict-free);
//  - the work is VALU arithmetic (FP32 march, FP64 normal taps); there is
//    no dense contraction, so no MFMA.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "de.h"
#include "internal.h"

namespace pr {

namespace {

constexpr uint32_t M_TRAVERSE = 0, M_MARCH = 1, M_NORMAL = 2, M_RAYDONE = 3, M_IDLE = 4,
                   M_NORMAL_READY = 5, M_WAIT = 6;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kLongJob = 48;    // evaluations after which a pixel counts as long-running
constexpr uint32_t kChunk = 64;      // jobs a wave reserves per queue atomic (>= the 64 lanes)
// ray kinds; odd kinds are shadow rays (any hit ends them).  K_HSHADOW is the
// shadow ray of a primary hit handed off to another lane of the wave.
constexpr uint32_t K_PRIMARY = 0, K_SHADOW = 1, K_BOUNCE = 2, K_BSHADOW = 3, K_HSHADOW = 5;
// hand-off slot states
constexpr uint32_t T_NONE = 0, T_POSTED = 1, T_TAKEN = 2, T_DONE = 3;

__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
  // Wellons' lowbias32 integer hash (public domain): xor-shift / multiply.
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

struct Ray {
  float ox, oy, oz, dx, dy, dz;
};

// Closed-interval slab test of a local ray against the local AABB (zero
// direction components use the containment test).  Returns t0 <= t1 iff the
// instance is a candidate.
__device__ __forceinline__ bool local_slab(const float o[3], const float d[3], const float lo[3],
                                           const float hi[3], float tmin, float tmax, float& t0,
                                           float& t1) {
  t0 = tmin;
  t1 = tmax;
  bool empty = false;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (d[i] != 0.0f) {
      float inv = 1.0f / d[i];
      float ta = (lo[i] - o[i]) * inv;
      float tb = (hi[i] - o[i]) * inv;
      t0 = fmaxf(t0, fminf(ta, tb));
      t1 = fminf(t1, fmaxf(ta, tb));
    } else {
      empty |= (o[i] < lo[i]) || (o[i] > hi[i]);
    }
  }
  return !empty && t0 <= t1;
}

// k-th of n indices visited from the middle outwards: m, m+1, m-1, m+2, ...
__device__ __forceinline__ uint32_t centre_out(uint32_t k, uint32_t n) {
  const uint32_t m = (n - 1) / 2;
  return k == 0 ? m : ((k & 1u) ? m + (k + 1) / 2 : m - k / 2);
}

// The q-th tile a request hands out: first the tiles of its rectangle
// [x0, x1) x [y0, y1), rows and columns each from the middle outwards (the
// fractal bodies sit in the middle), then every other tile in row-major
// order (rows above, the parts of the rectangle's rows left and right of it,
// rows below).  A bijection on [0, tiles_x * tiles_y); an empty rectangle
// gives plain row-major order.
__device__ __forceinline__ void tile_at(const ReqDev* R, uint32_t q, uint32_t& tx, uint32_t& ty) {
  const uint32_t nx = R->tiles_x;
  const uint32_t x0 = R->first_x0, x1 = R->first_x1, y0 = R->first_y0, y1 = R->first_y1;
  const uint32_t w = x1 - x0, h = y1 - y0;
  if (q < w * h) {
    ty = y0 + centre_out(q / w, h);
    tx = x0 + centre_out(q % w, w);
    return;
  }
  q -= w * h;
  if (q < y0 * nx) {
    ty = q / nx;
    tx = q % nx;
    return;
  }
  q -= y0 * nx;
  const uint32_t side = nx - w;   // tiles of a rectangle row outside the rectangle
  if (q < h * side) {
    ty = y0 + q / side;
    const uint32_t c = q % side;
    tx = c < x0 ? c : c + w;
    return;
  }
  q -= h * side;
  ty = y1 + q / nx;
  tx = q % nx;
}

// Ray-triangle distance in world space (Moeller-Trumbore; double-sided,
// closed barycentric bounds), +inf when the ray's line misses the triangle.
// The record holds v0 in Ainv[0..2], e1 = v1 - v0 in Ainv[3..5] and
// e2 = v2 - v0 in Ainv[6..8].
__device__ __forceinline__ float triangle_hit(const InstDev& I, float ox, float oy, float oz, float dx,
                                              float dy, float dz) {
  const float e1x = I.Ainv[3], e1y = I.Ainv[4], e1z = I.Ainv[5];
  const float e2x = I.Ainv[6], e2y = I.Ainv[7], e2z = I.Ainv[8];
  const float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
  const float det = e1x * px + e1y * py + e1z * pz;
  const float inv = 1.0f / det;
  const float sx = ox - I.Ainv[0], sy = oy - I.Ainv[1], sz = oz - I.Ainv[2];
  const float u = (sx * px + sy * py + sz * pz) * inv;
  const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
  const float v = (dx * qx + dy * qy + dz * qz) * inv;
  const float t = (e2x * qx + e2y * qy + e2z * qz) * inv;
  const bool in = det != 0.f && u >= 0.f && u <= 1.f && v >= 0.f && u + v <= 1.f;
  return in ? t : __builtin_inff();
}

// Sphere-trace query of one (ray, instance) pair, kept in LDS in a slot per
// lane, one field per row (structure of arrays, so the lanes of a wave touch
// consecutive words): the local ray, the march interval, the instance
// record's address, and a word packing the steps taken (bits 0-12), the
// march's state (bits 13-14) and the request index (bits 16-31).  A lane
// waiting for a normal keeps its hit in the same slot: local ray, hit
// distance, and the difference step in Q_T1.  Keeping this state in LDS
// rather than registers leaves the registers to the estimators, and lets any
// lane of the workgroup march any query.
constexpr int Q_OX = 0, Q_DX = 3, Q_T = 6, Q_T1 = 7, Q_PLO = 8, Q_PHI = 9, Q_META = 10, kQF = 11;
constexpr uint32_t S_CONT = 0, S_HIT = 1, S_MISS = 2;
constexpr int kTypeKeys = 8;                            // procedural types and the triangle tag

// The cutting plane of an instance along a local ray: n.(o' + t d') - d =
// x + t y, with x = -inf when the instance has no cut.
__device__ __forceinline__ float2 cut_line_of(const InstDev& I, const float ol[3], const float dl[3]) {
  const bool has_cut = I.cut[0] != 0.f || I.cut[1] != 0.f || I.cut[2] != 0.f;
  const float cx = I.cut[0] * ol[0] + I.cut[1] * ol[1] + I.cut[2] * ol[2] - I.cut[3];
  const float cy = I.cut[0] * dl[0] + I.cut[1] * dl[1] + I.cut[2] * dl[2];
  return make_float2(has_cut ? cx : -__builtin_inff(), cy);
}

// The whole path for one workgroup; the kernels below wrap it.  POOL selects
// the regrouping variant (see the burst below).
template <bool COUNT, bool POOL, bool DESCEND>
__device__ __forceinline__ void trace_body(const ReqDev* __restrict__ reqs, QueueDev* __restrict__ queue,
                                           int step_budget, unsigned long long* __restrict__ counts) {
  __shared__ uint16_t stack_mem[kStackDepth][kBlock];
  __shared__ unsigned long long cnt_lds[COUNT ? kNumCounts : 1];
  __shared__ NodeDev lds_nodes[kLdsNodes];
  __shared__ InstDev lds_insts[kLdsInsts];
  __shared__ ReqDev lds_reqs[kLdsReqs];
  __shared__ SceneConstsDev lds_consts;
  // query slots (see Q_*); pooled normal taps: lanes waiting for a normal
  // list themselves, then one wave-wide pass evaluates the six taps of up to
  // ten pending normals, one tap per lane, from the owners' slots
  __shared__ float qs[kQF][kBlock];
  __shared__ float nrm_res[kWavesPerBlock][6][kWave];
  __shared__ uint8_t nrm_owner[kWavesPerBlock][kWave];
  // regrouping variant: per type key, the set of slots whose query waits to
  // be marched (256 bits as 8 words)
  __shared__ uint32_t pend[POOL ? kTypeKeys : 1][POOL ? 8 : 1];
  // Shadow rays of primary hits that go on to a mirror bounce are handed to
  // idle lanes of the same wave, so the shadow ray and the bounce chain run
  // side by side.  Slot = owner lane: shadow-ray origin and Lambert factor,
  // replaced by the shaded primary colour when done; request and instance.
  __shared__ float tk_val[kWavesPerBlock][4][kWave];
  __shared__ uint32_t tk_ref[kWavesPerBlock][kWave];
  __shared__ uint32_t tk_state[kWavesPerBlock][kWave];
  __shared__ uint8_t tk_list[kWavesPerBlock][kWave];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const uint32_t total_jobs = queue->total_jobs;
  const uint32_t n_req = queue->n_req;
  const uint32_t n_sn = queue->n_stage_nodes;
  const uint32_t n_si = queue->n_stage_insts;
  const NodeDev* const staged_nodes_src = queue->stage_nodes;
  const InstDev* const staged_insts_src = queue->stage_insts;
  const SceneConstsDev* const staged_consts_src = queue->stage_consts;
  // stage the shared scene's top BVH levels, first instance records, its
  // constants and the first request records in LDS (16-byte copies)
  {
    const uint4* src = (const uint4*)staged_nodes_src;
    uint4* dst = (uint4*)lds_nodes;
    for (uint32_t i = tid; i < n_sn * 4; i += kBlock) dst[i] = src[i];
    src = (const uint4*)staged_insts_src;
    dst = (uint4*)lds_insts;
    for (uint32_t i = tid; i < n_si * 8; i += kBlock) dst[i] = src[i];
    if (n_sn && tid < (int)(sizeof(SceneConstsDev) / 16))
      ((uint4*)&lds_consts)[tid] = ((const uint4*)staged_consts_src)[tid];
    const uint32_t nr = n_req < kLdsReqs ? n_req : kLdsReqs;
    src = (const uint4*)reqs;
    dst = (uint4*)lds_reqs;
    for (uint32_t i = tid; i < nr * (sizeof(ReqDev) / 16); i += kBlock) dst[i] = src[i];
    if constexpr (COUNT)
      for (int i = tid; i < kNumCounts; i += kBlock) cnt_lds[i] = 0;
    __syncthreads();
  }

  // ---------------- per-lane state
  bool has_job = false;
  bool exhausted = false;
  uint32_t req_i = 0;
  int px = 0, py = 0;
  uint32_t s = 0, spp = 1;

  uint32_t mode = M_IDLE, kind = K_PRIMARY;
  Ray ray;
  float tmin = 0.f, limit = 0.f;  // closest: running best distance; any: tmax
  int best_slot = -1;
  uint32_t best_uid = 0xffffffffu;
  bool occluded = false;
  int sp = 0;
  int leaf_i = 0, leaf_n = 0;

  // current march / normal evaluation
  int cur_slot = -1;
  uint32_t cur_type = 0;
  float t = 0.f;
  uint32_t job_evals = 0;   // estimator evaluations of the current pixel job
  // tracked launches: finished jobs and rays begun for request rc_req, not
  // yet added to the request's device counters
  uint32_t rc_req = 0, rc_jobs = 0, rc_sh = 0, rc_bo = 0;
  uint32_t march_steps = 0; // steps of the current march already counted in job_evals
  int help_owner = -1;      // K_HSHADOW: lane whose primary hit this shadow ray serves
  bool donated = false;     // this lane's primary shadow ray was handed off
  float gx = 0.f, gy = 0.f, gz = 0.f;

  // shading stash
  float sh_lam = 0.f, sh_ar = 0.f, sh_ag = 0.f, sh_ab = 0.f;     // current hit
#ifdef PR_USER_ESTIMATORS
  // a hit shaded by a user closest-hit function: its colour unlit in sh_a*,
  // lit in sh_l* (the shadow ray's outcome selects one)
  bool sh_user = false;
  float sh_lr = 0.f, sh_lg = 0.f, sh_lb = 0.f;
#endif
  float p_cr = 0.f, p_cg = 0.f, p_cb = 0.f, p_rho = 0.f;         // primary local colour, rho
  Ray bounce_ray;
  float hpx = 0.f, hpy = 0.f, hpz = 0.f, hnx = 0.f, hny = 0.f, hnz = 0.f;

  // request constants (reloaded per job)
  const ReqDev* R = reqs;
  const InstDev* insts = nullptr;
  const NodeDev* nodes = nullptr;
  const SceneConstsDev* sc = nullptr;
  uint32_t lim_nodes = 0, lim_insts = 0;   // indices below these are read from LDS

  auto node_ptr = [&](uint32_t i) __attribute__((always_inline)) -> const NodeDev* {
    return i < lim_nodes ? &lds_nodes[i] : &nodes[i];
  };
  auto inst_ptr = [&](int i) __attribute__((always_inline)) -> const InstDev* {
    return (uint32_t)i < lim_insts ? &lds_insts[i] : &insts[i];
  };
  uint32_t max_steps = 1;
  float eps = 1e-4f;

  // post this lane's query (or waiting hit) to its slot
  auto q_post = [&](const InstDev* ip, const float* ol, const float* dl, float a, float b)
                    __attribute__((always_inline)) {
    qs[Q_OX + 0][tid] = ol[0];
    qs[Q_OX + 1][tid] = ol[1];
    qs[Q_OX + 2][tid] = ol[2];
    qs[Q_DX + 0][tid] = dl[0];
    qs[Q_DX + 1][tid] = dl[1];
    qs[Q_DX + 2][tid] = dl[2];
    qs[Q_T][tid] = a;
    qs[Q_T1][tid] = b;
    const uint64_t pv = (uint64_t)(uintptr_t)ip;
    qs[Q_PLO][tid] = __uint_as_float((uint32_t)pv);
    qs[Q_PHI][tid] = __uint_as_float((uint32_t)(pv >> 32));
    qs[Q_META][tid] = __uint_as_float(req_i << 16);
  };

  // the query in this lane's slot starts marching; the regrouping variant
  // also offers it to every wave of the workgroup
  auto start_march = [&]() __attribute__((always_inline)) {
    march_steps = 0;
    mode = M_MARCH;
    if constexpr (POOL) {
      const uint32_t key = cur_type < (uint32_t)kTypeKeys ? cur_type : (uint32_t)kTypeKeys - 1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      atomicOr(&pend[key][tid >> 5], 1u << (tid & 31));
    }
  };

  unsigned long long c_nodes = 0, c_clips = 0;
  // The job queue's partitions (chunk c belongs to partition c mod
  // kQueueParts; a partition's cursor counts its jobs past the chunks that
  // start the grid's waves).  A wave starts on chunk number `gwave` of its
  // home partition gwave mod kQueueParts and moves to the next partition
  // when its current one runs out.  Reservations are partition-local job
  // indices; part_job maps them to job indices.
  const uint32_t n_grid_waves = gridDim.x * (uint32_t)kWavesPerBlock;
  const uint32_t gwave = blockIdx.x * (uint32_t)kWavesPerBlock + (uint32_t)wv;
  const uint32_t n_chunks = (total_jobs + kChunk - 1u) / kChunk;
  auto part_chunks = [](uint32_t p, uint32_t c) -> uint32_t {
    return c > p ? (c - p + kQueueParts - 1u) / kQueueParts : 0u;   // chunks < c in partition p
  };
  uint32_t part = gwave % kQueueParts, part_moves = 0;
  uint32_t part_size = part_chunks(part, n_chunks) * kChunk;         // the partition's jobs
  uint32_t part_first = part_chunks(part, n_grid_waves) * kChunk;    // jobs of its first-round chunks
  auto part_job = [&](uint32_t k) -> uint32_t {
    return k < part_size ? (((k / kChunk) * kQueueParts + part) * kChunk) + k % kChunk : ~0u;
  };
  // this wave's reservation of partition-local job indices (wave-uniform)
  uint32_t res_cur = (gwave / kQueueParts) * kChunk, res_end = res_cur + kChunk;
  uint32_t seen = part_first;          // cursor position after this wave's last reservation
  // the last stretch of a partition: about one chunk for each wave that starts in it
  const uint32_t tail_jobs = n_grid_waves * kChunk / kQueueParts;

  auto begin_ray = [&](const Ray& r, uint32_t k, float t_lo, float t_hi) __attribute__((always_inline)) {
    ray = r;
    kind = k;
    tmin = t_lo;
    limit = t_hi;
    best_slot = -1;
    best_uid = 0xffffffffu;
    occluded = false;
    sp = 0;
    leaf_n = 0;
    leaf_i = 0;
    stack_mem[sp++][tid] = 0;
    mode = M_TRAVERSE;
    if constexpr (COUNT) atomicAdd(&cnt_lds[28 + (k == K_HSHADOW ? K_SHADOW : k)], 1ull);
    // a handed-off shadow ray is counted by the lane that posted it
    rc_sh += (k == K_SHADOW || k == K_BSHADOW) ? 1u : 0u;
    rc_bo += k == K_BOUNCE ? 1u : 0u;
  };

  auto primary_ray = [&]() __attribute__((always_inline)) {
    const float ex = R->eye[0], ey = R->eye[1], ez = R->eye[2];
    const float fx = R->fwd[0], fy = R->fwd[1], fz = R->fwd[2];
    const float rx = R->right[0], ry = R->right[1], rz = R->right[2];
    const float ux = fy * rz - fz * ry, uy = fz * rx - fx * rz, uz = fx * ry - fy * rx;
    float jx = 0.5f, jy = 0.5f;
    if (R->spp != 1 || R->jitter) {
      uint32_t k0 = lowbias32(R->seed_lo ^ lowbias32(R->seed_hi));
      uint32_t k = lowbias32(lowbias32(k0 ^ (uint32_t)(py * R->width + px)) ^ s);
      jx = (float)(lowbias32(k ^ 0xA511E9B3u) >> 8) * (1.0f / 16777216.0f);
      jy = (float)(lowbias32(k ^ 0x63D83595u) >> 8) * (1.0f / 16777216.0f);
    }
    // image-plane coordinates at distance 1 (x right, y up)
    const float kx = R->pix_kx;
    float sx = fmaf((float)px + jx, kx, -0.5f * kx * (float)R->width);
    float sy = fmaf((float)py + jy, R->pix_ky, R->pix_oy);
    float dx = fx + sx * rx + sy * ux, dy = fy + sx * ry + sy * uy, dz = fz + sx * rz + sy * uz;
    float dl = 1.0f / __builtin_sqrtf(dx * dx + dy * dy + dz * dz);
    Ray r{ex, ey, ez, dx * dl, dy * dl, dz * dl};
    begin_ray(r, K_PRIMARY, R->tmin, R->tmax);
  };

  // A job is one sample.  With several samples per pixel the samples of a
  // pixel are consecutive jobs and mostly run on lanes of one wave, but may
  // run on any lanes of any workgroup.  A finished sample's colour is turned
  // into signed 32.32 fixed point and posted to the lane's query slot (the
  // lane is idle from then on); at the start of the wave's next loop
  // iteration the wave sums the posted samples of each pixel (two's-
  // complement integer sums are exact, so nothing depends on which samples
  // meet where or in what order).  A pixel whose samples are all there
  // stores its mean at once.  Otherwise the group adds its sums to the
  // pixel's 64-bit accumulators with device-scope atomics, waits until those
  // adds are performed, then adds its sample count to the pixel's counter;
  // the group that completes the count takes the sums with atomic exchanges,
  // which also clear the accumulators for the next launch, and writes the
  // mean.  Colours are bounded by kMaxColour = 2^24 in magnitude (the scene
  // constants are validated on the host and user closest-hit outputs are
  // clamped), so each term is below 2^56 and 64 of them stay below 2^62.  A
  // NaN channel adds nothing and is counted instead, in a 7-bit field of the
  // counter word per channel (bits 0-6 count samples); the mean of a channel
  // that saw a NaN is NaN, as in floating point.
  bool fin_pend = false;   // a finished sample is posted in this lane's slot
  auto finish_sample = [&](float cr, float cg, float cb) __attribute__((always_inline)) {
    if (spp == 1) {
      float* o = R->out_rgb + ((size_t)py * R->width + px) * 3;
      o[0] = cr;
      o[1] = cg;
      o[2] = cb;
    } else {
      constexpr float kFix = 4294967296.0f;  // 2^32
      const bool nr = cr != cr, ng = cg != cg, nb = cb != cb;
      const uint64_t fr = (uint64_t)__float2ll_rn(nr ? 0.f : cr * kFix);
      const uint64_t fg = (uint64_t)__float2ll_rn(ng ? 0.f : cg * kFix);
      const uint64_t fb = (uint64_t)__float2ll_rn(nb ? 0.f : cb * kFix);
      qs[Q_OX + 0][tid] = __uint_as_float((uint32_t)fr);
      qs[Q_OX + 1][tid] = __uint_as_float((uint32_t)(fr >> 32));
      qs[Q_OX + 2][tid] = __uint_as_float((uint32_t)fg);
      qs[Q_DX + 0][tid] = __uint_as_float((uint32_t)(fg >> 32));
      qs[Q_DX + 1][tid] = __uint_as_float((uint32_t)fb);
      qs[Q_DX + 2][tid] = __uint_as_float((uint32_t)(fb >> 32));
      qs[Q_T][tid] = __uint_as_float(1u + (nr ? 1u << 7 : 0u) + (ng ? 1u << 14 : 0u) + (nb ? 1u << 21 : 0u));
      fin_pend = true;
    }
    ++rc_jobs;
    has_job = false;
    mode = M_IDLE;
  };

  // Sums the posted samples of each pixel (see above).  Runs before any lane
  // is given new work, so each posting lane is still bound to the request
  // and pixel of its sample.
  auto commit_samples = [&]() __attribute__((always_inline)) {
    const unsigned long long pend = __ballot(fin_pend);
    if (pend == 0ull) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // group the posting lanes by (request, pixel); the lowest lane of a
    // group leads it
    const uint32_t pkey = fin_pend ? (uint32_t)py * R->width + (uint32_t)px : 0u;
    unsigned long long grp = 0ull;
    for (unsigned long long rest = pend; rest != 0ull;) {
      const int lead = __ffsll((long long)rest) - 1;
      const uint32_t kr = (uint32_t)__shfl((int)req_i, lead), kp = (uint32_t)__shfl((int)pkey, lead);
      const unsigned long long g = __ballot(fin_pend && req_i == kr && pkey == kp);
      if (lane == lead) grp = g;
      rest &= ~g;
    }
    if (grp != 0ull) {
      uint64_t sr = 0, sg = 0, sb = 0;
      uint32_t add = 0;
      for (unsigned long long m = grp; m != 0ull; m &= m - 1ull) {
        const int sl = wv * kWave + (__ffsll((long long)m) - 1);
        sr += (uint64_t)__float_as_uint(qs[Q_OX + 0][sl]) | ((uint64_t)__float_as_uint(qs[Q_OX + 1][sl]) << 32);
        sg += (uint64_t)__float_as_uint(qs[Q_OX + 2][sl]) | ((uint64_t)__float_as_uint(qs[Q_DX + 0][sl]) << 32);
        sb += (uint64_t)__float_as_uint(qs[Q_DX + 1][sl]) | ((uint64_t)__float_as_uint(qs[Q_DX + 2][sl]) << 32);
        add += __float_as_uint(qs[Q_T][sl]);
      }
      const size_t pix = (size_t)pkey;
      float* o = R->out_rgb + pix * 3;
      uint32_t nan = add;
      bool done = (add & 127u) == spp;
      if (!done) {
        unsigned long long* acc = R->sample_acc + pix * 3;
        atomicAdd(acc + 0, (unsigned long long)sr);
        atomicAdd(acc + 1, (unsigned long long)sg);
        atomicAdd(acc + 2, (unsigned long long)sb);
        // vmcnt also counts stores and atomics without return: wait until the
        // three adds are acknowledged before the counter can reach its total
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        const uint32_t before = atomicAdd(&R->sample_cnt[pix], add);
        nan = before + add;
        done = (nan & 127u) == spp;
        if (done) {
          sr = atomicExch(acc + 0, 0ull);
          sg = atomicExch(acc + 1, 0ull);
          sb = atomicExch(acc + 2, 0ull);
          atomicExch(&R->sample_cnt[pix], 0u);
        }
      }
      if (done) {
        const double scale = 1.0 / (4294967296.0 * (double)spp);
        const double qnan = __builtin_nan("");
        o[0] = (float)((nan >> 7) & 127u ? qnan : (double)(long long)sr * scale);
        o[1] = (float)((nan >> 14) & 127u ? qnan : (double)(long long)sg * scale);
        o[2] = (float)((nan >> 21) & 127u ? qnan : (double)(long long)sb * scale);
      }
    }
    fin_pend = false;
  };

  auto bind_request = [&](uint32_t a) __attribute__((always_inline)) {
    req_i = a;
    R = a < kLdsReqs ? &lds_reqs[a] : reqs + a;
    insts = R->insts;
    nodes = R->nodes;
    sc = R->consts;
    if (n_sn != 0 && nodes == staged_nodes_src) {
      lim_nodes = n_sn;
      lim_insts = n_si;
      sc = &lds_consts;
    } else {
      lim_nodes = 0;
      lim_insts = 0;
    }
    max_steps = R->max_steps;
    eps = R->eps;
    spp = R->spp;
  };

  // the request a global job index belongs to (binary search)
  auto request_of = [&](uint32_t j) __attribute__((always_inline)) -> uint32_t {
    uint32_t a = 0, b = n_req;
    while (b - a > 1) {
      uint32_t m = (a + b) >> 1;
      if (reqs[m].job_begin <= j) a = m; else b = m;
    }
    return a;
  };

  auto start_job = [&](uint32_t j, uint32_t a) __attribute__((always_inline)) {
    bind_request(a);
    rc_req = a;   // counts of another request were flushed before this job
    uint32_t local = j - R->job_begin;
    const uint32_t per_tile = 64u * spp;
    // within a tile the samples of a pixel are consecutive jobs, and an 8x8
    // tile takes its pixels in Z order, so the 64 jobs of a chunk cover an
    // 8x8, 8x4 or 4x4 block of pixels at 1, 2 or 4 samples: the lanes of a
    // wave march nearly the same rays
    const uint32_t q = local / per_tile, rem = local - q * per_tile;
    const uint32_t li = rem / spp;
    const uint32_t tw = R->tile_w, th = 64u / tw;
    uint32_t lx = li % tw, ly = li / tw;
    if (tw == 8u) {
      lx = (li & 1u) | ((li >> 1) & 2u) | ((li >> 2) & 4u);
      ly = ((li >> 1) & 1u) | ((li >> 2) & 2u) | ((li >> 3) & 4u);
    }
    uint32_t tx, ty;
    tile_at(R, q, tx, ty);
    px = (int)(tx * tw + lx);
    py = (int)(ty * th + ly);
    if (px >= (int)R->width || py >= (int)R->height) {
      // ragged tile edge: nothing to render
      ++rc_jobs;
      has_job = false;
      mode = M_IDLE;
      return;
    }
    has_job = true;
    job_evals = 0;
    s = rem - li * spp;
    primary_ray();
  };

  // set up a candidate: local ray, clip, march state; returns true if the lane
  // leaves traversal (marching it, or a shadow ray found an occluder).
  // Triangles are intersected in closed form here (Moeller-Trumbore, world
  // space, double-sided) and never marched.
  auto try_candidate = [&](int slot) __attribute__((always_inline)) -> bool {
    const InstDev& I = *inst_ptr(slot);
    if (I.type == kTriangle) {
      // the hit distance becomes a one-step "march" whose estimate is 0, so
      // the burst records it under the same closest-/any-hit rules
      if (COUNT) ++c_clips;
      const float th = triangle_hit(I, ray.ox, ray.oy, ray.oz, ray.dx, ray.dy, ray.dz);
      if (!(th >= tmin && th <= limit)) return false;
      cur_slot = slot;
      cur_type = kTriangle;
      const float z3[3] = {0.f, 0.f, 0.f};
      q_post(&I, z3, z3, th, th);
      start_march();
      return true;
    }
    float d0 = ray.ox - I.b[0], d1 = ray.oy - I.b[1], d2 = ray.oz - I.b[2];
    float ol[3], dl[3];
    ol[0] = I.Ainv[0] * d0 + I.Ainv[1] * d1 + I.Ainv[2] * d2;
    ol[1] = I.Ainv[3] * d0 + I.Ainv[4] * d1 + I.Ainv[5] * d2;
    ol[2] = I.Ainv[6] * d0 + I.Ainv[7] * d1 + I.Ainv[8] * d2;
    dl[0] = I.Ainv[0] * ray.dx + I.Ainv[1] * ray.dy + I.Ainv[2] * ray.dz;
    dl[1] = I.Ainv[3] * ray.dx + I.Ainv[4] * ray.dy + I.Ainv[5] * ray.dz;
    dl[2] = I.Ainv[6] * ray.dx + I.Ainv[7] * ray.dy + I.Ainv[8] * ray.dz;
    float lo[3] = {I.lo[0], I.lo[1], I.lo[2]}, hi[3] = {I.hi[0], I.hi[1], I.hi[2]};
    float a0, a1;
    if (COUNT) ++c_clips;
    if (!local_slab(ol, dl, lo, hi, tmin, limit, a0, a1)) return false;
    cur_slot = slot;
    cur_type = I.type;
    q_post(&I, ol, dl, a0, a1);
    start_march();
    return true;
  };

  // traversal until a candidate is being marched or the ray is finished.
  // Stack entries (16 bit): an interior node index, or 0x8000 | node << 1 |
  // child for a leaf child whose candidates are deferred (the far child).
  auto traverse = [&]() __attribute__((always_inline)) {
    const float ix = 1.0f / (ray.dx != 0.f ? ray.dx : copysignf(1e-30f, ray.dx));
    const float iy = 1.0f / (ray.dy != 0.f ? ray.dy : copysignf(1e-30f, ray.dy));
    const float iz = 1.0f / (ray.dz != 0.f ? ray.dz : copysignf(1e-30f, ray.dz));
    // slab distances as one FMA each: (b - o) / d = b (1/d) - o (1/d)
    const float oxi = -ray.ox * ix, oyi = -ray.oy * iy, ozi = -ray.oz * iz;
    auto box_entry = [&](const float* lo, const float* hi) __attribute__((always_inline)) -> float {
      float tx0 = fmaf(lo[0], ix, oxi), tx1 = fmaf(hi[0], ix, oxi);
      float ty0 = fmaf(lo[1], iy, oyi), ty1 = fmaf(hi[1], iy, oyi);
      float tz0 = fmaf(lo[2], iz, ozi), tz1 = fmaf(hi[2], iz, ozi);
      float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), tmin));
      float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), limit));
      return tn <= tf ? tn : __builtin_inff();
    };
    for (;;) {
      while (leaf_i < leaf_n) {
        int slot = leaf_i++;
        if (try_candidate(slot)) return;
      }
      if (sp == 0) {
        mode = M_RAYDONE;
        return;
      }
      uint32_t e = stack_mem[--sp][tid];
      if constexpr (!DESCEND) {
        if (e & 0x8000u) {
          // deferred leaf child: read its range from the parent record
          const NodeDev* pn = node_ptr((e & 0x7fffu) >> 1);
          const uint32_t c = (e & 1u) ? pn->c1 : pn->c0;
          const uint32_t n = (e & 1u) ? pn->n1 : pn->n0;
          leaf_i = (int)c;
          leaf_n = (int)(c + n);
          continue;
        }
        const NodeDev nd = *node_ptr(e);
        if (COUNT) ++c_nodes;
        const float t0 = box_entry(nd.lo0, nd.hi0);
        const float t1c = (nd.n1 != kNoChild) ? box_entry(nd.lo1, nd.hi1) : __builtin_inff();
        const bool h0 = t0 != __builtin_inff(), h1 = t1c != __builtin_inff();
        if (!h0 && !h1) continue;
        // near child first; the far one (if hit) goes on the stack
        const bool near0 = h0 && (!h1 || t0 <= t1c);
        if (h0 && h1) {
          const uint32_t fc = near0 ? nd.c1 : nd.c0, fn = near0 ? nd.n1 : nd.n0;
          stack_mem[sp++][tid] = (uint16_t)(fn == 0 ? fc : (0x8000u | (e << 1) | (near0 ? 1u : 0u)));
        }
        const uint32_t nc = near0 ? nd.c0 : nd.c1, nn = near0 ? nd.n0 : nd.n1;
        if (nn == 0) {
          stack_mem[sp++][tid] = (uint16_t)nc;
        } else {
          leaf_i = (int)nc;
          leaf_n = (int)(nc + nn);
        }
      } else {
        // the four-wide tree (launches whose BVH is not all in LDS); stack
        // entries: a node index, or 0x8000 | node << 2 | child for a
        // deferred leaf child
        // child c's reference by selects on its two index bits (an equality
        // chain on c becomes a divergent branch tree, four per node visit)
        auto ref_at = [](const Node4Dev& nd, uint32_t c) __attribute__((always_inline)) -> uint32_t {
          const uint32_t r01 = (c & 1u) ? nd.ref1 : nd.ref0, r23 = (c & 1u) ? nd.ref3 : nd.ref2;
          return (c & 2u) ? r23 : r01;
        };
        if (e & 0x8000u) {
          const Node4Dev& pn = *(const Node4Dev*)node_ptr((e & 0x7fffu) >> 2);
          const uint32_t r = ref_at(pn, e & 3u);
          leaf_i = (int)(r & 0xffffffu);
          leaf_n = leaf_i + (int)((r >> 24) & 0x7fu) + 1;
          continue;
        }
        // descend: the nearest child next (an interior one without the
        // stack), the other hit children on the stack, farthest first
        for (;;) {
          const Node4Dev nd = *(const Node4Dev*)node_ptr(e);
          // slab distances of the grid boxes: (org + q step - o) / d
          const float sx = nd.step[0] * ix, sy = nd.step[1] * iy, sz = nd.step[2] * iz;
          const float bx = fmaf(nd.org[0], ix, oxi), by = fmaf(nd.org[1], iy, oyi), bz = fmaf(nd.org[2], iz, ozi);
          // children as sort keys: the entry distance's bits (it is at least
          // tmin >= 0, so with the sign of a -0 cleared the bits order as the
          // floats do) with the child index in the low two bits, 0x7f800000 | c
          // for a missed or absent child
          uint32_t key[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint8_t* q = nd.q + 6 * c;
            const float tx0 = fmaf((float)q[0], sx, bx), tx1 = fmaf((float)q[3], sx, bx);
            const float ty0 = fmaf((float)q[1], sy, by), ty1 = fmaf((float)q[4], sy, by);
            const float tz0 = fmaf((float)q[2], sz, bz), tz1 = fmaf((float)q[5], sz, bz);
            const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), tmin));
            const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), limit));
            const bool hit = ref_at(nd, (uint32_t)c) != kNoRef && tn <= tf;
            key[c] = (hit ? (__float_as_uint(tn) & 0x7ffffffcu) : 0x7f800000u) | (uint32_t)c;
          }
          // nearest first (ties within the two dropped bits by child index)
          auto cswap = [&](int a, int b) __attribute__((always_inline)) {
            const uint32_t lo = min(key[a], key[b]), hi = max(key[a], key[b]);
            key[a] = lo;
            key[b] = hi;
          };
          cswap(0, 1);
          cswap(2, 3);
          cswap(0, 2);
          cswap(1, 3);
          cswap(1, 2);
          if (key[0] >= 0x7f800000u) break;
#pragma unroll
          for (int k = 3; k >= 1; --k) {
            if (key[k] < 0x7f800000u) {
              const uint32_t c = key[k] & 3u, r = ref_at(nd, c);
              stack_mem[sp++][tid] = (uint16_t)((r >> 31) ? (0x8000u | (e << 2) | c) : r);
            }
          }
          const uint32_t r = ref_at(nd, key[0] & 3u);
          if (!(r >> 31)) {
            e = r;
            continue;
          }
          leaf_i = (int)(r & 0xffffffu);
          leaf_n = leaf_i + (int)((r >> 24) & 0x7fu) + 1;
          break;
        }
      }
    }
  };

  auto start_normal = [&](int slot, float th) __attribute__((always_inline)) {
    const InstDev* ip = inst_ptr(slot);
    const InstDev& I = *ip;
    if (I.type == kTriangle) {
      // face normal from the record, no estimator taps
      cur_slot = slot;
      t = th;
      mode = M_NORMAL_READY;
      return;
    }
    float d0 = ray.ox - I.b[0], d1 = ray.oy - I.b[1], d2 = ray.oz - I.b[2];
    float ol0 = I.Ainv[0] * d0 + I.Ainv[1] * d1 + I.Ainv[2] * d2;
    float ol1 = I.Ainv[3] * d0 + I.Ainv[4] * d1 + I.Ainv[5] * d2;
    float ol2 = I.Ainv[6] * d0 + I.Ainv[7] * d1 + I.Ainv[8] * d2;
    float dl0 = I.Ainv[0] * ray.dx + I.Ainv[1] * ray.dy + I.Ainv[2] * ray.dz;
    float dl1 = I.Ainv[3] * ray.dx + I.Ainv[4] * ray.dy + I.Ainv[5] * ray.dz;
    float dl2 = I.Ainv[6] * ray.dx + I.Ainv[7] * ray.dy + I.Ainv[8] * ray.dz;
    const float ol[3] = {ol0, ol1, ol2}, dl[3] = {dl0, dl1, dl2};
    q_post(ip, ol, dl, th, R->fd_h / I.sigma);
    cur_slot = slot;
    t = th;
    mode = M_NORMAL;
  };

  // mirror bounce from the primary hit: r = d - 2 (d.n) n, origin offset
  // along the normal
  auto start_bounce = [&]() __attribute__((always_inline)) {
    float dn = bounce_ray.dx * hnx + bounce_ray.dy * hny + bounce_ray.dz * hnz;
    float rx = bounce_ray.dx - 2.f * dn * hnx;
    float ry = bounce_ray.dy - 2.f * dn * hny;
    float rz = bounce_ray.dz - 2.f * dn * hnz;
    const float off = R->shadow_offset;
    Ray br{hpx + off * hnx, hpy + off * hny, hpz + off * hnz, rx, ry, rz};
    begin_ray(br, K_BOUNCE, 0.0f, R->tmax);
  };

  // run the handed-off shadow ray of lane `owner` (another lane's, or this
  // lane's own when nobody took it)
  auto run_handoff = [&](int owner) __attribute__((always_inline)) {
    help_owner = owner;
    if (owner != lane) {
      bind_request(tk_ref[wv][owner] >> 14);
      has_job = true;
      job_evals = 0;
    }
    const float sx = tk_val[wv][0][owner], sy = tk_val[wv][1][owner], sz = tk_val[wv][2][owner];
    float vx = sc->light[0] - sx, vy = sc->light[1] - sy, vz = sc->light[2] - sz;
    float dist = __builtin_sqrtf(vx * vx + vy * vy + vz * vz);
    float idist = 1.0f / dist;
    Ray srr{sx, sy, sz, vx * idist, vy * idist, vz * idist};
    begin_ray(srr, K_HSHADOW, 0.0f, dist);
  };

  // normal finished: shade prep, spawn the shadow ray (or skip it)
  auto after_normal = [&]() __attribute__((always_inline)) {
    const InstDev& I = *inst_ptr(cur_slot);
    float nx, ny, nz;
    if (I.type == kTriangle) {
      // double-sided: the face normal turned toward the incoming ray
      const float fx = I.b[0], fy = I.b[1], fz = I.b[2];
      const float side = (fx * ray.dx + fy * ray.dy + fz * ray.dz) > 0.f ? -1.f : 1.f;
      nx = side * fx;
      ny = side * fy;
      nz = side * fz;
    } else {
      nx = I.Ainv[0] * gx + I.Ainv[3] * gy + I.Ainv[6] * gz;   // A^-T g
      ny = I.Ainv[1] * gx + I.Ainv[4] * gy + I.Ainv[7] * gz;
      nz = I.Ainv[2] * gx + I.Ainv[5] * gy + I.Ainv[8] * gz;
      float ln = __builtin_sqrtf(nx * nx + ny * ny + nz * nz);
      if (ln > 0.f) {
        float il = 1.0f / ln;
        nx *= il; ny *= il; nz *= il;
      } else {
        nx = -ray.dx; ny = -ray.dy; nz = -ray.dz;
      }
    }
    float hx = ray.ox + t * ray.dx, hy = ray.oy + t * ray.dy, hz = ray.oz + t * ray.dz;
    float lx = sc->light[0] - hx, ly = sc->light[1] - hy, lz = sc->light[2] - hz;
    float ll = 1.0f / __builtin_sqrtf(lx * lx + ly * ly + lz * lz);
    sh_lam = fmaxf(0.f, (nx * lx + ny * ly + nz * lz) * ll);
    const float* mat = sc->shade + 4 * cur_slot;
    sh_ar = mat[0]; sh_ag = mat[1]; sh_ab = mat[2];
    const float refl = mat[3];
    hpx = hx; hpy = hy; hpz = hz; hnx = nx; hny = ny; hnz = nz;
    if (kind == K_PRIMARY) p_rho = refl;
    const float off = R->shadow_offset;
#ifdef PR_USER_ESTIMATORS
    // The type's closest-hit function, if one is registered, for both
    // outcomes of the shadow ray; such a hit traces its own shadow ray.
    sh_user = false;
    if (I.type >= PR_USER_TYPE_BASE) {
      float c0[3], c1[3];
      const float lux = lx * ll, luy = ly * ll, luz = lz * ll;
      if (user_shade(I.type, hx, hy, hz, nx, ny, nz, -ray.dx, -ray.dy, -ray.dz, lux, luy, luz, 0.f, mat,
                     sc->ambient, sc->light_rgb, I.prm, c0)) {
        user_shade(I.type, hx, hy, hz, nx, ny, nz, -ray.dx, -ray.dy, -ray.dz, lux, luy, luz, 1.f, mat,
                   sc->ambient, sc->light_rgb, I.prm, c1);
        sh_user = true;
        // outputs are clamped to the colour bound (NaN stays NaN)
        auto clampc = [](float v) { return v != v ? v : fminf(fmaxf(v, -kMaxColour), kMaxColour); };
        sh_ar = clampc(c0[0]); sh_ag = clampc(c0[1]); sh_ab = clampc(c0[2]);
        sh_lr = clampc(c1[0]); sh_lg = clampc(c1[1]); sh_lb = clampc(c1[2]);
      }
    }
    const bool may_hand_off = !sh_user;
#else
    constexpr bool may_hand_off = true;
#endif
    if (may_hand_off && kind == K_PRIMARY && R->shadows && R->bounces >= 1 && refl > 0.f) {
      // hand the shadow ray to an idle lane and start the mirror bounce now
      tk_val[wv][0][lane] = hx + off * nx;
      tk_val[wv][1][lane] = hy + off * ny;
      tk_val[wv][2][lane] = hz + off * nz;
      tk_val[wv][3][lane] = sh_lam;
      tk_ref[wv][lane] = (req_i << 14) | (uint32_t)cur_slot;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      tk_state[wv][lane] = T_POSTED;
      donated = true;
      ++rc_sh;
      start_bounce();
      return;
    }
    if (R->shadows) {
      float sx = hx + off * nx, sy = hy + off * ny, sz = hz + off * nz;
      float vx = sc->light[0] - sx, vy = sc->light[1] - sy, vz = sc->light[2] - sz;
      float dist = __builtin_sqrtf(vx * vx + vy * vy + vz * vz);
      float idist = 1.0f / dist;
      Ray srr{sx, sy, sz, vx * idist, vy * idist, vz * idist};
      uint32_t k = (kind == K_PRIMARY) ? K_SHADOW : K_BSHADOW;
      begin_ray(srr, k, 0.0f, dist);
    } else {
      occluded = false;
      kind = (kind == K_PRIMARY) ? K_SHADOW : K_BSHADOW;
      mode = M_RAYDONE;
    }
  };

  auto lambert = [&](float V, float& cr, float& cg, float& cb) __attribute__((always_inline)) {
#ifdef PR_USER_ESTIMATORS
    if (sh_user) {
      cr = V > 0.f ? sh_lr : sh_ar;
      cg = V > 0.f ? sh_lg : sh_ag;
      cb = V > 0.f ? sh_lb : sh_ab;
      return;
    }
#endif
    const float amb = sc->ambient;
    cr = sh_ar * (amb + V * sh_lam * sc->light_rgb[0]);
    cg = sh_ag * (amb + V * sh_lam * sc->light_rgb[1]);
    cb = sh_ab * (amb + V * sh_lam * sc->light_rgb[2]);
  };

  // The owner of a handed-off shadow ray, its bounce colour kept in p_c*:
  // combine once the primary colour is published, run the shadow ray itself
  // if no lane took it, or wait for the lane that did.
  auto collect = [&]() __attribute__((always_inline)) {
    const uint32_t st = tk_state[wv][lane];
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (st == T_DONE) {
      const float rho = p_rho;
      const float cr = tk_val[wv][0][lane], cg = tk_val[wv][1][lane], cb = tk_val[wv][2][lane];
      tk_state[wv][lane] = T_NONE;
      donated = false;
      finish_sample((1.f - rho) * cr + rho * p_cr, (1.f - rho) * cg + rho * p_cg,
                    (1.f - rho) * cb + rho * p_cb);
    } else if (st == T_POSTED) {
      tk_state[wv][lane] = T_TAKEN;
      run_handoff(lane);
    } else {
      mode = M_WAIT;
    }
  };

  // the mirror bounce's colour is known: blend with the primary colour
  auto end_bounce = [&](float br, float bg, float bb) __attribute__((always_inline)) {
    if (donated) {
      p_cr = br;
      p_cg = bg;
      p_cb = bb;
      collect();
      return;
    }
    const float rho = p_rho;
    finish_sample((1.f - rho) * p_cr + rho * br, (1.f - rho) * p_cg + rho * bg,
                  (1.f - rho) * p_cb + rho * bb);
  };

  // a ray has finished traversal: move the pixel's pipeline forward
  auto ray_done = [&]() __attribute__((always_inline)) {
    switch (kind) {
      case K_PRIMARY: {
        if (s == 0) {
          // depth and instance of sample 0's primary hit
          const size_t pix = (size_t)py * R->width + px;
          if (R->out_t) R->out_t[pix] = best_slot >= 0 ? limit : __builtin_inff();
          if (R->out_inst) R->out_inst[pix] = best_slot >= 0 ? (int)best_uid : -1;
        }
        if (best_slot < 0) {
          finish_sample(sc->background[0], sc->background[1], sc->background[2]);
        } else {
          start_normal(best_slot, limit);
        }
        break;
      }
      case K_SHADOW: {
        float cr, cg, cb;
        lambert(occluded ? 0.f : 1.f, cr, cg, cb);
        if (R->bounces >= 1 && p_rho > 0.f) {
          p_cr = cr; p_cg = cg; p_cb = cb;
          start_bounce();
        } else {
          finish_sample(cr, cg, cb);
        }
        break;
      }
      case K_BOUNCE: {
        if (best_slot < 0) {
          end_bounce(sc->background[0], sc->background[1], sc->background[2]);
        } else {
          start_normal(best_slot, limit);
        }
        break;
      }
      case K_BSHADOW: {
        float cr, cg, cb;
        lambert(occluded ? 0.f : 1.f, cr, cg, cb);
        end_bounce(cr, cg, cb);
        break;
      }
      default: {  // K_HSHADOW: shade the owner's primary hit, publish it
        const int ow = help_owner;
        const float* mat = sc->shade + 4 * (tk_ref[wv][ow] & 0x3fffu);
        const float lam = tk_val[wv][3][ow];
        const float V = occluded ? 0.f : 1.f;
        const float amb = sc->ambient;
        tk_val[wv][0][ow] = mat[0] * (amb + V * lam * sc->light_rgb[0]);
        tk_val[wv][1][ow] = mat[1] * (amb + V * lam * sc->light_rgb[1]);
        tk_val[wv][2][ow] = mat[2] * (amb + V * lam * sc->light_rgb[2]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        tk_state[wv][ow] = T_DONE;
        help_owner = -1;
        if (ow == lane) {
          collect();
        } else {
          has_job = false;
          mode = M_IDLE;
        }
        break;
      }
    }
  };

  // a march stopped with v < eps at t: record the hit
  auto record_hit = [&]() __attribute__((always_inline)) {
    if (kind & 1u) {
      occluded = true;
      mode = M_RAYDONE;
    } else {
      // closest hit: lexicographic minimum of (t, instance index)
      const uint32_t u = __float_as_uint(inst_ptr(cur_slot)->prm[7]);
      if (best_slot < 0 || t < limit || (t == limit && u < best_uid)) {
        limit = t;
        best_slot = cur_slot;
        best_uid = u;
      }
      mode = M_TRAVERSE;
    }
  };

  // A burst of up to `budget` lock-step estimator evaluations of the query
  // in slot q (for lanes with act): v = sigma DE(o' + t d'); hit if v < eps,
  // else t += v; miss once t passes t1 or the step budget is spent, or on a
  // NaN.  The burst ends once fewer than an eighth of end_n queries still
  // march: a control phase costs about four steps, so lanes that have
  // finished wait a few steps rather than forcing one.  The outcome and the
  // steps taken go back to the slot; returns the query's state.
  auto march_query = [&](bool act, int q, int end_n, int budget) __attribute__((always_inline)) -> uint32_t {
    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f, tq = 0.f, t1q = 0.f, sg = 1.f;
    float kp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float2 cl = make_float2(-__builtin_inff(), 0.f);
    uint32_t meta = 0, ty = kTriangle;
    float eq = 1.f;
    int mq = 1;
    if (act) {
      ox = qs[Q_OX + 0][q]; oy = qs[Q_OX + 1][q]; oz = qs[Q_OX + 2][q];
      dx = qs[Q_DX + 0][q]; dy = qs[Q_DX + 1][q]; dz = qs[Q_DX + 2][q];
      tq = qs[Q_T][q];
      t1q = qs[Q_T1][q];
      meta = __float_as_uint(qs[Q_META][q]);
      const InstDev* ip = (const InstDev*)(uintptr_t)((uint64_t)__float_as_uint(qs[Q_PLO][q]) |
                                                      ((uint64_t)__float_as_uint(qs[Q_PHI][q]) << 32));
      ty = ip->type;
      if (ty != kTriangle) {
        sg = ip->sigma;
#pragma unroll
        for (int i = 0; i < 6; ++i) kp[i] = ip->prm[i];
        const float o3[3] = {ox, oy, oz}, d3[3] = {dx, dy, dz};
        cl = cut_line_of(*ip, o3, d3);
      }
      const uint32_t rq = meta >> 16;
      const ReqDev* Rq = rq < kLdsReqs ? &lds_reqs[rq] : reqs + rq;
      eq = Rq->eps;
      mq = (int)Rq->max_steps;
    }
    int sq = (int)(meta & 0x1fffu);
    uint32_t st = S_CONT;
    const bool qcut = __ballot(act && cl.x != -__builtin_inff()) != 0ull;
    for (int it = 0; it < budget; ++it) {
      if (act && st == S_CONT) {
        const float qx = ox + tq * dx;
        const float qy = oy + tq * dy;
        const float qz = oz + tq * dz;
        int iters = 0;
        float de = 0.f;  // a triangle's hit was found in closed form: a zero estimate
        if (ty != kTriangle) de = de_eval(ty, qx, qy, qz, kp, &iters);
        if (qcut) {
          if (cl.x != -__builtin_inff() && de == de) de = fmaxf(de, cl.x + tq * cl.y);
        }
        if constexpr (COUNT) if (ty < PR_NUM_TYPES) {
          atomicAdd(&cnt_lds[ty], 1ull);
          atomicAdd(&cnt_lds[7 + ty], (unsigned long long)iters);
        }
        const float v = sg * de;
        const bool step = v >= eq;
        tq = step ? tq + v : tq;
        sq += step ? 1 : 0;
        if (!step || tq > t1q || sq >= mq) st = v < eq ? S_HIT : S_MISS;
      }
      const unsigned long long still = __ballot(act && st == S_CONT);
      if (still == 0ull || 8 * __popcll(still) < end_n) break;
    }
    if (act) {
      qs[Q_T][q] = tq;
      if constexpr (POOL) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      qs[Q_META][q] = __uint_as_float((meta & 0xffff0000u) | (st << 13) | (uint32_t)sq);
    }
    return st;
  };

  // regrouping variant: queries a wave claims per burst, compact_pct % of 64
  const uint32_t claim_cap = POOL ? max(1u, min(64u, (queue->compact_pct * 64u + 99u) / 100u)) : 64u;

  // Regrouping variant: the wave takes up to claim_cap waiting queries of the type
  // key that has the most (the higher key on a tie: the fractals), from any wave of the
  // workgroup, marches them in one burst, and offers the unfinished ones
  // again.  The waiting sets are words of LDS bits claimed by atomic
  // exchange, so no wave ever waits for another; a query is marched by one
  // wave at a time, and each (ray, instance) march is the same sequence as
  // in its own lane.
  auto pool_burst = [&]() __attribute__((always_inline)) {
    // lanes 8 k .. 8 k + 7 read the 8 words of key k
    const uint32_t word = pend[lane >> 3][lane & 7];
    uint32_t c = (uint32_t)__popc(word);
    c += (uint32_t)__shfl_xor((int)c, 1);
    c += (uint32_t)__shfl_xor((int)c, 2);
    c += (uint32_t)__shfl_xor((int)c, 4);
    uint32_t score = (c << 3) | (uint32_t)(lane >> 3);
    score = max(score, (uint32_t)__shfl_xor((int)score, 8));
    score = max(score, (uint32_t)__shfl_xor((int)score, 16));
    score = max(score, (uint32_t)__shfl_xor((int)score, 32));
    if ((score >> 3) == 0u) {
      __builtin_amdgcn_s_sleep(1);   // every waiting query is being marched elsewhere
      return;
    }
    const uint32_t k = score & 7u;
    uint32_t got = lane < 8 ? atomicExch(&pend[k][lane], 0u) : 0u;
    const uint32_t cnt = (uint32_t)__popc(got);
    uint32_t inc = cnt;
#pragma unroll
    for (int d = 1; d < 8; d <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)inc, d);
      if (lane >= d) inc += v;
    }
    const uint32_t exc = inc - cnt;
    const uint32_t keep = exc < claim_cap ? min(cnt, claim_cap - exc) : 0u;
    if (lane < 8 && keep < cnt) {
      // give back the claimed bits past the first `keep` ones
      uint32_t back = got;
      for (uint32_t i = 0; i < keep; ++i) back &= back - 1u;
      atomicOr(&pend[k][lane], back);
      got &= ~back;
    }
    const uint32_t n_take = min((uint32_t)__shfl((int)inc, 7), claim_cap);
    // lane j takes the j-th kept query in slot order
    uint32_t myw = 0, wi = 0, r = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const uint32_t gw = (uint32_t)__shfl((int)got, w), ew = (uint32_t)__shfl((int)exc, w);
      const uint32_t kw = (uint32_t)__popc(gw);
      if ((uint32_t)lane >= ew && (uint32_t)lane < ew + kw) {
        myw = gw;
        wi = (uint32_t)w;
        r = (uint32_t)lane - ew;
      }
    }
    for (uint32_t i = 0; i < r; ++i) myw &= myw - 1u;
    const bool act = (uint32_t)lane < n_take;
    const int q = act ? (int)(wi * 32u + (uint32_t)__ffs(myw) - 1u) : tid;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t st = march_query(act, q, (int)n_take, step_budget);
    if (act && st == S_CONT) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      atomicOr(&pend[k][q >> 5], 1u << (q & 31));
    }
  };

  // Tracked launches: the lanes that want it (want) add their finished jobs,
  // with the rays they began, to their request's device counters -- summed
  // over the wave per request, one atomic each.  All of the wave's pixel
  // stores are made visible first, and the ray counts are added before the
  // job count, so the wave whose add completes a request's job count sees
  // every pixel and ray of it: it copies the ray totals into the request's
  // host-visible record and sets its done flag (system scope).  A lane keeps
  // counting while it works for one request and flushes only before a job
  // of another one or when it runs out of jobs, since the fence and the
  // atomics are costly (the counts belong to rc_req however the lane is
  // occupied meanwhile: a lane helping another with its shadow ray begins no
  // counted ray).
  unsigned long long* const track = queue->track;
  DoneRec* const done_recs = queue->done_recs;
  auto flush_counts = [&](bool want) __attribute__((always_inline)) {
    const bool fl = want && (rc_jobs | rc_sh | rc_bo) != 0u;
    unsigned long long m = __ballot(fl);
    if (m == 0ull) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    while (m != 0ull) {
      const int leader = __ffsll((long long)m) - 1;
      const uint32_t r = (uint32_t)__shfl((int)rc_req, leader);
      const bool sel = fl && rc_req == r;
      uint32_t j = sel ? rc_jobs : 0u, a = sel ? rc_sh : 0u, b = sel ? rc_bo : 0u;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        j += (uint32_t)__shfl_xor((int)j, d);
        a += (uint32_t)__shfl_xor((int)a, d);
        b += (uint32_t)__shfl_xor((int)b, d);
      }
      if (lane == leader) {
        const ReqDev* Rr = r < kLdsReqs ? &lds_reqs[r] : reqs + r;
        const unsigned long long total = (unsigned long long)(Rr->job_end - Rr->job_begin);
        unsigned long long* tr = track + 3 * (size_t)r;
        if (a) atomicAdd(tr + 1, (unsigned long long)a);
        if (b) atomicAdd(tr + 2, (unsigned long long)b);
        const unsigned long long before =
            __hip_atomic_fetch_add(tr, (unsigned long long)j, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (before + j == total) {
          DoneRec* dr = done_recs + r;
          dr->rays_shadow = __hip_atomic_load(tr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          dr->rays_bounce = __hip_atomic_load(tr + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&dr->done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
      if (sel) rc_jobs = rc_sh = rc_bo = 0u;
      m &= ~__ballot(sel);
    }
  };

  // ---------------- main loop
  if constexpr (POOL) {
    if (tid < kTypeKeys * 8) pend[tid >> 3][tid & 7] = 0u;
    __syncthreads();
  }
  tk_state[wv][lane] = T_NONE;
  for (;;) {
    // owners waiting for a handed-off shadow ray; then idle lanes take the
    // posted ones (in lane order) before new jobs
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (has_job && mode == M_WAIT) collect();
    commit_samples();
    const unsigned long long posted = __ballot(tk_state[wv][lane] == T_POSTED);
    if (posted) {
      const unsigned long long idle = __ballot(!has_job);
      if (idle) {
        const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if (tk_state[wv][lane] == T_POSTED) tk_list[wv][__popcll(posted & lt)] = (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (!has_job) {
          const uint32_t r = (uint32_t)__popcll(idle & lt);
          if (r < (uint32_t)__popcll(posted)) {
            const int owner = tk_list[wv][r];
            tk_state[wv][owner] = T_TAKEN;
            run_handoff(owner);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    // Refill idle lanes.  Each wave holds a reservation of consecutive
    // indices [res_cur, res_end) of its current partition and takes a fresh
    // chunk of kChunk jobs with one atomic on the partition's cursor only
    // when the reservation cannot serve all idle lanes; a partition hands out
    // its jobs in increasing order, so once a lane draws an index past its
    // end, every index still reserved there is past the end too, and the
    // wave moves on to the next partition that has jobs beyond its first
    // round (after all of them, the wave's lanes are exhausted).
    const unsigned long long need = __ballot(!has_job && !exhausted);
    if (need) {
      const int leader = __ffsll((long long)need) - 1;
      const uint32_t n = (uint32_t)__popcll(need);
      const uint32_t have = res_end - res_cur;
      // near the end of the partition a wave takes only the jobs it can
      // start now, so no job waits in a busy wave's reservation while other
      // waves run dry
      const uint32_t take = (part_size - (seen < part_size ? seen : part_size)) < tail_jobs
                                ? n - (have < n ? have : n)
                                : kChunk;
      uint32_t nbase = 0;
      if (have < n) {
        if (lane == leader) nbase = atomicAdd(&queue->cursor[part][0], take) + part_first;
        nbase = __shfl(nbase, leader);
        seen = nbase + take;
      }
      uint32_t j = ~0u, a = 0;
      if (!has_job && !exhausted) {
        const uint32_t rank =
            (uint32_t)__popcll(need & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        j = part_job(rank < have ? res_cur + rank : nbase + (rank - have));
        if (j < total_jobs) a = request_of(j);
      }
      const bool ran_out = __ballot((!has_job && !exhausted) && j >= total_jobs) != 0ull;
      // a lane's counts are added to its request's counters before it starts
      // a job of another request, or once its partition runs out
      if (track) flush_counts((!has_job && !exhausted) && (j >= total_jobs || a != rc_req));
      if (!has_job && !exhausted && j < total_jobs) start_job(j, a);
      if (ran_out) {
        do {
          part = (part + 1u) % kQueueParts;
          ++part_moves;
          part_size = part_chunks(part, n_chunks) * kChunk;
          part_first = part_chunks(part, n_grid_waves) * kChunk;
        } while (part_moves < kQueueParts && part_size <= part_first);
        if (part_moves >= kQueueParts) exhausted = true;
        res_cur = res_end = 0;
        seen = part_first;
      } else if (have < n) {
        res_cur = nbase + (n - have);
        res_end = nbase + take;
      } else {
        res_cur += n;
      }
    }

    // marching lanes take their march's progress and outcome from their slots
    if (has_job && mode == M_MARCH) {
      const uint32_t meta = __float_as_uint(qs[Q_META][tid]);
      const uint32_t st = (meta >> 13) & 3u, sn = meta & 0x1fffu;
      job_evals += sn - march_steps;
      march_steps = sn;
      if (st != S_CONT) {
        if constexpr (POOL) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (st == S_HIT) {
          ++job_evals;
          t = qs[Q_T][tid];
          record_hit();
        } else {
          mode = M_TRAVERSE;
        }
      }
    }

    // control: advance every lane to its next estimator evaluation
    auto control = [&]() __attribute__((always_inline)) {
      while (has_job && mode != M_MARCH && mode != M_NORMAL && mode != M_WAIT) {
        if (mode == M_TRAVERSE) {
          traverse();
        } else if (mode == M_NORMAL_READY) {
          after_normal();
        } else if (mode == M_RAYDONE) {
          if (kind == K_PRIMARY) {
            // keep the primary direction for the mirror bounce
            bounce_ray = ray;
          }
          ray_done();
        }
      }
    };
    control();

    // pooled FP64 normal taps: lane j of a pass evaluates tap (j mod 6) of
    // the (j div 6)-th waiting lane
    const unsigned long long want = __ballot(has_job && mode == M_NORMAL);
    if (want) {
      if (has_job && mode == M_NORMAL) {
        const uint32_t rank =
            (uint32_t)__popcll(want & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        nrm_owner[wv][rank] = (uint8_t)lane;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const uint32_t n_taps = 6u * (uint32_t)__popcll(want);
      for (uint32_t base = 0; base < n_taps; base += kWave) {
        const uint32_t j = base + (uint32_t)lane;
        if (j < n_taps) {
          const uint32_t owner = nrm_owner[wv][j / 6];
          const uint32_t tap = j % 6, ax = tap >> 1;
          // the owner's hit: local ray, distance and step from its slot; the
          // hit point in FP64
          const int os = wv * kWave + (int)owner;
          const double tt = (double)qs[Q_T][os];
          const double px_ = (double)qs[Q_OX + 0][os] + tt * (double)qs[Q_DX + 0][os];
          const double py_ = (double)qs[Q_OX + 1][os] + tt * (double)qs[Q_DX + 1][os];
          const double pz_ = (double)qs[Q_OX + 2][os] + tt * (double)qs[Q_DX + 2][os];
          const double h = (tap & 1) ? -(double)qs[Q_T1][os] : (double)qs[Q_T1][os];
          const InstDev* ip = (const InstDev*)(uintptr_t)((uint64_t)__float_as_uint(qs[Q_PLO][os]) |
                                                          ((uint64_t)__float_as_uint(qs[Q_PHI][os]) << 32));
          float kp[6];
#pragma unroll
          for (int i = 0; i < 6; ++i) kp[i] = ip->prm[i];
          const uint32_t ty = ip->type;
          int iters;
          const double qx = px_ + (ax == 0 ? h : 0.0);
          const double qy = py_ + (ax == 1 ? h : 0.0);
          const double qz = pz_ + (ax == 2 ? h : 0.0);
          double v = de_eval64(ty, qx, qy, qz, kp, &iters);
          const float* cu = ip->cut;
          if (cu[0] != 0.f || cu[1] != 0.f || cu[2] != 0.f) {
            // CSG intersection with the kept half-space (NaN stays NaN)
            const double g = (double)cu[0] * qx + (double)cu[1] * qy + (double)cu[2] * qz - (double)cu[3];
            if (v == v) v = v > g ? v : g;
          }
          nrm_res[wv][tap][owner] = (float)v;
          if constexpr (COUNT) if (ty < PR_NUM_TYPES) {
            atomicAdd(&cnt_lds[14 + ty], 1ull);
            atomicAdd(&cnt_lds[21 + ty], (unsigned long long)iters);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (has_job && mode == M_NORMAL) {
        gx = nrm_res[wv][0][lane] - nrm_res[wv][1][lane];
        gy = nrm_res[wv][2][lane] - nrm_res[wv][3][lane];
        gz = nrm_res[wv][4][lane] - nrm_res[wv][5][lane];
        mode = M_NORMAL_READY;
      }
      control();
    }

    const unsigned long long busy = __ballot(has_job);
    if (!busy) {
      if (__ballot(!exhausted) == 0ull) break;
      continue;
    }
    // waves holding long-running pixels get issue priority, the longer the
    // higher: the slowest pixel chains bound the frame time
    constexpr uint32_t long_job = DESCEND ? 64u : kLongJob;
    if (__ballot(has_job && job_evals > 4 * long_job)) {
      __builtin_amdgcn_s_setprio(3);
    } else if (__ballot(has_job && job_evals > 2 * long_job)) {
      __builtin_amdgcn_s_setprio(2);
    } else if (__ballot(has_job && job_evals > long_job)) {
      __builtin_amdgcn_s_setprio(1);
    } else {
      __builtin_amdgcn_s_setprio(0);
    }

    if constexpr (POOL) {
      pool_burst();
    } else {
      // once the queue has nothing left for this wave, no lane waits for a
      // refill: bursts run four times longer, so the wave's last pixel
      // chains pass through fewer control phases
      const bool marching = has_job && mode == M_MARCH;
      const int budget = __ballot(!exhausted) == 0ull ? 4 * step_budget : step_budget;
      if (__ballot(marching)) march_query(marching, tid, __popcll(busy), budget);
    }
  }

  commit_samples();
  if (track) flush_counts(true);
  if constexpr (COUNT) {
    atomicAdd(&cnt_lds[32], c_nodes);
    atomicAdd(&cnt_lds[33], c_clips);
    __syncthreads();
    for (int i = tid; i < kNumCounts; i += kBlock) atomicAdd(&counts[i], cnt_lds[i]);
  }
}

}  // namespace

#ifndef PR_USER_ESTIMATORS

template <bool COUNT, bool POOL, bool DESCEND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void trace_kernel(
    const ReqDev* __restrict__ reqs, QueueDev* __restrict__ queue, int step_budget,
    unsigned long long* __restrict__ counts) {
  trace_body<COUNT, POOL, DESCEND>(reqs, queue, step_budget, counts);
}

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n;
}

int occupancy_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, trace_kernel<false, false, false>, kBlock, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int launch_trace(const ReqDev* reqs_dev, QueueDev* queue_dev, uint32_t total_jobs, uint32_t n_req,
                 const LaunchCfg& cfg, unsigned long long* counts_dev, void* stream) {
  (void)total_jobs;
  (void)n_req;
  dim3 grid(cfg.grid_blocks), block(kBlock);
  // the queue header carries the same compact_pct; it selects the kernel,
  // and so does whether the launch's BVH is all staged in LDS (see traverse)
  auto k = counts_dev ? (cfg.compact_pct > 0 ? trace_kernel<true, true, false> : trace_kernel<true, false, false>)
                      : (cfg.compact_pct > 0 ? trace_kernel<false, true, false>
                                             : (cfg.descend ? trace_kernel<false, false, true>
                                                            : trace_kernel<false, false, false>));
  hipLaunchKernelGGL(k, grid, block, 0, (hipStream_t)stream, reqs_dev, queue_dev, cfg.step_budget, counts_dev);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#endif  // !PR_USER_ESTIMATORS

}  // namespace pr

#ifdef PR_USER_ESTIMATORS
// Entry points of the run-time build that includes user estimators; looked
// up by name in the loaded code object.
extern "C" __global__ __launch_bounds__(pr::kBlock) __attribute__((amdgpu_waves_per_eu(3))) void pr_trace_user(
    const pr::ReqDev* __restrict__ reqs, pr::QueueDev* __restrict__ queue, int step_budget,
    unsigned long long* __restrict__ counts) {
  pr::trace_body<false, false, false>(reqs, queue, step_budget, counts);
}
extern "C" __global__ __launch_bounds__(pr::kBlock) __attribute__((amdgpu_waves_per_eu(3))) void pr_trace_user_count(
    const pr::ReqDev* __restrict__ reqs, pr::QueueDev* __restrict__ queue, int step_budget,
    unsigned long long* __restrict__ counts) {
  pr::trace_body<true, false, false>(reqs, queue, step_budget, counts);
}
#endif
