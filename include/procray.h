/*
 * procray.h -- C ABI of an MI355X (gfx950) ray tracer for procedural
 * primitives: sphere-traced signed distance functions and distance
 * estimators inside instanced axis-aligned bounding boxes.
 *
 * Paper: V. da Silva, T. Novello, H. Lopes, L. Velho, "Proceduray -- A
 * light-weight engine for procedural primitive ray tracing" (arXiv
 * 2012.10357).  The problem statement follows its host API: procedural
 * geometry is an AABB with a vector of instance transforms (Sec. 3.1 "BLAS
 * from Geometry"; Sec. 4.1, listing "Procedural geometry creation"), the
 * transforms sit in an instance buffer so that intersection runs in local
 * space (Sec. 4.1, listing "Instance buffer creation"), every instance
 * carries a primitive type, a material and an index (Sec. 4.1.1, listing
 * "Shader table entries creation"), rays are of two types -- radiance and
 * shadow -- each with a miss behaviour (listing "Ray creation"), shadow hit
 * groups are intersection-only (listing "Hit group creation"), and a frame
 * is one dispatch over all pixels (Sec. 2.2.3, DispatchRays / ray
 * generation "goes through a pixel").  The DXR shader tables, root
 * signatures and pipeline objects of the paper are replaced by plain
 * records and a type switch inside the kernels.
 *
 * Conventions for every function:
 *  - returns pr_status; on error the out-parameters are left untouched and
 *    pr_last_error() describes the problem (thread-local string);
 *  - every argument is validated on the host before any device work;
 *  - no C++ exception crosses this boundary;
 *  - "device pointer" means memory allocated on the current HIP device
 *    (hipMalloc, torch CUDA tensors); "host pointer" means ordinary memory.
 */
#ifndef PROCRAY_H
#define PROCRAY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_ABI_VERSION 8

typedef enum {
  PR_OK = 0,
  PR_ERR_INVALID_ARG = 1,   /* an argument failed validation */
  PR_ERR_OUT_OF_MEMORY = 2, /* device or pool allocation failed / budget exceeded */
  PR_ERR_DEVICE = 3,        /* a HIP call failed (e.g. no GPU) */
  PR_ERR_NOT_BUILT = 4,     /* render before pr_bvh_build */
  PR_ERR_BUSY = 5,          /* the object is in use by work in flight */
  PR_ERR_UNSUPPORTED = 6,   /* valid but outside what the kernels implement */
  PR_ERR_TIMEOUT = 7        /* a wait ran out of time */
} pr_status;

/* Primitive types.  Parameters (params[0..7], unused entries 0), all in the
 * geometry's local space:
 *   PR_SPHERE      r                            |p| - r
 *   PR_BOX         cx cy cz hx hy hz            exact box SDF
 *   PR_TORUS       R r                          axis = local y
 *   PR_BOXFRAME    b e                          12 edge bars of [-b,b]^3, half-thickness e
 *   PR_PACMAN      R alpha                      sphere R minus the wedge |atan2(y,x)| <= alpha (radians)
 *   PR_JULIA       c0 c1 c2 c3 n_iter bailout   quaternion z <- z^2 + c, z0 = (x,y,z,0)
 *   PR_MANDELBULB  power n_iter bailout         power must be 8; polar axis = local z
 * The sample scene of the paper (Sec. 4, Figs. 1, 4-6) uses pac-men, a 3-D
 * Julia set and a Mandelbulb; the other types are plain SDFs. */
typedef enum {
  PR_SPHERE = 0, PR_BOX = 1, PR_TORUS = 2, PR_BOXFRAME = 3,
  PR_PACMAN = 4, PR_JULIA = 5, PR_MANDELBULB = 6, PR_NUM_TYPES = 7
} pr_prim_type;

typedef struct { float lo[3], hi[3]; } pr_aabb;                          /* local space */

/* One procedural geometry: its type, local AABB and parameters (Sec. 4.1,
 * listing "Procedural geometry creation": a geometry is an AABB), and an
 * optional cutting plane (Fig. 5 shows the Julia set cut by planes).
 *   cut = {nx, ny, nz, d}: only the local half-space n.p <= d is kept, i.e.
 *   the estimator becomes max(DE(p), n.p - d), the CSG intersection of the
 *   primitive with the half-space.  n = (0, 0, 0) means no cut.  A non-zero
 *   n is normalised by pr_scene_create (d is divided by the same |n|).
 * 76 bytes. */
typedef struct { uint32_t type; pr_aabb aabb; float params[8]; float cut[4]; } pr_geometry;

/* One instance: geometry and material indices plus a row-major 3x4
 * local-to-world affine [A | b] (column vectors: world = A local + b).
 * The instance index is its position in the array, the sequential index of
 * Sec. 3.1 "BLAS from Geometry".  56 bytes. */
typedef struct { uint32_t geometry, material; float xform[12]; } pr_instance;

/* Material (the per-primitive constant buffer of Sec. 4.1.1): Lambert albedo
 * and mirror reflectivity rho in [0,1].  16 bytes. */
typedef struct { float albedo[3]; float reflectivity; } pr_material;

/* Scene constants (the scene constant buffer of the global root signature,
 * Sec. 4.1.1): point light, ambient term, background (miss) colour. 40 bytes. */
typedef struct { float light_pos[3], light_rgb[3], ambient, background[3]; } pr_scene_consts;

/* Pinhole camera with a vertical field of view in degrees. 40 bytes. */
typedef struct { float eye[3], target[3], up[3], vfov_deg; } pr_camera;

/* Render options.
 *  seed           jitter seed (64 bit)
 *  spp            samples per pixel, 1..64
 *  jitter         0: pixel centres when spp == 1; otherwise hashed offsets
 *  max_steps      sphere-tracing step budget per (ray, instance), 1..4096
 *  shadows        1: one shadow ray per radiance hit
 *  bounces        0 or 1: one mirror bounce per primary hit when rho > 0
 *  eps            stop threshold on the world-space estimator value (> 0)
 *  tmin, tmax     primary-ray interval, 0 <= tmin < tmax
 *  shadow_offset  secondary-ray origin offset along the normal (world units)
 *  fd_h           central-difference step of the normal (world units)
 *  tile_w, tile_h wave tile shape (tile_w * tile_h == 64) or 0,0 = default
 *  step_budget    march steps between re-balancing points, 0 = default
 *  flags          bit 0 (PR_RENDER_NATURAL_ORDER): hand out tiles in row-major
 *                 order; by default a launch first hands out the tiles of the
 *                 screen rectangle covered by the iterative fractals
 *                 (Julia, Mandelbulb) of scenes with at most 256 instances,
 *                 so their long sphere-tracing chains start early
 *  compact_pct    regrouping of live rays: 1..100 = a lane's sphere-trace
 *                 query waits in a workgroup-wide pool kept per primitive
 *                 type, and each march burst of a wave claims up to
 *                 compact_pct % of 64 waiting queries of the type with the
 *                 most waiting (the higher type on a tie), marches them and
 *                 returns the unfinished ones to the pool; PR_COMPACT_NEVER =
 *                 every wave marches its own lanes' queries; 0 = the choice
 *                 stored for the scene's size class (pr_autotune), else no
 *                 regrouping
 *  reserved       must be 0
 * The five scheduling fields never change results.  72 bytes. */
typedef struct {
  uint64_t seed;
  uint32_t spp, jitter, max_steps, shadows, bounces;
  float eps, tmin, tmax, shadow_offset, fd_h;
  uint32_t tile_w, tile_h, step_budget, flags;
  uint32_t compact_pct, reserved;
} pr_render_opts;
#define PR_RENDER_NATURAL_ORDER 1u
#define PR_COMPACT_NEVER 1000u

/* BVH build options: SAH bins (4..256), maximum leaf size (1..8), traversal
 * and leaf costs; flags bit 0 (PR_BVH_HOST_ONLY) builds without uploading,
 * for inspection with pr_scene_bvh_export.  NULL means defaults
 * {32, 1, 1.0, 4.0, 0}. */
#define PR_BVH_HOST_ONLY 1u
typedef struct { uint32_t sah_bins, max_leaf; float c_node, c_leaf; uint32_t flags; } pr_bvh_opts;

/* Flattened BVH node as exported (32 bytes).  count == 0: interior node with
 * children first and first+1; count > 0: leaf over instance_order[first ..
 * first+count). */
typedef struct { float lo[3]; uint32_t first; float hi[3]; uint32_t count; } pr_bvh_node;

typedef struct pr_scene pr_scene;
typedef struct pr_server pr_server;

/* ---------------------------------------------------------------- scenes */

/* Bound on the magnitude of every sample colour, per channel. */
#define PR_MAX_COLOUR 16777216.0f   /* 2^24 */

/* Copies all host arrays, validates them (known type; finite AABB with
 * lo <= hi; finite transform with |det A| > 1e-12; parameters in range:
 * radii > 0, 1 <= n_iter <= 64, bailout > 0, Mandelbulb power == 8 (else
 * PR_ERR_UNSUPPORTED); geometry and material indices in bounds; 1 <= n_inst
 * <= 16384, so that BVH stack entries fit 16 bits; colours bounded:
 * |background| <= PR_MAX_COLOUR and |albedo| (|ambient| + |light_rgb|) <=
 * PR_MAX_COLOUR per channel and material -- any sign is allowed -- so that
 * every built-in sample colour stays within PR_MAX_COLOUR) and precomputes
 * per-instance records (A^-1, smallest singular value of A, local AABB,
 * parameters, material) on the host.  Touches no
 * device.  The scene is owned by the caller until pr_scene_destroy. */
pr_status pr_scene_create(const pr_geometry* geoms, uint32_t n_geom,
                          const pr_instance* insts, uint32_t n_inst,
                          const pr_material* mats, uint32_t n_mat,
                          const pr_scene_consts* consts, pr_scene** out);

/* Adds a triangle mesh (Sec. 4.1, listing "Triangle geometry creation":
 * vertex and index arrays plus an instance vector; the paper's sample scene
 * has a triangle plane, Fig. 4) to a scene before pr_bvh_build.
 *  vertices   host, n_vertices x 3 float (local xyz)
 *  indices    host, n_triangles x 3 uint32, each < n_vertices
 *  instances  host, n_instances placements: material index and row-major
 *             3x4 local-to-world transform (the geometry field is ignored)
 * Triangles are double-sided and intersected in closed form.  Every
 * (instance, triangle) pair becomes one leaf item of the scene's BVH, in
 * world space; hits on it report the id n_proc + k in out_inst, where
 * n_proc counts the procedural instances of pr_scene_create and k numbers
 * the pairs instance-major across all added meshes.  Validation: finite
 * vertices and transforms (|det A| > 1e-12), indices and materials in
 * range, no degenerate (zero-area) triangle after the transform, at most
 * 16384 items per scene in total.  Clears a previous build; PR_ERR_BUSY
 * while renders of the scene may be in flight. */
pr_status pr_scene_add_mesh(pr_scene* scene, const float* vertices, uint32_t n_vertices,
                            const uint32_t* indices, uint32_t n_triangles,
                            const pr_instance* instances, uint32_t n_instances);

/* Builds a binned-SAH BVH over the instances' world AABBs (the TLAS of
 * Sec. 2.2.3 / Sec. 3.1; each geometry's BLAS is its single AABB) on the
 * host and uploads nodes and instance records to the current device.
 * Returns PR_ERR_BUSY if renders of this scene may still be in flight. */
pr_status pr_bvh_build(pr_scene* scene, const pr_bvh_opts* opts);

/* Copies the host BVH (nodes and the instance order of leaves) out for
 * inspection.  Pass NULL buffers to query the sizes. */
pr_status pr_scene_bvh_export(const pr_scene* scene, pr_bvh_node* nodes, uint32_t node_cap,
                              uint32_t* instance_order, uint32_t order_cap,
                              uint32_t* n_nodes, uint32_t* n_order);

/* Device bytes held by a built scene (instance records + BVH nodes). */
pr_status pr_scene_device_bytes(const pr_scene* scene, uint64_t* bytes);

/* Frees host and device memory.  PR_ERR_BUSY while renders are in flight. */
pr_status pr_scene_destroy(pr_scene* scene);

/* ---------------------------------------------------------- user estimators */

/* Programmable primitives (the flexibility the paper's hit groups and shader
 * tables give, Sec. 2.2.3 and Sec. 3, Eq. 1): a distance estimator supplied
 * as HIP C++ source and compiled into the trace kernel at run time.
 *  name   identifier [A-Za-z_][A-Za-z0-9_]*, at most 48 characters
 *  body   the body of
 *           template <typename R> R est(R x, R y, R z, const float* p)
 *         returning a lower bound on the distance from the local point
 *         (x, y, z) to the surface (negative inside), with p the geometry's
 *         params[0..6] (params[7] is not passed); R is float in the march and
 *         double in the normal taps.
 * On success *type_out receives the new primitive type (PR_USER_TYPE_BASE +
 * k, at most PR_MAX_USER_TYPES per process) for pr_geometry.type.  Launches
 * touching a scene with such a type use a code object built on first use by
 * running hipcc (PR_HIPCC, else /opt/rocm/bin/hipcc) with the library's own
 * flags into a cache directory (PR_USER_CACHE, else $TMPDIR or /tmp); a
 * compile error returns PR_ERR_INVALID_ARG from that render with the
 * compiler's message in pr_last_error().  Registration copies the strings. */
#define PR_USER_TYPE_BASE 8u
#define PR_MAX_USER_TYPES 16u
pr_status pr_register_estimator(const char* name, const char* body, uint32_t* type_out);
/* Compiles the registered estimators now (no device needed), so that source
 * errors surface here rather than at the first render: PR_ERR_INVALID_ARG
 * with the compiler's message.  PR_OK when nothing is registered. */
pr_status pr_build_estimators(void);

/* The closest-hit half of a user hit group (the paper's hit groups pair an
 * intersection routine with a closest-hit shader per geometry, Sec. 2.2.3,
 * Eq. 1; listing "Hit group creation"): hits on instances of user type
 * `type` (from pr_register_estimator) take their colour from this function
 * instead of the built-in Lambert term; the blend with a mirror bounce stays
 * built in.  `body` is HIP C++, the body of
 *   void f(float px, float py, float pz,   world hit point
 *          float nx, float ny, float nz,   unit world normal
 *          float vx, float vy, float vz,   unit direction from the hit toward the ray's origin
 *          float lx, float ly, float lz,   unit direction from the hit toward the light
 *          float lit,                      1 if the shadow ray reached the light (or shadows
 *                                          are off), else 0
 *          const float* albedo,            the instance material's rgb
 *          float ambient, const float* light_rgb,
 *          const float* k,                 the geometry's params[0..6]
 *          float* rgb)                     out: the hit's colour
 * It must depend on its arguments only: it is evaluated for lit = 0 and
 * lit = 1 before the shadow ray returns.  Each output channel is clamped to
 * [-PR_MAX_COLOUR, PR_MAX_COLOUR] (a NaN stays NaN).  One per type; registering again
 * replaces the body.  Built with the estimators (pr_build_estimators or the
 * first render that needs them), with the same errors.  PR_ERR_INVALID_ARG
 * for a type that is not a registered user type or a body that is empty or
 * over 64 KiB; the body is copied. */
pr_status pr_register_closest_hit(uint32_t type, const char* body);

/* ---------------------------------------------------------------- rendering */

/* One frame (DispatchRays, Sec. 2.2.3): per pixel and sample a camera ray,
 * closest-hit traversal, sphere-traced intersection, Lambert shading with
 * a shadow ray and an optional mirror bounce; the colour is the mean over
 * samples.  Enqueued on hip_stream (a hipStream_t, NULL = null stream) and
 * returns immediately.
 *  out_rgb   device, width*height*3 float32, row-major, row 0 = top (required)
 *  out_t     device, width*height float32, primary-ray hit distance of sample
 *            0, +inf on a miss (nullable)
 *  out_inst  device, width*height int32, instance index hit by the primary
 *            ray of sample 0, -1 on a miss (nullable)
 * Output buffers are owned by the caller and must stay alive until the
 * stream has finished.  1 <= width, height <= 16384.
 * With spp > 1 every sample is its own job; the library keeps 28 bytes per
 * pixel of scratch per in-flight launch (grown on demand, kept for reuse) for
 * exact signed fixed-point colour sums (32.32 bits; sample colours are within
 * PR_MAX_COLOUR) and per-pixel sample counters, so results do not depend on
 * the order in which samples finish; a channel that is NaN in any sample is
 * NaN in the mean.
 * PR_ERR_OUT_OF_MEMORY if that scratch cannot be allocated. */
pr_status pr_render(pr_scene* scene, const pr_camera* cam, const pr_render_opts* opts,
                    uint32_t width, uint32_t height,
                    float* out_rgb, float* out_t, int32_t* out_inst, void* hip_stream);

/* pr_render for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc): the
 * same frame and the same results, with no allocation of any kind on the
 * device or in pinned host memory.  The launch record and, for spp > 1, the
 * per-pixel accumulators live in a fixed scratch array of
 * PR_NOALLOC_SCRATCH_BYTES per device, held from the library's first use of
 * the device until the process ends; the request reaches the device as a
 * kernel argument.  Arguments and errors as for pr_render, and:
 *  - spp > 1 needs 4096 + 28 * width * height bytes (rounded up) of the
 *    scratch: at most about 2.39 million pixels (1920x1080 fits); larger
 *    requests return PR_ERR_INVALID_ARG before any device work;
 *  - scenes with user estimators return PR_ERR_UNSUPPORTED (their kernel is
 *    built and loaded at run time);
 *  - every call on a device shares that device's scratch: calls that may
 *    overlap on one device (other streams, other threads) race and must be
 *    serialised by the caller; the array keeps the last call's contents, and
 *    each call clears what it needs at zero itself. */
#define PR_NOALLOC_SCRATCH_BYTES (64u << 20)
pr_status pr_render_noalloc(pr_scene* scene, const pr_camera* cam, const pr_render_opts* opts,
                            uint32_t width, uint32_t height,
                            float* out_rgb, float* out_t, int32_t* out_inst, void* hip_stream);

/* Work counters of one frame, for flop accounting: the same render run by
 * an instrumented build of the kernel (never the timed one), synchronous.
 * counts (host, PR_NUM_COUNTS uint64):
 *   [0..6]   sphere-trace estimator evaluations per primitive type
 *   [7..13]  fractal map iterations inside those evaluations per type
 *   [14..20] estimator evaluations of normals per type
 *   [21..27] fractal iterations inside normal evaluations per type
 *   [28..31] rays: primary, shadow, bounce, bounce-shadow
 *   [32]     BVH nodes visited, [33] candidate slab clips */
#define PR_NUM_COUNTS 34
pr_status pr_render_counts(pr_scene* scene, const pr_camera* cam, const pr_render_opts* opts,
                           uint32_t width, uint32_t height, float* out_rgb, uint64_t* counts);

/* ---------------------------------------------------------------- batching */

typedef struct {
  pr_scene* scene; pr_camera cam; pr_render_opts opts; uint32_t width, height;
  float* out_rgb; float* out_t; int32_t* out_inst;   /* device; out_t/out_inst nullable */
  uint64_t user_tag;
} pr_request;

/* use_graph: 1 = replay a captured hipGraph of (request-table copy, queue
 * reset, persistent kernel); tile_w/tile_h/step_budget/compact_pct: 0 =
 * autotuned (compact_pct as in pr_render_opts, for the whole launch). */
typedef struct { uint32_t tile_w, tile_h, step_budget, use_graph, compact_pct; } pr_batch_opts;

/* Renders n requests (possibly of different scenes, resolutions and sample
 * counts) in one persistent launch that pops tiles from a device queue
 * spanning all requests.  Each request's output equals what pr_render gives
 * for it alone.  Enqueued on hip_stream; 1 <= n <= 4096. */
pr_status pr_render_batch(const pr_request* reqs, uint32_t n, const pr_batch_opts* opts,
                          void* hip_stream);

/* Autotuner: times the candidate tile shapes, step budgets and regrouping
 * choices on the given requests (synchronously, several launches each) and
 * stores the best for scenes of this size class; later calls with 0 fields
 * use it.  best
 * (nullable) receives the choice.  The cache is saved to the JSON file named
 * by the PR_AUTOTUNE_CACHE environment variable when set. */
pr_status pr_autotune(const pr_request* reqs, uint32_t n, pr_batch_opts* best);

/* ---------------------------------------------------------------- serving */

typedef struct {
  uint64_t hbm_budget_bytes;   /* output-pool budget; requests are admitted while they fit */
  uint32_t max_inflight;       /* concurrent launches (streams), 1..8 */
  uint32_t device;             /* HIP device ordinal */
  uint32_t max_batch;          /* requests per launch, 1..4096 */
  uint32_t use_graph;          /* replay captured graphs for launches */
} pr_server_opts;

/* rays_shadow counts the shadow rays of primary and bounce hits, rays_bounce
 * the mirror-bounce rays (both counted on the device as the request runs). */
typedef struct {
  pr_status status;
  const float* rgb; const float* t; const int32_t* inst;  /* device, valid until release */
  uint32_t width, height;
  double t_submit, t_admit, t_launch, t_done;             /* seconds, steady clock */
  uint64_t rays_primary, rays_shadow, rays_bounce, user_tag;
} pr_request_result;

typedef struct {
  uint64_t submitted, admitted, completed, rejected, launches;
  uint64_t pool_bytes_in_use, pool_bytes_peak;
} pr_server_stats;

/* Continuous-batching server: a scheduler thread admits queued requests
 * FIFO while their footprint (outputs, plus the per-sample scratch of
 * requests with spp > 1) fits the budget, launches the admitted
 * ones together on a free stream while earlier launches are still running,
 * and records completion times.  A request completes when its own pixels
 * are done -- the device sets a flag in pinned host memory that the
 * scheduler polls -- so it can be waited for and released while the rest of
 * its launch still runs.  Scenes stay resident on the device. */
pr_status pr_server_create(const pr_server_opts* opts, pr_server** out);
/* The same scheduler driven by a simulated device: a launch "completes"
 * 20 us + us_per_mpix microseconds per million pixel-samples after it
 * starts, and no device memory is allocated or touched (output pointers
 * are placeholders that must not be dereferenced).  Meant for host-only
 * tests of admission, batching and latency accounting; scenes need only a
 * host BVH (PR_BVH_HOST_ONLY). */
pr_status pr_server_create_simulated(const pr_server_opts* opts, uint32_t us_per_mpix,
                                     pr_server** out);
/* Registers a built scene; the server does not take ownership. */
pr_status pr_server_add_scene(pr_server* srv, pr_scene* scene, uint32_t* scene_slot);
/* Queues a request (out_* fields are ignored: the server allocates outputs
 * from its pool).  PR_ERR_OUT_OF_MEMORY if it can never fit the budget. */
pr_status pr_server_submit(pr_server* srv, const pr_request* req, uint64_t* ticket);
/* Waits up to timeout_ms for a ticket; PR_ERR_TIMEOUT if not done. */
pr_status pr_server_wait(pr_server* srv, uint64_t ticket, uint32_t timeout_ms,
                         pr_request_result* out);
/* Returns the ticket's outputs to the pool. */
pr_status pr_server_release(pr_server* srv, uint64_t ticket);
pr_status pr_server_stats_get(pr_server* srv, pr_server_stats* out);
/* Drains in-flight work, then frees everything. */
pr_status pr_server_destroy(pr_server* srv);

/* ---------------------------------------------------------------- misc */

/* Thread-local description of the last error, valid until the next call. */
const char* pr_last_error(void);
/* PR_ABI_VERSION */
uint32_t pr_abi_version(void);
/* Number of HIP devices visible (0 when none); never fails. */
uint32_t pr_device_count(void);
/* Launch shape of the persistent kernel on the current device: compute units
 * and resident workgroups (256 threads each) per compute unit, as used to
 * size every launch's grid.  Both host, non-NULL.  PR_ERR_DEVICE without a
 * GPU. */
pr_status pr_launch_shape(uint32_t* compute_units, uint32_t* workgroups_per_cu);

#ifdef __cplusplus
}
#endif
#endif /* PROCRAY_H */
