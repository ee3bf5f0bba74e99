/*
 * stereort.h -- C ABI of the stereo Whitted ray tracer for AMD Instinct MI355X (gfx950).
 *
 * The problem (the paper, Sections 2-3): a stereo pair is two projections of one
 * scene onto the screen plane, one from each of the observer's two eyes, and
 * each projection is synthesised by backward ray tracing.  The two channels
 * ("parallel level 1") and the pixels inside each channel ("parallel level 2")
 * are independent, so both eyes are rendered by one pass over one ray queue.
 * The paper's Table 1 singles out BVH trees as fast to build and GPU-friendly;
 * scenes are accelerated by a BVH built on the device from the Morton order.  The paper
 * reports that up to 40% of its synthesis time goes to CPU-GPU transfer, so the
 * scene stays resident and the images are read back asynchronously.
 *
 * Conventions (every call):
 *   - Returns rt_status; RT_OK == 0.  Never aborts, never throws.  After a
 *     failure rt_last_error() returns a message for the calling thread.
 *   - All device memory is owned by the caller (allocate it with hipMalloc or a
 *     framework allocator); the library owns only small host-side handles.
 *   - Streams are hipStream_t values passed as void*.  NULL is the null stream.
 *   - Work is enqueued asynchronously on the given stream unless a call says
 *     it blocks.
 *
 * Geometry and ids:
 *   - Primitive ids follow input order: triangles [0,T), spheres [T,T+S),
 *     planes [T+S,T+S+P).  -1 means "no hit".
 *   - Closest hit = smallest t; exact ties in t go to the smaller id.
 *     Triangles are closed (edges inclusive), two-sided, Moller-Trumbore.
 *   - Secondary rays (shadow, reflection) start at t > 1e-4 scene units and
 *     skip the primitive they leave.
 *
 * Shading (Whitted recursion without refraction, Phong lighting model):
 *   radiance = ambient*kd + sum over point lights with N.L > 0 and no occluder
 *              of I*(kd*(N.L) + ks*max(0,R.V)^n), R = 2(N.L)N - L
 *            + kr * radiance(mirror ray), up to max_depth mirror bounces;
 *   a ray that hits nothing returns the background colour.  N is the flat
 *   geometric normal turned towards the incoming ray.  No distance falloff.
 *
 * Stereo camera (off-axis pair): eye e in {0 = left, 1 = right} sits at
 *   center + s_e*right, s_0 = -baseline/2, s_1 = +baseline/2, with
 *   right = normalize(up x forward).  The ray of pixel (col, row) (row 0 on
 *   top) passes through the pixel centre of a pinhole image of horizontal
 *   field of view hfov_deg; with convergence > 0 each eye's frustum is sheared
 *   so that both image centres meet at center + convergence*forward.
 */
#ifndef STEREORT_H
#define STEREORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RT_OK = 0,
  RT_ERR_INVALID_ARGUMENT = 1, /* a size, pointer, flag or value is out of range */
  RT_ERR_BUFFER_TOO_SMALL = 2, /* storage / scratch / workspace shorter than required */
  RT_ERR_DEVICE = 3,           /* a HIP runtime call failed, or no usable device */
  RT_ERR_UNSUPPORTED = 4       /* valid but not supported by this build */
} rt_status;

/* Message describing the calling thread's last failure ("" if none).  Valid
 * until the thread's next call into the library. */
const char* rt_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t rt_version(void);

/* ---------------------------------------------------------------------------------------------
 * Scenes
 * ------------------------------------------------------------------------------------------- */

typedef struct {
  float albedo[3];      /* kd: diffuse reflectance, also scales the ambient term */
  float specular[3];    /* ks: Phong specular reflectance */
  float reflectance[3]; /* kr: mirror reflectance (0 = no reflection ray) */
  float shininess;      /* n: Phong exponent, > 0 */
} rt_material;

typedef struct {
  float position[3];
  float intensity[3];
} rt_light;

enum {
  RT_ACCEL_PLOC = 0u,   /* default: triangles through a 4-wide BVH whose binary tree comes from
                           locally-ordered clustering over the Morton order (Meister and Bittner 2018),
                           cut into 4-wide nodes by a surface-area cost table.  If that tree is too deep
                           for the traversal stack (a long chain of nested boxes can make it so), the
                           build falls back to RT_ACCEL_KARRAS and rt_scene_info.builder says so */
  RT_ACCEL_NONE = 1u,   /* brute force: every triangle is tested for every ray */
  RT_ACCEL_KARRAS = 2u, /* the linear BVH proper: binary tree from Karras (2012) emission over the sorted
                           Morton codes and a bottom-up box refit (no SAH), same 4-wide layout */
  /* earlier names of the same values */
  RT_ACCEL_LBVH = RT_ACCEL_PLOC,
  RT_ACCEL_LBVH_KARRAS = RT_ACCEL_KARRAS
};

typedef struct {
  int64_t num_triangles;          /* T >= 0 */
  const float* triangles;         /* device, [T][3][3] vertex positions */
  const uint32_t* tri_material;   /* device, [T] material index */
  int32_t num_spheres;            /* S >= 0 */
  const float* spheres;           /* device, [S][4] centre xyz, radius > 0 */
  const uint32_t* sphere_material;/* device, [S] */
  int32_t num_planes;             /* P >= 0 */
  const float* planes;            /* device, [P][4] unit normal xyz, offset d (points with n.x = d) */
  const uint32_t* plane_material; /* device, [P] */
  int32_t num_materials;          /* 1 .. RT_MAX_MATERIALS */
  const rt_material* materials;   /* host, copied during rt_scene_build */
  int32_t num_lights;             /* 0 .. RT_MAX_LIGHTS */
  const rt_light* lights;         /* host, copied during rt_scene_build */
  float ambient[3];
  float background[3];
  uint32_t flags; /* RT_ACCEL_* */
} rt_scene_desc;

#define RT_MAX_LIGHTS 8
#define RT_MAX_MATERIALS 65536
#define RT_MAX_TRIANGLES ((int64_t)1 << 29)

typedef struct rt_scene_s* rt_scene;

/* Device bytes the built scene occupies (storage) and the temporary device
 * bytes the build needs (scratch), for the counts and flags in desc.  Pure
 * host computation; pointers in desc may be NULL. */
rt_status rt_scene_storage_size(const rt_scene_desc* desc, size_t* storage_bytes, size_t* scratch_bytes);

/* Builds the scene into caller-owned device memory and returns a host handle.
 * Validates the descriptor on the host and the device arrays on the device
 * (finite coordinates, triangle vertices within +-RT_MAX_COORD, positive radii,
 * material indices in range); a bad
 * array gives RT_ERR_INVALID_ARGUMENT.  Copies materials and lights from host
 * memory.  BLOCKS until the build has finished on `stream` (it reads back the
 * validation result).  The input arrays and the scratch may be reused or freed
 * once it returns; `storage` must stay allocated and unmodified until
 * rt_scene_release.  Storage and scratch must be 256-byte aligned. */
rt_status rt_scene_build(const rt_scene_desc* desc, void* storage, size_t storage_bytes, void* scratch,
                         size_t scratch_bytes, void* stream, rt_scene* out);

/* Frees the host handle.  The caller must ensure no render using it is still
 * in flight; storage stays the caller's. */
rt_status rt_scene_release(rt_scene scene);

typedef struct {
  int64_t num_triangles, num_spheres, num_planes, num_lights, num_materials;
  int32_t bvh_depth;     /* levels from the root to the deepest leaf (0 without a BVH) */
  int32_t leaf_size;     /* largest number of triangles per leaf */
  int64_t num_nodes;     /* BVH nodes (node_bytes / num_nodes bytes each) */
  int64_t node_bytes, triangle_bytes;
  float bounds_lo[3], bounds_hi[3];
  int32_t builder;       /* RT_ACCEL_* that built the tree (RT_ACCEL_KARRAS after a fallback; RT_ACCEL_NONE
                            without a tree) */
  int32_t reserved;
} rt_scene_info;

rt_status rt_scene_get_info(rt_scene scene, rt_scene_info* info);

/* ---------------------------------------------------------------------------------------------
 * Stereo rendering
 * ------------------------------------------------------------------------------------------- */

typedef struct {
  float center[3];  /* cyclopean eye position */
  float forward[3]; /* viewing direction (any length > 0) */
  float up[3];      /* not parallel to forward */
  float hfov_deg;   /* horizontal field of view of each eye, (0, 180) */
  float baseline;   /* interocular distance B >= 0 */
  float convergence;/* distance of zero parallax; <= 0 selects parallel axes */
  int32_t width, height; /* per eye, >= 1 */
  int32_t max_depth;     /* mirror bounces after the primary hit, 0 .. RT_MAX_DEPTH */
} rt_stereo_camera;

#define RT_MAX_DEPTH 8
/* Largest |coordinate| of a triangle vertex.  The tree's widest grid step then
 * stays small enough that the traversal's scaled step over a clamped reciprocal
 * direction (up to 1e20) is finite; FP32 triangle tests lose their accuracy long
 * before this scale anyway. */
#define RT_MAX_COORD 1e12f
#define RT_MAX_PIXELS ((int64_t)1 << 28) /* width * height per eye */

enum {
  RT_COUNT_PRIMARY = 0,    /* primary rays traced */
  RT_COUNT_REFLECTION = 1, /* mirror rays traced */
  RT_COUNT_SHADOW = 2,     /* shadow rays traced */
  RT_COUNT_CLOSEST_NODES = 3, /* BVH node visits by closest-hit rays (RT_FLAG_COUNT_WORK) */
  RT_COUNT_CLOSEST_TRIS = 4,  /* triangle tests by closest-hit rays (RT_FLAG_COUNT_WORK) */
  RT_COUNT_ANY_NODES = 5,     /* BVH node visits by shadow rays (RT_FLAG_COUNT_WORK) */
  RT_COUNT_ANY_TRIS = 6,      /* triangle tests by shadow rays (RT_FLAG_COUNT_WORK) */
  RT_COUNT_ERRORS = 7,        /* launches that stopped a ray on an internal consistency check (always 0
                                 unless the library is broken) */
  RT_NUM_COUNTERS = 8
};

typedef struct {
  float* radiance[2];       /* device, [H][W][3] linear RGB per eye (required) */
  float* hit_t[2];          /* device, [H][W] primary hit distance, +inf on a miss (optional) */
  int32_t* hit_prim[2];     /* device, [H][W] primary hit id, -1 on a miss (optional) */
  int32_t* path_prims[2];   /* device, [H][W][D+1] hit id per depth, -1 miss, -2 not spawned
                               (optional, written with RT_FLAG_PATH_IDS) */
  uint8_t* shadow_state[2]; /* device, [H][W][D+1][L] 0 not cast, 1 occluded, 2 visible
                               (optional, written with RT_FLAG_PATH_IDS) */
  float* host_radiance[2];  /* pinned host, [H][W][3]: radiance copied back (optional) */
  int64_t* ray_counts;      /* device, [RT_NUM_COUNTERS]; the render ADDS its counts (optional) */
} rt_stereo_output;

enum {
  RT_FLAG_PATH_IDS = 1u << 0,   /* write path_prims / shadow_state */
  RT_FLAG_COUNT_WORK = 1u << 1, /* count node visits and triangle tests (slower kernels) */
  RT_FLAG_BRUTE_FORCE = 1u << 2, /* test every triangle even if the scene has a BVH */
  RT_FLAG_READBACK_KERNEL = 1u << 3 /* read back through a narrow copy kernel writing through the pinned
                                       buffer's device view (when it has one) instead of the default
                                       hipMemcpyAsync */
};

/* Device workspace bytes for rendering a whole stereo frame of `camera` with
 * `num_lights` lights in one pass.  A smaller workspace is accepted by
 * rt_render_stereo, which then renders the frame in several passes over
 * pixel tiles (results do not depend on the workspace size), down to
 * rt_render_workspace_min. */
rt_status rt_render_workspace_size(const rt_stereo_camera* camera, int32_t num_lights, size_t* bytes);
rt_status rt_render_workspace_min(int32_t num_lights, size_t* bytes);

typedef struct rt_timer_s* rt_timer;

/* Renders both eyes of `camera` into `out`.  Asynchronous on `stream`.  If
 * out->host_radiance is set, the radiance is also copied into that pinned
 * host memory (hipHostMalloc) on `copy_stream` (NULL: on `stream`) once
 * rendering is done;
 * synchronise copy_stream before reading it.  `timer` (optional) records
 * per-kernel device time (see rt_timer_read).  The workspace must be 256-byte
 * aligned and must not be used by another render in flight. */
rt_status rt_render_stereo(rt_scene scene, const rt_stereo_camera* camera, const rt_stereo_output* out,
                           void* workspace, size_t workspace_bytes, uint32_t flags, void* stream,
                           void* copy_stream, rt_timer timer);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): rt_render_stereo with
 * the library's own fixed device scratch as the workspace, so the caller
 * passes only the scene, the camera and the outputs.  The scratch is a
 * file-scope device array of RT_NOALLOC_SCRATCH_BYTES, one per GPU the library
 * runs on, held until the process ends; the frame is rendered in as many
 * passes over pixel tiles as it takes to fit (results are bitwise those of
 * rt_render_stereo).  Nothing is allocated: no hipMalloc, hipFree or timer
 * events.  Every call on one GPU uses that GPU's one array, so calls whose
 * work overlaps on a GPU (on different streams, or from different threads
 * without ordering) RACE and corrupt each other's results: order them on one
 * stream or synchronise between them.  A scene whose smallest pass does not
 * fit the scratch gives RT_ERR_BUFFER_TOO_SMALL (never for RT_MAX_LIGHTS
 * lights and a tree the build accepts).  Asynchronous on `stream`; host
 * readback as in rt_render_stereo. */
#define RT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
rt_status rt_render_stereo_noalloc(rt_scene scene, const rt_stereo_camera* camera, const rt_stereo_output* out,
                                   uint32_t flags, void* stream, void* copy_stream);

typedef struct {
  rt_scene scene;
  rt_stereo_camera camera;
  rt_stereo_output out;
} rt_batch_item;

/* Renders n >= 1 stereo pairs (any mix of scenes, resolutions, depths and
 * baselines) on `stream` as one pipeline: the paths of all items share the
 * ray queues and every traversal launch, so small renders fill the GPU
 * together instead of one after another.  Each item's outputs are bitwise
 * identical to rendering it alone with rt_render_stereo.  The workspace
 * (rt_render_batch_workspace_size for one pass; less makes more passes)
 * starts with the batch's item table.  Host readbacks are ordered on `stream`.
 * The batch's total ray counts are added to items[0].out.ray_counts if set;
 * other items' ray_counts are not written. */
rt_status rt_render_batch_workspace_size(const rt_batch_item* items, int32_t n, size_t* bytes);
rt_status rt_render_batch(const rt_batch_item* items, int32_t n, void* workspace, size_t workspace_bytes,
                          uint32_t flags, void* stream, rt_timer timer);

/* Graph capture of a batch: the render passes of a batch are captured once
 * into a HIP graph and replayed by rt_batch_graph_launch for later batches of
 * the same shape (item count, and per item width, height, max_depth and light
 * count; the scenes, poses, baselines and outputs may change).  Each launch
 * re-uploads the item table outside the graph, replays the graph on `stream`
 * and reads back host_radiance buffers.  The workspace and flags are fixed at
 * capture; items[0].out.ray_counts must stay the same pointer.  Capture
 * enqueues the item-table upload on `stream`, then records the passes without
 * running them. */
typedef struct rt_batch_graph_s* rt_batch_graph;
rt_status rt_batch_graph_create(const rt_batch_item* items, int32_t n, void* workspace, size_t workspace_bytes,
                                uint32_t flags, void* stream, rt_batch_graph* out);
rt_status rt_batch_graph_launch(rt_batch_graph graph, const rt_batch_item* items, int32_t n, void* stream);
rt_status rt_batch_graph_destroy(rt_batch_graph graph);

/* Launch tuning (process-wide).  Results are identical for every setting; only
 * speed changes.  trace_blocks_per_cu: persistent traversal workgroups per CU
 * (0 = as many as fit); stream_blocks: grid of the streaming launches, in units
 * of 256 threads (the shading kernel's 512-thread blocks take half as many);
 * max_pass_paths: largest number of paths per pass (>= 4096).  Defaults: 0, 8192,
 * 2^25. */
typedef struct {
  int32_t trace_blocks_per_cu;
  int32_t stream_blocks;
  int64_t max_pass_paths;
} rt_tuning;
rt_status rt_get_tuning(rt_tuning* out);
rt_status rt_set_tuning(const rt_tuning* tuning);

/* Autotuner: renders the batch (with `repeats` timed repetitions) under each
 * candidate tuning, keeps the fastest, installs it with rt_set_tuning and
 * returns it (and its time per batch in ms).  Blocks until done; the batch's
 * outputs hold a normal render afterwards. */
rt_status rt_autotune_batch(const rt_batch_item* items, int32_t n, void* workspace, size_t workspace_bytes,
                            uint32_t flags, void* stream, int32_t repeats, rt_tuning* best, double* best_ms);

/* ---------------------------------------------------------------------------------------------
 * Stereo-pair building (the paper's post-processing of the two channels, Section 3, Fig. 2)
 * ------------------------------------------------------------------------------------------- */

enum {
  RT_COMPOSE_ANAGLYPH_RED_CYAN = 0, /* W x H: red from the left eye, green and blue from the right */
  RT_COMPOSE_SIDE_BY_SIDE = 1       /* 2W x H: left eye's image, then the right eye's */
};

/* Builds an 8-bit RGBA display image from the two eyes' linear radiance
 * ([H][W][3] FP32 each, device) into `out` (device, 4 bytes per output pixel,
 * RGBA in memory order).  Each channel is encoded as
 * floor(255 * sqrt(clamp(x * exposure, 0, 1)) + 0.5) with correctly rounded
 * FP32 operations; alpha is 255.  Asynchronous on `stream`. */
rt_status rt_compose_stereo(const float* left, const float* right, int32_t width, int32_t height, int32_t mode,
                            float exposure, uint8_t* out, void* stream);

/* Copies `bytes` (a multiple of 4) of device memory into pinned host memory
 * with the narrow readback kernel (hipMemcpyAsync when `host` has no device
 * view).  Asynchronous on `stream`. */
rt_status rt_copy_to_host(const void* device, void* host, size_t bytes, void* stream);

/* ---------------------------------------------------------------------------------------------
 * Per-kernel timing (the paper's per-stage time accounting, Section 4)
 * ------------------------------------------------------------------------------------------- */

enum {
  RT_STAGE_TRACE = 0,    /* BVH traversal: closest-hit rays of depth d fused with shadow rays of depth d-1 */
  RT_STAGE_SHADE = 1,    /* shading and ray spawning */
  RT_STAGE_RESOLVE = 2,  /* adding the unoccluded lights' terms */
  RT_STAGE_SETUP = 3,    /* queue resets and counter updates */
  RT_STAGE_READBACK = 4, /* device-to-host copy */
  RT_NUM_STAGES = 8
};

typedef struct {
  double ms[RT_NUM_STAGES];        /* summed device time */
  int64_t launches[RT_NUM_STAGES]; /* number of timed launches */
} rt_timing;

/* A timer records a HIP event pair around every kernel (and copy) a render
 * enqueues.  rt_timer_read waits for the recorded events, adds their elapsed
 * times into *out (which it does not clear first) and forgets them. */
rt_status rt_timer_create(rt_timer* out);
rt_status rt_timer_destroy(rt_timer timer);
rt_status rt_timer_read(rt_timer timer, rt_timing* out);

#ifdef __cplusplus
}
#endif

#endif /* STEREORT_H */
