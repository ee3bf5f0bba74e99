// C ABI of the stereo ray tracer: argument validation, memory planning, timers and the
// host-side driving of the device passes.  No kernels live here.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rt_internal.h"

namespace srt {

struct Scene {
  DevScene dev;
  int device;
  rt_scene_info info;
};

struct TimerImpl {
  struct Rec {
    int stage;
    hipEvent_t start, end;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t pending_start = nullptr;
  int pending_stage = -1;
  hipError_t error = hipSuccess;

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      error = r;
      return nullptr;
    }
    return e;
  }
};

void timer_begin(TimerImpl* t, int stage, hipStream_t s) {
  hipEvent_t e = t->take();
  if (!e) return;
  hipError_t r = hipEventRecord(e, s);
  if (r != hipSuccess) t->error = r;
  t->pending_start = e;
  t->pending_stage = stage;
}

void timer_end(TimerImpl* t, int stage, hipStream_t s) {
  if (!t->pending_start || t->pending_stage != stage) return;
  hipEvent_t e = t->take();
  if (!e) return;
  hipError_t r = hipEventRecord(e, s);
  if (r != hipSuccess) t->error = r;
  t->recs.push_back({stage, t->pending_start, e});
  t->pending_start = nullptr;
  t->pending_stage = -1;
}

}  // namespace srt

struct rt_scene_s : srt::Scene {};
struct rt_timer_s : srt::TimerImpl {};

namespace {

thread_local std::string g_error;

// Launch tuning (process-wide): results never depend on it, only speed does.
std::mutex g_tuning_mutex;
rt_tuning g_tuning = {0, 8192, int64_t(1) << 25};

rt_tuning current_tuning() {
  std::lock_guard<std::mutex> lock(g_tuning_mutex);
  return g_tuning;
}

rt_status fail(rt_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

rt_status ok() {
  g_error.clear();
  return RT_OK;
}

rt_status hip_fail(hipError_t e, const char* what) {
  return fail(RT_ERR_DEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

rt_status validate_desc(const rt_scene_desc* d) {
  if (!d) return fail(RT_ERR_INVALID_ARGUMENT, "scene descriptor is NULL");
  if (d->num_triangles < 0 || d->num_triangles > RT_MAX_TRIANGLES)
    return fail(RT_ERR_INVALID_ARGUMENT, "num_triangles %lld out of range [0, %lld]", (long long)d->num_triangles,
                (long long)RT_MAX_TRIANGLES);
  if (d->num_spheres < 0 || d->num_spheres > (1 << 20))
    return fail(RT_ERR_INVALID_ARGUMENT, "num_spheres %d out of range", d->num_spheres);
  if (d->num_planes < 0 || d->num_planes > (1 << 16))
    return fail(RT_ERR_INVALID_ARGUMENT, "num_planes %d out of range", d->num_planes);
  if (d->num_materials < 1 || d->num_materials > RT_MAX_MATERIALS)
    return fail(RT_ERR_INVALID_ARGUMENT, "num_materials %d out of range [1, %d]", d->num_materials, RT_MAX_MATERIALS);
  if (d->num_lights < 0 || d->num_lights > RT_MAX_LIGHTS)
    return fail(RT_ERR_INVALID_ARGUMENT, "num_lights %d out of range [0, %d]", d->num_lights, RT_MAX_LIGHTS);
  if (d->flags != RT_ACCEL_PLOC && d->flags != RT_ACCEL_NONE && d->flags != RT_ACCEL_KARRAS)
    return fail(RT_ERR_INVALID_ARGUMENT, "unknown scene flags 0x%x", d->flags);
  if (!finite3(d->ambient) || !finite3(d->background))
    return fail(RT_ERR_INVALID_ARGUMENT, "ambient and background must be finite");
  return RT_OK;
}

rt_status validate_camera(const rt_stereo_camera* c) {
  if (!c) return fail(RT_ERR_INVALID_ARGUMENT, "camera is NULL");
  if (!finite3(c->center) || !finite3(c->forward) || !finite3(c->up))
    return fail(RT_ERR_INVALID_ARGUMENT, "camera vectors must be finite");
  if (!(c->hfov_deg > 0.f && c->hfov_deg < 180.f))
    return fail(RT_ERR_INVALID_ARGUMENT, "hfov_deg %g outside (0, 180)", double(c->hfov_deg));
  if (!(std::isfinite(c->baseline) && c->baseline >= 0.f))
    return fail(RT_ERR_INVALID_ARGUMENT, "baseline must be finite and >= 0");
  if (!std::isfinite(c->convergence)) return fail(RT_ERR_INVALID_ARGUMENT, "convergence must be finite");
  if (c->width < 1 || c->height < 1 || int64_t(c->width) * c->height > RT_MAX_PIXELS)
    return fail(RT_ERR_INVALID_ARGUMENT, "image size %dx%d out of range", c->width, c->height);
  if (c->max_depth < 0 || c->max_depth > RT_MAX_DEPTH)
    return fail(RT_ERR_INVALID_ARGUMENT, "max_depth %d out of range [0, %d]", c->max_depth, RT_MAX_DEPTH);
  double f[3] = {c->forward[0], c->forward[1], c->forward[2]}, u[3] = {c->up[0], c->up[1], c->up[2]};
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0.0)) return fail(RT_ERR_INVALID_ARGUMENT, "forward must be non-zero");
  double cr[3] = {u[1] * f[2] - u[2] * f[1], u[2] * f[0] - u[0] * f[2], u[0] * f[1] - u[1] * f[0]};
  double cl = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  double ul = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (!(cl > 1e-12 * fl * ul)) return fail(RT_ERR_INVALID_ARGUMENT, "up must not be parallel to forward");
  return RT_OK;
}

srt::DevCamera make_dev_camera(const rt_stereo_camera* c) {
  srt::DevCamera d{};
  double f[3], up[3];
  for (int k = 0; k < 3; ++k) {
    d.C[k] = c->center[k];
    f[k] = c->forward[k];
    up[k] = c->up[k];
  }
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (int k = 0; k < 3; ++k) d.f[k] = f[k] / fl;
  double r[3] = {up[1] * d.f[2] - up[2] * d.f[1], up[2] * d.f[0] - up[0] * d.f[2], up[0] * d.f[1] - up[1] * d.f[0]};
  double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (int k = 0; k < 3; ++k) d.r[k] = r[k] / rl;
  d.u[0] = d.f[1] * d.r[2] - d.f[2] * d.r[1];
  d.u[1] = d.f[2] * d.r[0] - d.f[0] * d.r[2];
  d.u[2] = d.f[0] * d.r[1] - d.f[1] * d.r[0];
  const double half = 0.5 * double(c->hfov_deg) * M_PI / 180.0;
  d.fpx = 0.5 * double(c->width) / std::tan(half);
  d.cx = 0.5 * double(c->width);
  d.cy = 0.5 * double(c->height);
  d.half_baseline = 0.5 * double(c->baseline);
  d.inv_convergence = c->convergence > 0.f ? 1.0 / double(c->convergence) : 0.0;
  d.W = c->width;
  d.H = c->height;
  d.D = c->max_depth;
  d.tiles_x = (c->width + srt::kTile - 1) / srt::kTile;
  d.tiles_y = (c->height + srt::kTile - 1) / srt::kTile;
  return d;
}

int64_t total_paths(const rt_stereo_camera* c) {
  int64_t tx = (c->width + srt::kTile - 1) / srt::kTile, ty = (c->height + srt::kTile - 1) / srt::kTile;
  return tx * ty * srt::kPathsPerTile;
}

constexpr int64_t kMinChunk = 32 * srt::kPathsPerTile;
constexpr int64_t kMaxChunk = int64_t(1) << 25;

// Largest pass size (multiple of a tile pair) whose workspace fits `bytes`.  stack_entries / stack_threads
// size the traversal-stack spill area (0: the most any accepted tree and grid can need).
int64_t chunk_for(int64_t total, int32_t L, size_t bytes, srt::RenderPlan* plan, int stack_entries = 0,
                  int stack_threads = 0) {
  const int64_t cap = std::max<int64_t>(kMinChunk, std::min(kMaxChunk, current_tuning().max_pass_paths));
  int64_t hi_tiles = std::max<int64_t>(1, std::min(total, cap) / srt::kPathsPerTile);
  int64_t lo_tiles = std::min<int64_t>(kMinChunk / srt::kPathsPerTile, hi_tiles);
  auto need = [&](int64_t tiles) {
    return srt::plan_render(tiles * srt::kPathsPerTile, L, 0, plan, stack_entries, stack_threads);
  };
  if (need(lo_tiles) > bytes) return 0;
  while (lo_tiles < hi_tiles) {
    int64_t mid = (lo_tiles + hi_tiles + 1) / 2;
    if (need(mid) <= bytes)
      lo_tiles = mid;
    else
      hi_tiles = mid - 1;
  }
  need(lo_tiles);
  return lo_tiles * srt::kPathsPerTile;
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

rt_status check_output(const rt_stereo_output* o, uint32_t flags) {
  if (!o) return fail(RT_ERR_INVALID_ARGUMENT, "output is NULL");
  if (!o->radiance[0] || !o->radiance[1]) return fail(RT_ERR_INVALID_ARGUMENT, "radiance outputs are required");
  if ((flags & RT_FLAG_PATH_IDS) &&
      !(o->path_prims[0] && o->path_prims[1] && o->shadow_state[0] && o->shadow_state[1]))
    return fail(RT_ERR_INVALID_ARGUMENT, "RT_FLAG_PATH_IDS needs path_prims and shadow_state for both eyes");
  if (!!o->host_radiance[0] != !!o->host_radiance[1])
    return fail(RT_ERR_INVALID_ARGUMENT, "host_radiance must be given for both eyes or neither");
  return RT_OK;
}

constexpr uint32_t kKnownFlags = RT_FLAG_PATH_IDS | RT_FLAG_COUNT_WORK | RT_FLAG_BRUTE_FORCE | RT_FLAG_READBACK_KERNEL;
constexpr int kReadbackBlocks = 32;

srt::DevOutputs dev_outputs(const rt_stereo_output* o, uint32_t flags) {
  srt::DevOutputs d{};
  const bool ids = (flags & RT_FLAG_PATH_IDS) != 0;
  for (int e = 0; e < 2; ++e) {
    d.radiance[e] = o->radiance[e];
    d.hit_t[e] = o->hit_t[e];
    d.hit_prim[e] = o->hit_prim[e];
    d.path_prims[e] = ids ? o->path_prims[e] : nullptr;
    d.shadow_state[e] = ids ? o->shadow_state[e] : nullptr;
  }
  return d;
}

// Copies both eyes' radiance into the pinned host buffers of `out`, ordered after `stream`.
rt_status readback(const rt_stereo_camera* cam, const rt_stereo_output* out, uint32_t flags, hipStream_t stream,
                   hipStream_t copy_stream, srt::TimerImpl* timer) {
  if (!out->host_radiance[0]) return RT_OK;
  const size_t bytes = size_t(cam->width) * size_t(cam->height) * 12;
  hipStream_t cs = copy_stream ? copy_stream : stream;
  hipError_t e = hipSuccess;
  if (cs != stream) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipEventRecord(ev, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(e, "stream ordering for readback");
  }
  // Default: hipMemcpyAsync.  With RT_FLAG_READBACK_KERNEL a narrow copy kernel (a few
  // workgroups) writes through the pinned buffer's device view instead, when the buffer has one.
  void* dview[2] = {nullptr, nullptr};
  bool use_kernel = (flags & RT_FLAG_READBACK_KERNEL) != 0;
  for (int eye = 0; eye < 2 && use_kernel; ++eye)
    if (hipHostGetDevicePointer(&dview[eye], out->host_radiance[eye], 0) != hipSuccess || !dview[eye]) {
      (void)hipGetLastError();
      use_kernel = false;
    }
  if (timer) srt::timer_begin(timer, RT_STAGE_READBACK, cs);
  for (int eye = 0; eye < 2 && e == hipSuccess; ++eye)
    e = use_kernel ? srt::copy_to_host(out->radiance[eye], dview[eye], bytes, kReadbackBlocks, cs)
                   : hipMemcpyAsync(out->host_radiance[eye], out->radiance[eye], bytes, hipMemcpyDeviceToHost, cs);
  if (timer) srt::timer_end(timer, RT_STAGE_READBACK, cs);
  if (e != hipSuccess) return hip_fail(e, "readback");
  return RT_OK;
}

srt::BuildPlan plan_for(const rt_scene_desc* d, bool ploc) {
  return srt::plan_build(d->num_triangles, d->num_spheres, d->num_planes, d->num_materials, d->num_lights,
                         d->flags != RT_ACCEL_NONE, ploc);
}

// The traversal stack holds at most (width - 1) entries per level of the tree.
bool stack_fits(int32_t depth) { return (srt::kNodeWidth - 1) * depth < srt::kStackMax; }

rt_status build_status(const srt::BuildResult& res) {
  if (res.status_bits & 1u)
    return fail(RT_ERR_INVALID_ARGUMENT, "a triangle vertex is not finite or exceeds %g in magnitude", RT_MAX_COORD);
  if (res.status_bits & 2u) return fail(RT_ERR_INVALID_ARGUMENT, "a triangle material index is out of range");
  if (res.status_bits & 4u)
    return fail(RT_ERR_INVALID_ARGUMENT, "a sphere is not finite, has radius <= 0 or a material out of range");
  if (res.status_bits & 8u)
    return fail(RT_ERR_INVALID_ARGUMENT, "a plane is not finite, has a zero normal or a material out of range");
  if (res.status_bits & 16u) return fail(RT_ERR_DEVICE, "internal error: inconsistent BVH hierarchy");
  return RT_OK;
}

rt_status current_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  return RT_OK;
}

// Renders the frame in passes of `chunk` paths with the workspace laid out by `plan`.
rt_status render_passes(const rt_scene_s* scene, const rt_stereo_camera* cam, const rt_stereo_output* out, char* ws,
                        const srt::RenderPlan& plan, int64_t chunk, uint32_t flags, hipStream_t stream,
                        hipStream_t copy_stream, srt::TimerImpl* timer) {
  const int64_t total = total_paths(cam);
  srt::RenderArgs ra{};
  ra.stream_blocks = current_tuning().stream_blocks;
  ra.one.sc = scene->dev;
  ra.one.cam = make_dev_camera(cam);
  ra.one.out = dev_outputs(out, flags);
  ra.one.path_offset = 0;
  ra.items = nullptr;
  ra.num_items = 1;
  ra.max_lights = scene->dev.L;
  ra.max_depth = cam->max_depth;
  ra.ray_counts = out->ray_counts;
  ra.flags = flags;
  ra.ws = ws;
  ra.plan = plan;
  for (int64_t begin = 0; begin < total; begin += chunk) {
    ra.path_begin = begin;
    ra.path_count = std::min(chunk, total - begin);
    hipError_t e = srt::render_chunk(ra, stream, timer);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return readback(cam, out, flags, stream, copy_stream, timer);
}

rt_status check_scene_device(const rt_scene_s* scene, int* dev) {
  rt_status st = current_device(dev);
  if (st != RT_OK) return st;
  if (*dev != scene->device)
    return fail(RT_ERR_INVALID_ARGUMENT, "scene was built on device %d, current device is %d", scene->device, *dev);
  return RT_OK;
}

rt_status render_one(const rt_scene_s* scene, const rt_stereo_camera* cam, const rt_stereo_output* out, char* ws,
                     size_t ws_bytes, uint32_t flags, hipStream_t stream, hipStream_t copy_stream,
                     srt::TimerImpl* timer) {
  srt::RenderPlan plan;
  const int64_t chunk = chunk_for(total_paths(cam), scene->dev.L, ws_bytes, &plan);
  if (chunk == 0) {
    size_t need = 0;
    rt_render_workspace_min(scene->dev.L, &need);
    return fail(RT_ERR_BUFFER_TOO_SMALL, "workspace of %zu bytes is below the minimum of %zu bytes", ws_bytes, need);
  }
  int dev = 0;
  rt_status st = check_scene_device(scene, &dev);
  if (st != RT_OK) return st;
  plan.grid_trace = srt::trace_grid_size(dev, current_tuning().trace_blocks_per_cu, false);
  return render_passes(scene, cam, out, ws, plan, chunk, flags, stream, copy_stream, timer);
}

size_t batch_table_bytes(int32_t n) { return (size_t(n) * sizeof(srt::DevItem) + 255) & ~size_t(255); }

struct BatchPlan {
  std::vector<srt::DevItem> table;
  std::vector<int64_t> shape;  // item count, then per item: width, height, depth, lights
  srt::DevItem* dtable = nullptr;
  srt::RenderArgs ra{};
  int64_t total = 0, chunk = 0;
};

rt_status prepare_batch(const rt_batch_item* items, int32_t n, void* workspace, size_t workspace_bytes,
                        uint32_t flags, BatchPlan* bp) {
  if (n < 1 || !items) return fail(RT_ERR_INVALID_ARGUMENT, "bad batch arguments");
  if (flags & ~kKnownFlags) return fail(RT_ERR_INVALID_ARGUMENT, "unknown render flags 0x%x", flags);
  if (!workspace || !aligned256(workspace))
    return fail(RT_ERR_INVALID_ARGUMENT, "workspace must be a 256-byte aligned device pointer");
  int dev = 0;
  rt_status st = current_device(&dev);
  if (st != RT_OK) return st;
  bp->table.assign(static_cast<size_t>(n), srt::DevItem{});
  bp->shape.assign(1, n);
  int32_t lmax = 0, dmax = 0;
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    const rt_batch_item& it = items[i];
    if (!it.scene) return fail(RT_ERR_INVALID_ARGUMENT, "item %d has no scene", i);
    if (it.scene->device != dev)
      return fail(RT_ERR_INVALID_ARGUMENT, "item %d's scene was built on device %d, current device is %d", i,
                  it.scene->device, dev);
    if ((st = validate_camera(&it.camera)) != RT_OK) return st;
    if ((st = check_output(&it.out, flags)) != RT_OK) return st;
    srt::DevItem& d = bp->table[size_t(i)];
    d.sc = it.scene->dev;
    d.cam = make_dev_camera(&it.camera);
    d.out = dev_outputs(&it.out, flags);
    d.path_offset = total;
    total += total_paths(&it.camera);
    lmax = std::max(lmax, it.scene->dev.L);
    dmax = std::max(dmax, it.camera.max_depth);
    bp->shape.insert(bp->shape.end(), {it.camera.width, it.camera.height, it.camera.max_depth, it.scene->dev.L});
  }
  if (total >= (int64_t(1) << 31)) return fail(RT_ERR_UNSUPPORTED, "a batch is limited to 2^31 paths");
  const size_t tbytes = batch_table_bytes(n);
  if (workspace_bytes <= tbytes) return fail(RT_ERR_BUFFER_TOO_SMALL, "workspace smaller than the item table");
  srt::RenderPlan plan;
  const int64_t chunk = chunk_for(total, lmax, workspace_bytes - tbytes, &plan);
  if (chunk == 0) return fail(RT_ERR_BUFFER_TOO_SMALL, "workspace of %zu bytes is too small", workspace_bytes);
  const rt_tuning tune = current_tuning();
  plan.grid_trace = srt::trace_grid_size(dev, tune.trace_blocks_per_cu, true);
  char* ws = static_cast<char*>(workspace);
  bp->dtable = reinterpret_cast<srt::DevItem*>(ws);
  srt::RenderArgs& ra = bp->ra;
  ra.items = bp->dtable;
  ra.num_items = n;
  ra.max_lights = lmax;
  ra.max_depth = dmax;
  ra.ray_counts = items[0].out.ray_counts;
  ra.flags = flags;
  ra.ws = ws + tbytes;
  ra.plan = plan;
  ra.stream_blocks = tune.stream_blocks;
  bp->total = total;
  bp->chunk = chunk;
  return RT_OK;
}

rt_status run_batch_passes(BatchPlan& bp, hipStream_t stream, srt::TimerImpl* timer) {
  for (int64_t begin = 0; begin < bp.total; begin += bp.chunk) {
    bp.ra.path_begin = begin;
    bp.ra.path_count = std::min(bp.chunk, bp.total - begin);
    hipError_t e = srt::render_chunk(bp.ra, stream, timer);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return RT_OK;
}

}  // namespace

struct rt_batch_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> shape;
  uint32_t flags = 0;
  void* workspace = nullptr;
  size_t workspace_bytes = 0;
  int64_t* ray_counts = nullptr;
};

// The fixed device scratch of rt_render_stereo_noalloc: one array per GPU the library runs on,
// held until the process ends.  In host code `scratch` names a host-side stand-in, not device
// memory; its device address on the current GPU comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[RT_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mutex;
std::vector<char*> g_scratch_ptr;  // per device ordinal; nullptr until looked up

// The device address of `scratch` on device `dev` (the current device).
rt_status scratch_on_device(int dev, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (dev < 0) return fail(RT_ERR_DEVICE, "no current device");
  if (size_t(dev) >= g_scratch_ptr.size()) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || !aligned256(p)) return fail(RT_ERR_DEVICE, "the device scratch is not 256-byte aligned");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return RT_OK;
}

}  // namespace

extern "C" {

const char* rt_last_error(void) { return g_error.c_str(); }

int32_t rt_version(void) { return 100; }

rt_status rt_scene_storage_size(const rt_scene_desc* desc, size_t* storage_bytes, size_t* scratch_bytes) {
  rt_status s = validate_desc(desc);
  if (s != RT_OK) return s;
  if (!storage_bytes || !scratch_bytes) return fail(RT_ERR_INVALID_ARGUMENT, "size outputs are NULL");
  const srt::BuildPlan p = plan_for(desc, desc->flags == RT_ACCEL_PLOC);
  *storage_bytes = p.storage_bytes;
  *scratch_bytes = p.scratch_bytes;
  if (desc->flags == RT_ACCEL_PLOC)  // room for the fallback build as well
    *scratch_bytes = std::max(*scratch_bytes, plan_for(desc, false).scratch_bytes);
  return ok();
}

rt_status rt_scene_build(const rt_scene_desc* desc, void* storage, size_t storage_bytes, void* scratch,
                         size_t scratch_bytes, void* stream, rt_scene* out) {
  rt_status s = validate_desc(desc);
  if (s != RT_OK) return s;
  if (!out) return fail(RT_ERR_INVALID_ARGUMENT, "output handle pointer is NULL");
  *out = nullptr;
  if ((desc->num_triangles > 0 && (!desc->triangles || !desc->tri_material)) ||
      (desc->num_spheres > 0 && (!desc->spheres || !desc->sphere_material)) ||
      (desc->num_planes > 0 && (!desc->planes || !desc->plane_material)) || !desc->materials ||
      (desc->num_lights > 0 && !desc->lights))
    return fail(RT_ERR_INVALID_ARGUMENT, "an array with a non-zero count is NULL");
  for (int i = 0; i < desc->num_materials; ++i) {
    const rt_material& m = desc->materials[i];
    if (!finite3(m.albedo) || !finite3(m.specular) || !finite3(m.reflectance) || !std::isfinite(m.shininess) ||
        !(m.shininess > 0.f))
      return fail(RT_ERR_INVALID_ARGUMENT, "material %d has a non-finite value or shininess <= 0", i);
  }
  for (int i = 0; i < desc->num_lights; ++i)
    if (!finite3(desc->lights[i].position) || !finite3(desc->lights[i].intensity))
      return fail(RT_ERR_INVALID_ARGUMENT, "light %d is not finite", i);
  srt::BuildPlan plan = plan_for(desc, desc->flags == RT_ACCEL_PLOC);
  if (!storage || !scratch) return fail(RT_ERR_INVALID_ARGUMENT, "storage and scratch must be device pointers");
  if (!aligned256(storage) || !aligned256(scratch))
    return fail(RT_ERR_INVALID_ARGUMENT, "storage and scratch must be 256-byte aligned");
  if (storage_bytes < plan.storage_bytes)
    return fail(RT_ERR_BUFFER_TOO_SMALL, "storage of %zu bytes, %zu required", storage_bytes, plan.storage_bytes);
  if (scratch_bytes < plan.scratch_bytes)
    return fail(RT_ERR_BUFFER_TOO_SMALL, "scratch of %zu bytes, %zu required", scratch_bytes, plan.scratch_bytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  srt::BuildResult res{};
  char* st = static_cast<char*>(storage);
  e = srt::build_scene_device(desc, plan, st, static_cast<char*>(scratch), static_cast<hipStream_t>(stream), &res);
  if (e != hipSuccess) return hip_fail(e, "scene build");
  if ((s = build_status(res)) != RT_OK) return s;
  int32_t builder = !plan.bvh ? int32_t(RT_ACCEL_NONE) : (plan.ploc ? int32_t(RT_ACCEL_PLOC) : int32_t(RT_ACCEL_KARRAS));
  if (plan.bvh && plan.ploc && !stack_fits(res.depth)) {
    // The clustering tree is too deep for the traversal stack: rebuild the same storage with the Karras
    // tree, whose depth the Morton code bounds (its scratch is smaller than the clustering build's, and
    // rt_scene_storage_size asks for the larger of the two).
    const srt::BuildPlan kplan = plan_for(desc, false);
    if (kplan.storage_bytes <= storage_bytes && kplan.scratch_bytes <= scratch_bytes) {
      e = srt::build_scene_device(desc, kplan, st, static_cast<char*>(scratch), static_cast<hipStream_t>(stream),
                                  &res);
      if (e != hipSuccess) return hip_fail(e, "scene build (fallback tree)");
      if ((s = build_status(res)) != RT_OK) return s;
      plan = kplan;
      builder = RT_ACCEL_KARRAS;
    }
  }
  if (!stack_fits(res.depth)) return fail(RT_ERR_UNSUPPORTED, "BVH depth %d exceeds the traversal stack", res.depth);

  rt_scene_s* h = new (std::nothrow) rt_scene_s();
  if (!h) return fail(RT_ERR_DEVICE, "out of host memory");
  srt::DevScene& d = h->dev;
  d.nodes = reinterpret_cast<const float4*>(st + plan.nodes_off);
  d.tris = reinterpret_cast<const float4*>(st + plan.tris_off);
  d.spheres = reinterpret_cast<const float4*>(st + plan.spheres_off);
  d.sphere_mat = reinterpret_cast<const uint32_t*>(st + plan.sphere_mat_off);
  d.planes = reinterpret_cast<const float4*>(st + plan.planes_off);
  d.plane_mat = reinterpret_cast<const uint32_t*>(st + plan.plane_mat_off);
  d.materials = reinterpret_cast<const float4*>(st + plan.mats_off);
  d.lights = reinterpret_cast<const float4*>(st + plan.lights_off);
  d.T = int32_t(desc->num_triangles);
  d.S = desc->num_spheres;
  d.P = desc->num_planes;
  d.L = desc->num_lights;
  d.M = desc->num_materials;
  d.root = res.root;
  d.num_nodes = int32_t(res.num_nodes);
  d.has_bvh = plan.bvh ? 1 : 0;
  for (int k = 0; k < 3; ++k) {
    d.ambient[k] = desc->ambient[k];
    d.background[k] = desc->background[k];
  }
  h->device = dev;
  rt_scene_info& info = h->info;
  info.num_triangles = desc->num_triangles;
  info.num_spheres = desc->num_spheres;
  info.num_planes = desc->num_planes;
  info.num_lights = desc->num_lights;
  info.num_materials = desc->num_materials;
  info.bvh_depth = plan.bvh ? res.depth : 0;
  info.builder = builder;
  info.leaf_size = desc->num_triangles > 0 ? (plan.bvh ? srt::leaf_size() : 1) : 0;
  info.num_nodes = res.num_nodes;
  info.node_bytes = res.num_nodes * srt::kNodeBytes;
  info.triangle_bytes = desc->num_triangles * 48;
  for (int k = 0; k < 3; ++k) {
    info.bounds_lo[k] = res.lo[k];
    info.bounds_hi[k] = res.hi[k];
  }
  *out = h;
  return ok();
}

rt_status rt_scene_release(rt_scene scene) {
  if (!scene) return fail(RT_ERR_INVALID_ARGUMENT, "scene is NULL");
  delete scene;
  return ok();
}

rt_status rt_scene_get_info(rt_scene scene, rt_scene_info* info) {
  if (!scene || !info) return fail(RT_ERR_INVALID_ARGUMENT, "scene or info is NULL");
  *info = scene->info;
  return ok();
}

rt_status rt_render_workspace_size(const rt_stereo_camera* camera, int32_t num_lights, size_t* bytes) {
  rt_status s = validate_camera(camera);
  if (s != RT_OK) return s;
  if (num_lights < 0 || num_lights > RT_MAX_LIGHTS || !bytes)
    return fail(RT_ERR_INVALID_ARGUMENT, "num_lights out of range or bytes is NULL");
  srt::RenderPlan plan;
  *bytes = srt::plan_render(std::min(total_paths(camera), kMaxChunk), num_lights, 0, &plan);
  return ok();
}

rt_status rt_render_workspace_min(int32_t num_lights, size_t* bytes) {
  if (num_lights < 0 || num_lights > RT_MAX_LIGHTS || !bytes)
    return fail(RT_ERR_INVALID_ARGUMENT, "num_lights out of range or bytes is NULL");
  srt::RenderPlan plan;
  *bytes = srt::plan_render(kMinChunk, num_lights, 0, &plan);
  return ok();
}

rt_status rt_render_stereo(rt_scene scene, const rt_stereo_camera* camera, const rt_stereo_output* out,
                           void* workspace, size_t workspace_bytes, uint32_t flags, void* stream, void* copy_stream,
                           rt_timer timer) {
  if (!scene) return fail(RT_ERR_INVALID_ARGUMENT, "scene is NULL");
  rt_status s = validate_camera(camera);
  if (s != RT_OK) return s;
  if ((s = check_output(out, flags)) != RT_OK) return s;
  if (flags & ~kKnownFlags) return fail(RT_ERR_INVALID_ARGUMENT, "unknown render flags 0x%x", flags);
  if (!workspace || !aligned256(workspace))
    return fail(RT_ERR_INVALID_ARGUMENT, "workspace must be a 256-byte aligned device pointer");
  s = render_one(scene, camera, out, static_cast<char*>(workspace), workspace_bytes, flags,
                 static_cast<hipStream_t>(stream), static_cast<hipStream_t>(copy_stream), timer);
  if (s != RT_OK) return s;
  if (timer && timer->error != hipSuccess) return hip_fail(timer->error, "timer event");
  return ok();
}

rt_status rt_render_stereo_noalloc(rt_scene scene, const rt_stereo_camera* camera, const rt_stereo_output* out,
                                   uint32_t flags, void* stream, void* copy_stream) {
  if (!scene) return fail(RT_ERR_INVALID_ARGUMENT, "scene is NULL");
  rt_status s = validate_camera(camera);
  if (s != RT_OK) return s;
  if ((s = check_output(out, flags)) != RT_OK) return s;
  if (flags & ~kKnownFlags) return fail(RT_ERR_INVALID_ARGUMENT, "unknown render flags 0x%x", flags);
  int dev = 0;
  if ((s = check_scene_device(scene, &dev)) != RT_OK) return s;
  char* ws = nullptr;
  if ((s = scratch_on_device(dev, &ws)) != RT_OK) return s;
  // The spill area is sized to this scene's tree and the traversal grid actually launched, so the
  // fixed scratch leaves the most room for the pass's queues.
  srt::RenderPlan plan;
  const int grid = srt::trace_grid_size(dev, current_tuning().trace_blocks_per_cu, false);
  const int64_t chunk = chunk_for(total_paths(camera), scene->dev.L, RT_NOALLOC_SCRATCH_BYTES, &plan,
                                  srt::spill_entries_for_depth(scene->info.bvh_depth), grid * srt::kTraceBlock);
  if (chunk == 0)
    return fail(RT_ERR_BUFFER_TOO_SMALL, "the smallest pass for %d lights and tree depth %d does not fit the %zu-byte "
                "device scratch", scene->dev.L, scene->info.bvh_depth, size_t(RT_NOALLOC_SCRATCH_BYTES));
  plan.grid_trace = grid;
  s = render_passes(scene, camera, out, ws, plan, chunk, flags, static_cast<hipStream_t>(stream),
                    static_cast<hipStream_t>(copy_stream), nullptr);
  if (s != RT_OK) return s;
  return ok();
}

rt_status rt_render_batch_workspace_size(const rt_batch_item* items, int32_t n, size_t* bytes) {
  if (n < 1 || !items || !bytes) return fail(RT_ERR_INVALID_ARGUMENT, "bad batch arguments");
  int64_t total = 0;
  int32_t lmax = 0;
  for (int i = 0; i < n; ++i) {
    if (!items[i].scene) return fail(RT_ERR_INVALID_ARGUMENT, "item %d has no scene", i);
    rt_status s = validate_camera(&items[i].camera);
    if (s != RT_OK) return s;
    total += total_paths(&items[i].camera);
    lmax = std::max(lmax, items[i].scene->dev.L);
  }
  srt::RenderPlan plan;
  *bytes = batch_table_bytes(n) + srt::plan_render(std::min(total, kMaxChunk), lmax, 0, &plan);
  return ok();
}

rt_status rt_render_batch(const rt_batch_item* items, int32_t n, void* workspace, size_t workspace_bytes,
                          uint32_t flags, void* stream_in, rt_timer timer) {
  BatchPlan bp;
  rt_status st = prepare_batch(items, n, workspace, workspace_bytes, flags, &bp);
  if (st != RT_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(stream_in);
  hipError_t e = srt::upload_items(bp.table.data(), n, bp.dtable, stream);
  if (e != hipSuccess) return hip_fail(e, "item table upload");
  if ((st = run_batch_passes(bp, stream, timer)) != RT_OK) return st;
  for (int i = 0; i < n; ++i)
    if ((st = readback(&items[i].camera, &items[i].out, flags, stream, nullptr, timer)) != RT_OK) return st;
  if (timer && timer->error != hipSuccess) return hip_fail(timer->error, "timer event");
  return ok();
}

rt_status rt_batch_graph_create(const rt_batch_item* items, int32_t n, void* workspace, size_t workspace_bytes,
                                uint32_t flags, void* stream_in, rt_batch_graph* out) {
  if (!out) return fail(RT_ERR_INVALID_ARGUMENT, "graph pointer is NULL");
  *out = nullptr;
  if (flags & RT_FLAG_COUNT_WORK) return fail(RT_ERR_UNSUPPORTED, "RT_FLAG_COUNT_WORK is not captured into graphs");
  BatchPlan bp;
  rt_status st = prepare_batch(items, n, workspace, workspace_bytes, flags, &bp);
  if (st != RT_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(stream_in);
  if (!stream) return fail(RT_ERR_INVALID_ARGUMENT, "graph capture needs a non-null stream");
  hipError_t e = srt::upload_items(bp.table.data(), n, bp.dtable, stream);
  if (e != hipSuccess) return hip_fail(e, "item table upload");
  e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  st = run_batch_passes(bp, stream, nullptr);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(stream, &graph);
  if (st != RT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(e, "hipGraphInstantiate");
  }
  rt_batch_graph_s* g = new (std::nothrow) rt_batch_graph_s();
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return fail(RT_ERR_DEVICE, "out of host memory");
  }
  g->graph = graph;
  g->exec = exec;
  g->shape = bp.shape;
  g->flags = flags;
  g->workspace = workspace;
  g->workspace_bytes = workspace_bytes;
  g->ray_counts = items[0].out.ray_counts;
  *out = g;
  return ok();
}

rt_status rt_batch_graph_launch(rt_batch_graph g, const rt_batch_item* items, int32_t n, void* stream_in) {
  if (!g) return fail(RT_ERR_INVALID_ARGUMENT, "graph is NULL");
  BatchPlan bp;
  rt_status st = prepare_batch(items, n, g->workspace, g->workspace_bytes, g->flags, &bp);
  if (st != RT_OK) return st;
  if (bp.shape != g->shape)
    return fail(RT_ERR_INVALID_ARGUMENT, "the batch's shape (item count, sizes, depths, lights) differs from the "
                                         "captured one");
  if (items[0].out.ray_counts != g->ray_counts)
    return fail(RT_ERR_INVALID_ARGUMENT, "items[0].out.ray_counts differs from the captured pointer");
  hipStream_t stream = static_cast<hipStream_t>(stream_in);
  hipError_t e = srt::upload_items(bp.table.data(), n, bp.dtable, stream);
  if (e != hipSuccess) return hip_fail(e, "item table upload");
  e = hipGraphLaunch(g->exec, stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  for (int i = 0; i < n; ++i)
    if ((st = readback(&items[i].camera, &items[i].out, g->flags, stream, nullptr, nullptr)) != RT_OK) return st;
  return ok();
}

rt_status rt_batch_graph_destroy(rt_batch_graph g) {
  if (!g) return fail(RT_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return ok();
}

rt_status rt_get_tuning(rt_tuning* out) {
  if (!out) return fail(RT_ERR_INVALID_ARGUMENT, "tuning pointer is NULL");
  *out = current_tuning();
  return ok();
}

rt_status rt_set_tuning(const rt_tuning* t) {
  if (!t) return fail(RT_ERR_INVALID_ARGUMENT, "tuning pointer is NULL");
  if (t->trace_blocks_per_cu < 0 || t->trace_blocks_per_cu > 32 || t->stream_blocks < 1 ||
      t->stream_blocks > (1 << 20) || t->max_pass_paths < kMinChunk)
    return fail(RT_ERR_INVALID_ARGUMENT, "tuning out of range");
  std::lock_guard<std::mutex> lock(g_tuning_mutex);
  g_tuning = *t;
  return ok();
}

rt_status rt_autotune_batch(const rt_batch_item* items, int32_t n, void* workspace, size_t workspace_bytes,
                            uint32_t flags, void* stream_in, int32_t repeats, rt_tuning* best, double* best_ms) {
  if (!best || repeats < 1) return fail(RT_ERR_INVALID_ARGUMENT, "bad autotune arguments");
  hipStream_t stream = static_cast<hipStream_t>(stream_in);
  const rt_tuning start = current_tuning();
  const int per_cu_options[] = {0, 5, 4, 3, 2};
  const int64_t pass_options[] = {int64_t(1) << 25, int64_t(1) << 23, int64_t(1) << 21};
  const int stream_options[] = {2048, 8192};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(RT_ERR_DEVICE, "events");
  double best_t = 1e300;
  rt_tuning best_cfg = start;
  rt_status st = RT_OK;
  for (int pc : per_cu_options)
    for (int64_t pp : pass_options)
      for (int sb : stream_options) {
        rt_tuning cand{pc, sb, pp};
        if ((st = rt_set_tuning(&cand)) != RT_OK) break;
        if ((st = rt_render_batch(items, n, workspace, workspace_bytes, flags, stream, nullptr)) != RT_OK) break;
        (void)hipEventRecord(e0, stream);
        for (int r = 0; r < repeats && st == RT_OK; ++r)
          st = rt_render_batch(items, n, workspace, workspace_bytes, flags, stream, nullptr);
        (void)hipEventRecord(e1, stream);
        float ms = 0.f;
        if (st != RT_OK || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          if (st == RT_OK) st = fail(RT_ERR_DEVICE, "autotune timing failed");
          break;
        }
        if (ms / repeats < best_t) {
          best_t = ms / repeats;
          best_cfg = cand;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != RT_OK) {
    rt_set_tuning(&start);
    return st;
  }
  rt_set_tuning(&best_cfg);
  *best = best_cfg;
  if (best_ms) *best_ms = best_t;
  return ok();
}

rt_status rt_compose_stereo(const float* left, const float* right, int32_t width, int32_t height, int32_t mode,
                            float exposure, uint8_t* out, void* stream) {
  if (!left || !right || !out) return fail(RT_ERR_INVALID_ARGUMENT, "compose needs left, right and out");
  if (width < 1 || height < 1 || int64_t(width) * height > RT_MAX_PIXELS)
    return fail(RT_ERR_INVALID_ARGUMENT, "image size %dx%d out of range", width, height);
  if (mode != RT_COMPOSE_ANAGLYPH_RED_CYAN && mode != RT_COMPOSE_SIDE_BY_SIDE)
    return fail(RT_ERR_INVALID_ARGUMENT, "unknown compose mode %d", mode);
  if (!std::isfinite(exposure) || !(exposure > 0.f))
    return fail(RT_ERR_INVALID_ARGUMENT, "exposure must be finite and > 0");
  if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(RT_ERR_INVALID_ARGUMENT, "out must be 4-byte aligned");
  hipError_t e = srt::compose_stereo(left, right, width, height, mode, exposure, out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "compose launch");
  return ok();
}

rt_status rt_copy_to_host(const void* device, void* host, size_t bytes, void* stream) {
  if (!device || !host || bytes % 4 != 0) return fail(RT_ERR_INVALID_ARGUMENT, "bad copy arguments");
  void* view = nullptr;
  hipError_t e;
  if (hipHostGetDevicePointer(&view, host, 0) == hipSuccess && view) {
    e = srt::copy_to_host(device, view, bytes, kReadbackBlocks, static_cast<hipStream_t>(stream));
  } else {
    (void)hipGetLastError();
    e = hipMemcpyAsync(host, device, bytes, hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream));
  }
  if (e != hipSuccess) return hip_fail(e, "copy to host");
  return ok();
}

rt_status rt_timer_create(rt_timer* out) {
  if (!out) return fail(RT_ERR_INVALID_ARGUMENT, "timer pointer is NULL");
  *out = new (std::nothrow) rt_timer_s();
  if (!*out) return fail(RT_ERR_DEVICE, "out of host memory");
  return ok();
}

rt_status rt_timer_destroy(rt_timer timer) {
  if (!timer) return fail(RT_ERR_INVALID_ARGUMENT, "timer is NULL");
  for (auto& r : timer->recs) {
    (void)hipEventSynchronize(r.end);
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.end);
  }
  for (hipEvent_t e : timer->pool) (void)hipEventDestroy(e);
  if (timer->pending_start) (void)hipEventDestroy(timer->pending_start);
  delete timer;
  return ok();
}

rt_status rt_timer_read(rt_timer timer, rt_timing* out) {
  if (!timer || !out) return fail(RT_ERR_INVALID_ARGUMENT, "timer or output is NULL");
  hipError_t err = hipSuccess;
  for (auto& r : timer->recs) {
    hipError_t e = hipEventSynchronize(r.end);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.end);
    if (e != hipSuccess && err == hipSuccess) err = e;
    if (r.stage >= 0 && r.stage < RT_NUM_STAGES) {
      out->ms[r.stage] += double(ms);
      out->launches[r.stage] += 1;
    }
    timer->pool.push_back(r.start);
    timer->pool.push_back(r.end);
  }
  timer->recs.clear();
  if (err != hipSuccess) return hip_fail(err, "timer read");
  return ok();
}

}  // extern "C"
