// Internal declarations shared by the library's translation units (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "../../include/stereort.h"

namespace srt {

// ---------------------------------------------------------------------------------------------
// Device scene view (passed by value as a kernel argument)
// ---------------------------------------------------------------------------------------------
//
// BVH4 node, 64 bytes = 4 x float4 (quantised child boxes, the default):
//   n[0] = (p.x, p.y, p.z, S.x) with p the node's lower corner and S = 2^24 s, s the per-axis grid
//          steps, powers of two
//   n[1] = child references as int bits
//   n[2] = (lo.x, hi.x, lo.y, hi.y), n[3] = (lo.z, hi.z, S.y, S.z): 8-bit grid coordinates, child k
//          in byte k; child k's box on an axis is [p + lo_k s, p + hi_k s] (exact values), which
//          contains its padded FP32 box.  An empty slot has lo = 255 > hi = 0 on every axis and
//          repeats child 0's reference, so even a spurious entry only revisits child 0.
// BVH4 node with FP32 child boxes (SRT_QNODE=0), 128 bytes = 8 x float4, one lane per child:
//   n[0..5] = lo.x, hi.x, lo.y, hi.y, lo.z, hi.z of children 0..3
//   n[6]    = child references as int bits;  n[7] unused
//   an empty child slot has a box at +inf on every axis (never entered).
// A child reference >= 0 is an internal node index; < 0 is a leaf ~(first << 2 | (count - 1)),
// covering triangle records [first, first + count).
//
// Triangle record, 48 bytes = 3 x float4, in leaf order:
//   r[0] = (v0.xyz, original triangle id as int bits)
//   r[1] = (e1.xyz = v1 - v0, material as int bits)
//   r[2] = (e2.xyz = v2 - v0, 0)
//
// Primitive keys inside the kernels: triangle record index [0,T), sphere T+s, plane T+S+p.
// Output ids are the input order (a record carries its original id).

#ifndef SRT_QNODE
#define SRT_QNODE 1
#endif
constexpr bool kQuantNodes = SRT_QNODE != 0;
constexpr int kNodeWidth = 4;
constexpr int kNodeFloat4 = kQuantNodes ? 4 : 8;
constexpr int kNodeBytes = 16 * kNodeFloat4;
constexpr int kLeafMaxTris = 4;
constexpr int kTriFloat4 = 3;
constexpr int kMatFloat4 = 3;    // (kd, n), (ks, 0), (kr, 0)
constexpr int kLightFloat4 = 2;  // (pos, 0), (I, 0)
constexpr float kSecondaryTmin = 1e-4f;
constexpr int kStackMax = 128;   // traversal stack entries per lane (LDS ring + spill area)
constexpr int kTraceBlock = 256; // threads per traversal workgroup

struct DevScene {
  const float4* nodes;
  const float4* tris;
  const float4* spheres;
  const uint32_t* sphere_mat;
  const float4* planes;
  const uint32_t* plane_mat;
  const float4* materials;
  const float4* lights;
  int32_t T, S, P, L, M;
  int32_t root;     // node reference of the root; meaningless when T == 0
  int32_t num_nodes;
  int32_t has_bvh;  // 0: triangle records are in input order and are brute-forced
  float ambient[3], background[3];
};

// Camera constants in FP64 (primary rays are generated in FP64 and rounded once to FP32).
struct DevCamera {
  double C[3], f[3], r[3], u[3];
  double fpx, cx, cy, half_baseline, inv_convergence;
  int32_t W, H, D;
  int32_t tiles_x, tiles_y;
};

// Output pointers of one stereo render (device; optional ones may be null).
struct DevOutputs {
  float* radiance[2];
  float* hit_t[2];
  int32_t* hit_prim[2];
  int32_t* path_prims[2];
  uint8_t* shadow_state[2];
};

// One render of a batch: its scene, camera, outputs, and where its paths start in the batch's path space.
struct DevItem {
  DevScene sc;
  DevCamera cam;
  DevOutputs out;
  int64_t path_offset;
};

// Device-scope atomics on one address serialise; the traversal's work cursor is split into this
// many counters, each serving an interleaved share of the batches.
#ifndef SRT_WORK_COUNTERS
#define SRT_WORK_COUNTERS 16
#endif
constexpr int kWorkCounters = SRT_WORK_COUNTERS;

// Work counters inside the render workspace.
struct Counters {
  uint32_t refl_count[RT_MAX_DEPTH + 2];                   // entries of the mirror-ray queue at depth d
  uint32_t shadow_count[RT_MAX_DEPTH + 2][RT_MAX_LIGHTS];  // shadow records of depth d towards light l
  // work cursors of the trace launch of depth d, one per counter group, 256 bytes apart
  uint32_t trace_work[RT_MAX_DEPTH + 2][kWorkCounters][64];
  uint32_t primary;                                        // valid primary paths
  uint32_t error;                                          // consistency-check hits
  unsigned long long work[4];                              // node visits / tri tests (closest, shadow)
};

// Tile order of paths: a tile of 8x8 pixels of the left eye, then the same tile of the right eye.
constexpr int kTile = 8;
constexpr int kPathsPerTile = 2 * kTile * kTile;

struct Scene;  // host handle body

// ---------------------------------------------------------------------------------------------
// Host-side entry points of the translation units
// ---------------------------------------------------------------------------------------------

struct BuildPlan {
  int64_t T;
  size_t nodes_off, tris_off, spheres_off, sphere_mat_off, planes_off, plane_mat_off, mats_off, lights_off;
  size_t storage_bytes;
  // scratch
  size_t keys0_off, keys1_off, ids0_off, ids1_off, lo_off, hi_off, partial_off, hist_off, children_off,
      parent_off, flags_off, nodebox_off, status_off, range_off, frontier_off[2], sel_off, nint_off;
  size_t ploc_lo_off[2], ploc_hi_off[2], ploc_ref_off[2], ploc_nn_off, ploc_keep_off, ploc_merge_off;
  size_t dp_cost_off, dp_choice_off;
  size_t scan_tmp_off;
  size_t scratch_bytes;
  int64_t num_blocks_prep, num_sort_blocks;
  bool bvh;
  bool ploc;
};

// bvh: build a tree over the triangles; ploc: its binary tree by clustering (else Karras emission + refit)
BuildPlan plan_build(int64_t T, int64_t S, int64_t P, int64_t M, int64_t L, bool bvh, bool ploc);
int leaf_size();  // largest number of triangles the build puts in one leaf (1..kLeafMaxTris)

struct BuildResult {
  uint32_t status_bits;  // 1 non-finite vertex, 2 triangle material out of range, 4 sphere, 8 plane
  int32_t depth;
  int32_t max_leaf;
  int64_t num_nodes;
  float lo[3], hi[3];
  int32_t root;
};

// Enqueues the LBVH build; blocks until done and reads back BuildResult.
hipError_t build_scene_device(const rt_scene_desc* desc, const BuildPlan& plan, char* storage, char* scratch,
                              hipStream_t stream, BuildResult* result);

struct RenderPlan {
  int64_t chunk_paths;  // paths per pass (multiple of kPathsPerTile)
  size_t counters_off, ro_off[2], rd_off[2], thr_off[2], hit_off, resinfo_off[2], srec_off[2], sowner_off[2],
      contrib_off[2], vis_off[2], gstack_off;
  size_t bytes;
  int grid_trace;     // persistent workgroups for the traversal kernels
  int stack_entries;  // traversal-stack spill entries per lane
  int stack_threads;  // traversal threads the spill area covers (at least grid_trace x 256)
};

// Persistent traversal workgroups: CUs x min(occupancy limit of the single or batch kernel,
// blocks_per_cu if > 0).
int trace_grid_size(int device, int blocks_per_cu, bool multi);
// stack_entries <= 0: the most any tree the build accepts needs; stack_threads <= 0: the largest grid.
size_t plan_render(int64_t chunk_paths, int32_t num_lights, int grid_trace, RenderPlan* plan, int stack_entries = 0,
                   int stack_threads = 0);
// Spill entries per lane that a tree of this depth can need.
int spill_entries_for_depth(int32_t bvh_depth);

struct TimerImpl;
void timer_begin(TimerImpl* t, int stage, hipStream_t s);
void timer_end(TimerImpl* t, int stage, hipStream_t s);

struct RenderArgs {
  // single render: `one` (kernels keep its scene and camera in scalar registers)
  // batch: `items` (device table of num_items entries; each ray finds its item by path id)
  DevItem one;
  const DevItem* items;
  int32_t num_items;
  int32_t max_lights, max_depth;
  int64_t* ray_counts;  // device, optional
  uint32_t flags;
  char* ws;
  RenderPlan plan;
  int64_t path_begin, path_count;  // this pass's range of the (batch's) path space
  int64_t stream_blocks;           // workgroups of the shading / resolve launches
};

// Writes `n` items into the device table at `dst` (stream-ordered, no host staging).
hipError_t upload_items(const DevItem* items, int n, DevItem* dst, hipStream_t stream);

hipError_t render_chunk(const RenderArgs& a, hipStream_t stream, TimerImpl* timer);
hipError_t compose_stereo(const float* left, const float* right, int W, int H, int mode, float exposure,
                          uint8_t* out, hipStream_t s);
// Copies `bytes` (a multiple of 4) from device memory into pinned host memory through its device view.
hipError_t copy_to_host(const void* src, void* host_dst_device_view, size_t bytes, int blocks, hipStream_t s);

}  // namespace srt
