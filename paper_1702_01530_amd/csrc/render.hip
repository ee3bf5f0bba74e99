// Stereo Whitted ray tracing on gfx950: wavefront-persistent kernels.
//
// A pass renders a range of paths (a path = one pixel of one eye; an 8x8 tile
// of the left eye is followed by the same tile of the right eye, so both of
// the paper's parallel levels -- the two channels and the pixels inside each
// -- share one queue and one launch).  With D mirror bounces, for d = 0..D+1:
//   k_trace(d)    persistent BVH traversal of the closest-hit rays of depth d
//                 (primary rays generated in-register, FP64 rounded once to
//                 FP32) together with the shadow rays spawned at depth d-1;
//                 the two ray kinds fill one grid, so neither leaves a tail
//   k_shade(d)    Phong shading of the depth-d hits: adds the ambient (or
//                 background) term, spawns one shadow ray per light with
//                 N.L > 0 into that light's queue and a mirror ray into the
//                 next depth's queue; queues are compacted with wave ballots
//                 and one atomic per block and queue
//   k_resolve(d-1) adds the unoccluded lights' terms of depth d-1 in light order
// Queues and per-depth buffers are double-buffered by depth parity.  Every
// pixel's radiance is accumulated by one thread at a time in a fixed order,
// so results do not depend on queue order, pass size or concurrent work.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "rt_internal.h"

#ifndef SRT_STACK_LDS
#define SRT_STACK_LDS 16
#endif
#ifndef SRT_TRACE_WAVES_PER_EU
#define SRT_TRACE_WAVES_PER_EU 7
#endif

namespace srt {
namespace {

constexpr int kBlock = kTraceBlock;
constexpr int kWaves = kBlock / 64;
constexpr int kStackLds = SRT_STACK_LDS;       // traversal stack entries per lane kept in LDS (power of two)
constexpr int kStackGlobal = kStackMax - kStackLds;  // older entries spill to the workspace
constexpr int kMaxTraceBlocks = 2048;
// Shading blocks are large: queue slots are reserved with one device-scope atomic per block
// iteration and queue, and atomics on one address serialise.
#ifndef SRT_SHADE_BLOCK
#define SRT_SHADE_BLOCK 512
#endif
constexpr int kShadeBlock = SRT_SHADE_BLOCK;
constexpr int kShadeWaves = kShadeBlock / 64;
static_assert((kStackLds & (kStackLds - 1)) == 0, "LDS stack size must be a power of two");
// The builder emits the 4-wide tree level by level, so nodes 0 .. kLdsNodes-1 are its top levels,
// which every ray crosses.  A single-scene traversal block copies them into LDS once per launch and
// reads them from there, off the vector-memory path.  85 nodes are levels 0-3; a deeper copy
// loses more to waves whose lanes split between LDS and global reads than it saves.
#ifndef SRT_LDS_NODES
#define SRT_LDS_NODES 85
#endif
constexpr int kLdsNodes = kQuantNodes ? SRT_LDS_NODES : 0;

// ---------------------------------------------------------------------------------------------
// Small vector helpers
// ---------------------------------------------------------------------------------------------

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ inline float3 f3(float4 v) { return make_float3(v.x, v.y, v.z); }
__device__ inline float3 operator+(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline float3 operator-(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float3 operator*(float s, float3 a) { return make_float3(s * a.x, s * a.y, s * a.z); }
__device__ inline float3 mul(float3 a, float3 b) { return make_float3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ inline float dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline float3 cross(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline float3 normalize(float3 a) { return (1.0f / sqrtf(dot(a, a))) * a; }

// 1/d with exact zeros replaced by a tiny same-signed value, so that the slab
// products stay finite (no 0 * inf) for axis-parallel rays.
__device__ inline float safe_rcp(float x) {
  const float tiny = 1e-20f;
  if (fabsf(x) < tiny) x = copysignf(tiny, x);
  return 1.0f / x;
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline uint64_t lanemask_lt() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Next float above a non-negative x (+inf stays +inf): lets a `t < tmax` test admit t == x.
__device__ inline float next_up(float x) { return x == INFINITY ? x : __int_as_float(__float_as_int(x) + 1); }

__device__ inline uint32_t round64(uint32_t x) { return (x + 63u) & ~63u; }

// ---------------------------------------------------------------------------------------------
// Kernel arguments
// ---------------------------------------------------------------------------------------------

struct KArgs {
  DevItem one;            // single render (MULTI = false)
  const DevItem* items;   // batch table (MULTI = true)
  int32_t num_items;
  int32_t lstride;        // light slots per entry in contrib/vis (max lights over the items)
  int32_t dmax;           // max reflection depth over the items
  Counters* ctr;
  float4* ro[2];       // mirror/primary ray queue by depth parity: origin + pass-local path index bits
  float4* rd[2];       // direction + excluded primitive key bits
  float4* thr[2];      // throughput
  float2* hit;         // (t, key bits) of the closest-hit rays of the current depth
  uint2* resinfo[2];   // per entry of a depth: (pass-local path index, mask of lights with a shadow ray)
  float4* srec[2];     // shadow records [light][cap]: (origin, excluded key bits)
  uint32_t* sowner[2]; // [light][cap]: entry that owns the record
  float4* contrib[2];  // [cap][lstride]: the light's term times throughput
  uint8_t* vis[2];     // [cap][lstride]: 1 = light visible
  uint32_t* gstack;
  int32_t gstack_entries; // spill entries per lane in gstack
  int64_t path_begin, path_count;
  uint32_t cap;           // entries per queue
  int32_t brute;
  int32_t trace_threads;  // threads in the persistent traversal grid (gstack stride)
};
// Kernels take KArgs by value as their first argument, so its bytes start the kernel-argument
// segment (kernel_args reads them there).
static_assert(std::is_trivially_copyable<KArgs>::value && std::is_standard_layout<KArgs>::value,
              "KArgs must be plain data");

// The item a path belongs to: binary search over the items' first path ids.
template <bool MULTI>
__device__ inline int item_of(const KArgs& a, int64_t p) {
  if (!MULTI) return 0;
  int lo = 0, hi = a.num_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.items[mid].path_offset <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <bool MULTI>
__device__ inline const DevItem& item_ref(const KArgs& a, int k) {
  return MULTI ? a.items[k] : a.one;
}

// ---------------------------------------------------------------------------------------------
// Camera
// ---------------------------------------------------------------------------------------------

__device__ inline bool path_pixel(const DevCamera& c, int64_t p, int* eye, int* x, int* y) {
  int64_t tile = p / kPathsPerTile;
  int r = int(p % kPathsPerTile);
  *eye = r >> 6;
  int w = r & 63;
  int tx = int(tile % c.tiles_x), ty = int(tile / c.tiles_x);
  *x = tx * kTile + (w & 7);
  *y = ty * kTile + (w >> 3);
  return *x < c.W && *y < c.H;
}

// Off-axis stereo pinhole: eye at C + s r (s = -+B/2), pixel-centre ray sheared by -s/Z0.
// Computed in FP64 and rounded once to FP32.
__device__ inline void primary_ray(const DevCamera& c, int eye, int x, int y, float3* o, float3* d) {
  double s = eye == 0 ? -c.half_baseline : c.half_baseline;
  double O[3], D[3];
  double a = (double(x) + 0.5 - c.cx) / c.fpx - s * c.inv_convergence;
  double b = -(double(y) + 0.5 - c.cy) / c.fpx;
  for (int k = 0; k < 3; ++k) {
    O[k] = c.C[k] + s * c.r[k];
    D[k] = c.f[k] + a * c.r[k] + b * c.u[k];
  }
  double inv = 1.0 / sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
  *o = make_float3(float(O[0]), float(O[1]), float(O[2]));
  *d = make_float3(float(D[0] * inv), float(D[1] * inv), float(D[2] * inv));
}

// ---------------------------------------------------------------------------------------------
// Ray-primitive tests (FP32)
// ---------------------------------------------------------------------------------------------

// Moller-Trumbore; closed triangle; only det == 0 rejected.  Returns t or +inf.
__device__ inline float tri_t(const float4* __restrict__ recs, int r, float3 o, float3 d, float tmin, float tmax,
                              int* id_out) {
  const float4 a = recs[3 * r], b = recs[3 * r + 1], c = recs[3 * r + 2];
  *id_out = __float_as_int(a.w);
  const float3 e1 = f3(b), e2 = f3(c);
  const float3 T = o - f3(a);
  const float3 P = cross(d, e2);
  const float det = dot(e1, P);
  if (det == 0.0f) return INFINITY;
  const float inv = 1.0f / det;
  const float u = dot(T, P) * inv;
  if (!(u >= 0.0f && u <= 1.0f)) return INFINITY;
  const float3 Q = cross(T, e1);
  const float v = dot(d, Q) * inv;
  if (!(v >= 0.0f && u + v <= 1.0f)) return INFINITY;
  const float t = dot(e2, Q) * inv;
  return (t > tmin && t < tmax) ? t : INFINITY;
}

// Sphere with unit d: b = -oc.d, h^2 = |oc + b d|^2, disc = r^2 - h^2, roots b -+ sqrt(disc).
__device__ inline float sphere_t(float4 s, float3 o, float3 d, float tmin, float tmax) {
  const float3 oc = o - f3(s);
  const float b = -dot(oc, d);
  const float3 foot = oc + b * d;
  const float disc = s.w * s.w - dot(foot, foot);
  if (disc < 0.0f) return INFINITY;
  const float q = sqrtf(disc);
  const float t0 = b - q, t1 = b + q;
  if (t0 > tmin && t0 < tmax) return t0;
  if (t1 > tmin && t1 < tmax) return t1;
  return INFINITY;
}

__device__ inline float plane_t(float4 p, float3 o, float3 d, float tmin, float tmax) {
  const float nd = p.x * d.x + p.y * d.y + p.z * d.z;
  if (nd == 0.0f) return INFINITY;
  const float t = (p.w - (p.x * o.x + p.y * o.y + p.z * o.z)) / nd;
  return (t > tmin && t < tmax) ? t : INFINITY;
}

// Slab test of one child box; returns the entry distance, or +inf when missed.
__device__ inline float slab(float lox, float hix, float loy, float hiy, float loz, float hiz, float3 inv, float3 oi,
                             float tmin, float tmax) {
  const float x0 = fmaf(lox, inv.x, -oi.x), x1 = fmaf(hix, inv.x, -oi.x);
  const float y0 = fmaf(loy, inv.y, -oi.y), y1 = fmaf(hiy, inv.y, -oi.y);
  const float z0 = fmaf(loz, inv.z, -oi.z), z1 = fmaf(hiz, inv.z, -oi.z);
  const float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), tmin));
  const float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tmax));
  return tn <= tf ? tn : INFINITY;
}

// Entry distances of the four children of BVH4 node `node` (+inf where the ray misses the child's
// box inside [tmin, tmax]; with HITS_ONLY 0 instead of the distance of a hit child) and their references.
// Reads node `node` of the LDS array `lnodes`.  Written as LDS instructions because the compiler
// merges two plain reads of the same shape from LDS and global memory into one flat read, which
// takes the vector-memory path for every lane.
__device__ __attribute__((always_inline)) inline void lds_read_node(const float4* lnodes, int node, float4& a,
                                                                    float4& b, float4& c, float4& d) {
  typedef __attribute__((address_space(3))) const float4 lds_float4;
  const uint32_t addr = uint32_t(uintptr_t((const lds_float4*)lnodes)) + uint32_t(node) * 64u;
  asm volatile(
      "ds_read_b128 %0, %4\n\t"
      "ds_read_b128 %1, %4 offset:16\n\t"
      "ds_read_b128 %2, %4 offset:32\n\t"
      "ds_read_b128 %3, %4 offset:48\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d)
      : "v"(addr)
      : "memory");
}

// Nodes below `kc` are read from the LDS copy `lnodes` of the top of the tree.
template <bool HITS_ONLY, bool PERM_GRID>
__device__ __attribute__((always_inline)) inline void node4_children(const float4* __restrict__ nodes,
                                                                     const float4* lnodes, int kc, int node,
                                                                     float3 inv, float3 oi, float tmin, float tmax,
                                                                     float (&t)[4], int (&r)[4]) {
#if SRT_QNODE
  // Slab planes of child k on axis a are p_a + q s_a, i.e. t = q (s_a / d_a) + (p_a - o_a) / d_a; the
  // near and far planes of an axis are picked once per node from the ray's direction sign.  A byte q
  // placed in the low byte of an FP16 value is the subnormal q 2^-24, exactly; one v_perm_b32 makes
  // two such values from two grid bytes, and v_fma_mix_f32 takes one as its FP16 multiplicand.  The
  // node stores S = 2^24 s, so q 2^-24 (S / d) = q (s / d) exactly and each plane is the same fused
  // multiply-add, to the bit, as with q converted to FP32.  S / d is finite for every direction
  // because vertices lie within RT_MAX_COORD.
  float4 n0, n1, n2, n3;
  if (node < kc) {
    lds_read_node(lnodes, node, n0, n1, n2, n3);
  } else {
    const float4* n = nodes + 4 * node;
    n0 = n[0];
    n1 = n[1];
    n2 = n[2];
    n3 = n[3];
  }
  const float ax = n0.w * inv.x, ay = n3.z * inv.y, az = n3.w * inv.z;  // 2^24 s / d; S is a power of two: exact
  const float bx = fmaf(n0.x, inv.x, -oi.x), by = fmaf(n0.y, inv.y, -oi.y), bz = fmaf(n0.z, inv.z, -oi.z);
  const bool px = inv.x >= 0.f, py = inv.y >= 0.f, pz = inv.z >= 0.f;
  const uint32_t qlx = __float_as_uint(n2.x), qhx = __float_as_uint(n2.y), qly = __float_as_uint(n2.z),
                 qhy = __float_as_uint(n2.w), qlz = __float_as_uint(n3.x), qhz = __float_as_uint(n3.y);
  const uint32_t nx = px ? qlx : qhx, fx = px ? qhx : qlx, ny = py ? qly : qhy, fy = py ? qhy : qly,
                 nz = pz ? qlz : qhz, fz = pz ? qhz : qlz;
  // bytes 2j and 2j+1 of w as the FP16 pair (q 2^-24, q' 2^-24): selector byte 0x0c gives a zero byte
  auto grid_pair = [](uint32_t w, int j) {
    return __builtin_bit_cast(half2_t, __builtin_amdgcn_perm(0u, w, j ? 0x0c030c02u : 0x0c010c00u));
  };
  half2_t hnx[2], hfx[2], hny[2], hfy[2], hnz[2], hfz[2];
  if (PERM_GRID) {
    for (int j = 0; j < 2; ++j) {
      hnx[j] = grid_pair(nx, j), hfx[j] = grid_pair(fx, j), hny[j] = grid_pair(ny, j), hfy[j] = grid_pair(fy, j);
      hnz[j] = grid_pair(nz, j), hfz[j] = grid_pair(fz, j);
    }
  }
  // Without PERM_GRID the bytes are converted to FP32 and scaled by s / d = 2^-24 (S / d), exact: the same
  // planes to the bit with fewer live registers (the batch kernel also holds each lane's scene fields).
  const float sx = ax * 0x1p-24f, sy = ay * 0x1p-24f, sz = az * 0x1p-24f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    auto q = [k](const half2_t (&h)[2]) { return float((k & 1) ? h[k >> 1].y : h[k >> 1].x); };
    auto b = [k](uint32_t w) { return float((w >> (8 * k)) & 0xffu); };
    const float xn = PERM_GRID ? fmaf(q(hnx), ax, bx) : fmaf(b(nx), sx, bx);
    const float xf = PERM_GRID ? fmaf(q(hfx), ax, bx) : fmaf(b(fx), sx, bx);
    const float yn = PERM_GRID ? fmaf(q(hny), ay, by) : fmaf(b(ny), sy, by);
    const float yf = PERM_GRID ? fmaf(q(hfy), ay, by) : fmaf(b(fy), sy, by);
    const float zn = PERM_GRID ? fmaf(q(hnz), az, bz) : fmaf(b(nz), sz, bz);
    const float zf = PERM_GRID ? fmaf(q(hfz), az, bz) : fmaf(b(fz), sz, bz);
    const float tn = fmaxf(fmaxf(xn, yn), fmaxf(zn, tmin));
    const float tf = fminf(fminf(xf, yf), fminf(zf, tmax));
    // HITS_ONLY: 0 for a hit child, +inf otherwise (an occlusion query needs no entry distance)
    t[k] = tn <= tf ? (HITS_ONLY ? 0.0f : tn) : INFINITY;
  }
  r[0] = __float_as_int(n1.x);
  r[1] = __float_as_int(n1.y);
  r[2] = __float_as_int(n1.z);
  r[3] = __float_as_int(n1.w);
#else
  const float4* n = nodes + 8 * node;
  const float4 lx = n[0], hx = n[1], ly = n[2], hy = n[3], lz = n[4], hz = n[5], cr = n[6];
  t[0] = slab(lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, inv, oi, tmin, tmax);
  t[1] = slab(lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, inv, oi, tmin, tmax);
  t[2] = slab(lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, inv, oi, tmin, tmax);
  t[3] = slab(lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, inv, oi, tmin, tmax);
  if (HITS_ONLY)
    for (int k = 0; k < 4; ++k) t[k] = t[k] < INFINITY ? 0.0f : INFINITY;
  r[0] = __float_as_int(cr.x);
  r[1] = __float_as_int(cr.y);
  r[2] = __float_as_int(cr.z);
  r[3] = __float_as_int(cr.w);
#endif
}

// ---------------------------------------------------------------------------------------------
// Traversal stack: kStackLds entries per lane in LDS used as a ring; older entries spill to
// a lane-interleaved area of the workspace.
// ---------------------------------------------------------------------------------------------

struct Stack {
  uint32_t* lds;     // &lds_stack[threadIdx.x], stride kBlock
  uint32_t* global;  // &gstack[global thread], stride gstride
  int gstride;
  int gcap;          // spill entries per lane
  int sp;
  bool overflow;

  __device__ inline void push(int v) {
    if (sp >= kStackLds) {
      if (sp - kStackLds >= gcap) {  // excluded by the depth checks on the host; never write out of bounds
        overflow = true;
        return;
      }
      global[size_t(sp - kStackLds) * gstride] = lds[(sp & (kStackLds - 1)) * kBlock];
    }
    lds[(sp & (kStackLds - 1)) * kBlock] = uint32_t(v);
    ++sp;
  }
  // Pushes the np (1..3) entries c3, c2, c1 of which the last np are live (c1 ends on top).  With
  // room for three entries below the LDS ring's wrap point all three slots are written
  // unconditionally (entries above the new top are dead), so the common case takes no branch.
  __device__ inline void push_sorted(int c1, int c2, int c3, int np) {
    if (sp + 3 <= kStackLds) {
      const int s0 = np == 1 ? c1 : (np == 2 ? c2 : c3);
      const int s1 = np == 2 ? c1 : c2;
      lds[sp * kBlock] = uint32_t(s0);
      lds[(sp + 1) * kBlock] = uint32_t(s1);
      lds[(sp + 2) * kBlock] = uint32_t(c1);
      sp += np;
    } else {
      if (np >= 3) push(c3);
      if (np >= 2) push(c2);
      push(c1);
    }
  }
  __device__ inline int pop() {
    --sp;
    int v = int(lds[(sp & (kStackLds - 1)) * kBlock]);
    if (sp >= kStackLds) lds[(sp & (kStackLds - 1)) * kBlock] = global[size_t(sp - kStackLds) * gstride];
    return v;
  }
};

// Orders four (entry distance, child) pairs by distance; missed children (at +inf) sort last.
__device__ __attribute__((always_inline)) inline void sort4(float (&t)[4], int (&r)[4]) {
  auto cas = [&](int i, int j) {
    const bool sw = t[j] < t[i];
    const float ti = t[i], tj = t[j];
    const int ri = r[i], rj = r[j];
    t[i] = sw ? tj : ti;
    t[j] = sw ? ti : tj;
    r[i] = sw ? rj : ri;
    r[j] = sw ? ri : rj;
  };
  cas(0, 1);
  cas(2, 3);
  cas(0, 2);
  cas(1, 3);
  cas(1, 2);
}

// Value of the `node` register once a ray's traversal is finished (never a node index).
constexpr int kDoneRef = 0x7fffffff;

struct Best {
  float t;
  int key;
  int id;
};

// ANY = false: closest hit, minimum t, exact ties to the smaller original id; best.t starts at +inf.
// ANY = true : occlusion, stops at the first primitive with t in (tmin, best.t); best.key >= 0 if found.
// Candidates are tested against next_up(best.t) in the closest-hit case so that an exact tie in t
// reaches the (t, id) comparison, and boxes entered exactly at best.t are not culled.
template <bool ANY, bool COUNT, bool PERM_GRID>
__device__ inline void traverse(const DevScene& sc, const float4* lnodes, int kc, float3 o, float3 d, float tmin,
                                int exclude, bool brute, Best& best, Stack& st, uint32_t& nnodes, uint32_t& ntris) {
  // upper end of the interval a candidate or a box must start in: best.t for an occlusion query, the
  // next float above best.t for a closest hit; it changes only when a hit is accepted
  float limit = ANY ? best.t : next_up(best.t);
  auto accept = [&](float t, int key, int id) -> bool {  // returns true when the traversal can stop
    if (key == exclude || !(t < INFINITY)) return false;
    if (ANY) {
      best.t = t;
      best.key = key;
      best.id = id;
      return true;
    }
    if (t < best.t || (t == best.t && id < best.id)) {
      best.t = t;
      best.key = key;
      best.id = id;
      limit = __int_as_float(__float_as_int(t) + 1);  // t is finite here
    }
    return false;
  };

  for (int s = 0; s < sc.S; ++s) {
    const int key = sc.T + s;
    if (accept(sphere_t(sc.spheres[s], o, d, tmin, limit), key, key)) return;
  }
  for (int p = 0; p < sc.P; ++p) {
    const int key = sc.T + sc.S + p;
    if (accept(plane_t(sc.planes[p], o, d, tmin, limit), key, key)) return;
  }
  if (sc.T == 0) return;
  if (brute || !sc.has_bvh) {
    for (int r = 0; r < sc.T; ++r) {
      int id;
      const float t = tri_t(sc.tris, r, o, d, tmin, limit, &id);
      if (COUNT) ++ntris;
      if (accept(t, r, id)) return;
    }
    return;
  }
  const float3 inv = make_float3(safe_rcp(d.x), safe_rcp(d.y), safe_rcp(d.z));
  const float3 oi = mul(o, inv);
  // Each iteration takes one internal-node step and then, if the lane now holds a leaf, tests it,
  // so the leaf step of a wave runs with every lane that reached a leaf in this iteration.
  int node = sc.root;
  st.sp = 0;
  // A valid tree visits each node and leaf at most once; the cap only guards against a corrupt one
  // (T <= 2^29, so it fits 32 bits).
  for (int guard = 2 * sc.T + 64; guard > 0; --guard) {
    if (node >= 0) {
      if (node >= sc.num_nodes) {  // corrupt reference: stop this ray, never read out of bounds
        st.overflow = true;
        return;
      }
      if (COUNT) ++nnodes;
      const float tmax = limit;
      float t[4];
      int r[4];
      node4_children<ANY, PERM_GRID>(sc.nodes, lnodes, kc, node, inv, oi, tmin, tmax, t, r);
      if (ANY) {
        // occlusion: the order of the hit children does not change the answer, so they are taken in
        // slot order (the same for every lane of the wave) without sorting: the first hit child next,
        // the later hit children pushed so that they pop in slot order
        const bool h0 = t[0] == 0.0f, h1 = t[1] == 0.0f, h2 = t[2] == 0.0f, h3 = t[3] == 0.0f;
        if (h0 || h1 || h2 || h3) {
          node = h0 ? r[0] : (h1 ? r[1] : (h2 ? r[2] : r[3]));
          const bool g1 = h1 && h0, g2 = h2 && (h0 || h1), g3 = h3 && (h0 || h1 || h2);  // hits after the first
          const int np = int(g1) + int(g2) + int(g3);
          if (np > 0) st.push_sorted(g1 ? r[1] : (g2 ? r[2] : r[3]), (g1 && g2) ? r[2] : r[3], r[3], np);
        } else {
          node = st.sp > 0 ? st.pop() : kDoneRef;
        }
      } else {
        sort4(t, r);
        if (t[0] < INFINITY) {
          node = r[0];
          const int np = int(t[1] < INFINITY) + int(t[2] < INFINITY) + int(t[3] < INFINITY);
          if (np > 0) st.push_sorted(r[1], r[2], r[3], np);
        } else {
          node = st.sp > 0 ? st.pop() : kDoneRef;
        }
      }
    }
    if (node < 0) {
      const int code = ~node;
      const int first = code >> 2, count = (code & 3) + 1;
      if (first + count > sc.T) {
        st.overflow = true;
        return;
      }
      for (int k = 0; k < count; ++k) {
        const int r = first + k;
        if (r == exclude) continue;  // the secondary ray's own primitive: not fetched
        int id;
        const float t = tri_t(sc.tris, r, o, d, tmin, limit, &id);
        if (COUNT) ++ntris;
        if (accept(t, r, id)) return;
      }
      node = st.sp > 0 ? st.pop() : kDoneRef;
    }
    if (node == kDoneRef) return;
  }
  st.overflow = true;
}

__device__ inline void add_work(Counters* ctr, int slot, uint32_t v) {
  // wave reduction, one 64-bit atomic per wave
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane_id() == 0 && v) atomicAdd(&ctr->work[slot], (unsigned long long)v);
}

// ---------------------------------------------------------------------------------------------
// k_trace: closest-hit rays of depth `depth` and shadow rays of depth `depth - 1` in one
// persistent grid.  The work space is [closest rays | shadow rays of light 0 | light 1 | ...],
// each range padded to a multiple of 64 so that every wave batch is one kind of ray.
// ---------------------------------------------------------------------------------------------

// Traversal occupancy: the traversal kernels are held to kTraceWaves waves per SIMD, a budget of
// 72 VGPRs.  The single-scene kernel meets it without spilling; the batch kernel, whose scene fields
// are per-lane values, spills two VGPRs and is still faster (2097 vs 1846 stereo frames/s on the
// 64-pair batch).  The instrumented kernels are left free.
constexpr int kTraceWaves = SRT_TRACE_WAVES_PER_EU;
#define SRT_TRACE_ATTR __attribute__((amdgpu_waves_per_eu(COUNT || kTraceWaves <= 0 ? 1 : kTraceWaves)))

// The kernel's arguments read afresh from the kernel-argument segment: the empty asm hides that the
// pointer is loop-invariant, so fields used once per batch are loaded where they are used instead of
// being kept in scalar registers across the traversal loop, where they would spill.  A kernel's
// first argument starts the segment.
__device__ __attribute__((always_inline)) inline const KArgs& kernel_args() {
  typedef __attribute__((address_space(4))) const KArgs kargs_t;
  const kargs_t* p = (const kargs_t*)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *(const KArgs*)p;
}

template <bool COUNT, bool MULTI>
__global__ __launch_bounds__(kBlock) SRT_TRACE_ATTR void k_trace(KArgs a, int depth) {
  __shared__ uint32_t lstack[kStackLds * kBlock];
  __shared__ float4 lnodes[kLdsNodes > 0 ? 4 * kLdsNodes : 1];
  const int lane = lane_id();
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  Stack st{&lstack[threadIdx.x], a.gstack + gtid, a.trace_threads, a.gstack_entries, 0, false};
  const int LS = a.lstride;
  int kc = 0;  // nodes held in lnodes (the same for the whole block)
  if (!MULTI && kLdsNodes > 0 && a.one.sc.has_bvh && a.one.sc.T > 0 && !a.brute) {
    kc = min(kLdsNodes, a.one.sc.num_nodes);
    for (int i = threadIdx.x; i < 4 * kc; i += kBlock) lnodes[i] = a.one.sc.nodes[i];
    __syncthreads();
  }
  const bool closest = depth <= a.dmax;
  const bool shadows = depth >= 1;
  const int q = depth & 1;
  const int sq = (depth + 1) & 1;  // parity of depth - 1
  const uint32_t nc = closest ? (depth == 0 ? uint32_t(a.path_count) : a.ctr->refl_count[depth]) : 0u;
  const uint32_t nc_pad = round64(nc);
  uint32_t total = nc_pad;
  if (shadows)
    for (int l = 0; l < LS; ++l) total += round64(a.ctr->shadow_count[depth - 1][l]);
  uint32_t c_nodes = 0, c_tris = 0, s_nodes = 0, s_tris = 0;
  // Work comes in wave-wide batches of 64 items (larger grabs unbalance the launch's end, and
  // refilling single lanes stalls the wave on every refill).  Device-scope atomics on one address
  // serialise, so: wave w's first batch is batch w, with no atomic (a launch whose work fits in
  // the first round takes none); later batches b = nwaves + c + K k come from counter c = w mod K
  // of K = min(kWorkCounters, nwaves) interleaved counters, so K atomics proceed at once.
  const uint32_t nwaves = gridDim.x * uint32_t(kWaves);
  const uint32_t wid = blockIdx.x * uint32_t(kWaves) + uint32_t(threadIdx.x >> 6);
  const uint32_t nbatches = total / 64u;  // total is a multiple of 64
  const uint32_t ncounters = nwaves < uint32_t(kWorkCounters) ? nwaves : uint32_t(kWorkCounters);  // each served
  const uint32_t home = wid % ncounters;
  uint32_t batch = wid;
  for (bool first = true;; first = false) {
    if (!first) {
      if (nwaves + home >= nbatches) break;  // no batch left for this counter
      uint32_t k = 0;
      if (lane == 0) k = atomicAdd(&a.ctr->trace_work[depth][home][0], 1u);
      batch = nwaves + home + ncounters * __shfl(k, 0);
    }
    if (batch >= nbatches) break;
    const KArgs& a = kernel_args();  // the same values as the parameter, see kernel_args
    const uint32_t base = batch * 64u;
    if (base < nc_pad) {
      // ---- closest-hit batch
      const uint32_t e = base + lane;
      if (e < nc) {
        float3 o, d;
        int exclude = -1;
        bool valid = true;
        int k;
        if (depth == 0) {
          const int64_t p = a.path_begin + e;
          k = item_of<MULTI>(a, p);
          const DevItem& it = item_ref<MULTI>(a, k);
          const DevCamera& cam = it.cam;
          int eye, x, y;
          valid = path_pixel(cam, p - it.path_offset, &eye, &x, &y);
          if (valid) {
            primary_ray(cam, eye, x, y, &o, &d);
            a.ro[q][e] = make_float4(o.x, o.y, o.z, __int_as_float(int(e)));
            a.rd[q][e] = make_float4(d.x, d.y, d.z, __int_as_float(-1));
          } else {
            a.ro[q][e] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
          }
        } else {
          const float4 ro = a.ro[q][e], rd = a.rd[q][e];
          o = f3(ro);
          d = f3(rd);
          exclude = __float_as_int(rd.w);
          k = item_of<MULTI>(a, a.path_begin + uint32_t(__float_as_int(ro.w)));
        }
        if (valid) {
          const DevScene sc = item_ref<MULTI>(a, k).sc;
          Best b{INFINITY, -1, 0x7fffffff};
          traverse<false, COUNT, !MULTI>(sc, lnodes, kc, o, d, depth == 0 ? 0.0f : kSecondaryTmin, exclude,
                                         a.brute != 0, b, st, c_nodes, c_tris);
          a.hit[e] = make_float2(b.t, __int_as_float(b.key));
        }
      }
    } else {
      // ---- shadow batch: find the light whose (64-aligned) range holds this batch
      uint32_t start = nc_pad;
      int l = 0;
      uint32_t cnt = a.ctr->shadow_count[depth - 1][0];
      while (l + 1 < LS && base >= start + round64(cnt)) {
        start += round64(cnt);
        ++l;
        cnt = a.ctr->shadow_count[depth - 1][l];
      }
      const uint32_t i = base - start + lane;
      if (i < cnt) {
        const size_t slot = size_t(l) * a.cap + i;
        const float4 rec = a.srec[sq][slot];
        const uint32_t owner = a.sowner[sq][slot];
        const int k = MULTI ? item_of<MULTI>(a, a.path_begin + a.resinfo[sq][owner].x) : 0;
        const DevScene sc = item_ref<MULTI>(a, k).sc;
        const float3 P = f3(rec);
        const float3 Lv = f3(sc.lights[2 * l]) - P;
        const float dist = sqrtf(dot(Lv, Lv));
        const float3 Ld = (1.0f / dist) * Lv;
        Best b{dist, -1, 0};
        traverse<true, COUNT, !MULTI>(sc, lnodes, kc, P, Ld, kSecondaryTmin, __float_as_int(rec.w), a.brute != 0, b,
                                      st, s_nodes, s_tris);
        a.vis[sq][size_t(owner) * LS + l] = b.key < 0 ? 1 : 0;
      }
    }
  }
  if (st.overflow) atomicOr(&a.ctr->error, 1u);
  if (COUNT) {
    add_work(a.ctr, 0, c_nodes);
    add_work(a.ctr, 1, c_tris);
    add_work(a.ctr, 2, s_nodes);
    add_work(a.ctr, 3, s_tris);
  }
}

__device__ inline void material_of(const DevScene& sc, int key, float4* m0, float4* m1, float4* m2) {
  uint32_t mat;
  if (key < sc.T) {
    mat = uint32_t(__float_as_int(sc.tris[3 * key + 1].w));
  } else if (key < sc.T + sc.S) {
    mat = sc.sphere_mat[key - sc.T];
  } else {
    mat = sc.plane_mat[key - sc.T - sc.S];
  }
  *m0 = sc.materials[3 * mat];
  *m1 = sc.materials[3 * mat + 1];
  *m2 = sc.materials[3 * mat + 2];
}

__device__ inline float3 geometric_normal(const DevScene& sc, int key, float3 P) {
  if (key < sc.T) {
    const float3 e1 = f3(sc.tris[3 * key + 1]), e2 = f3(sc.tris[3 * key + 2]);
    return normalize(cross(e1, e2));
  }
  if (key < sc.T + sc.S) {
    const float4 s = sc.spheres[key - sc.T];
    return (1.0f / s.w) * (P - f3(s));
  }
  const float4 p = sc.planes[key - sc.T - sc.S];
  return normalize(make_float3(p.x, p.y, p.z));
}

__device__ inline int32_t out_id(const DevScene& sc, int key) {
  if (key < 0) return -1;
  if (key < sc.T) return __float_as_int(sc.tris[3 * key].w);
  return key;
}

// ---------------------------------------------------------------------------------------------
// k_shade: one thread per hit of depth `depth`.  Each block takes 256 consecutive entries per
// iteration; new shadow records (one queue per light) and mirror rays are compacted with wave
// ballots, a block prefix over the waves and one atomic per block and queue.
// ---------------------------------------------------------------------------------------------

template <bool PATH_IDS, bool MULTI>
__global__ __launch_bounds__(kShadeBlock) void k_shade(KArgs a, int depth) {
  __shared__ uint32_t wcnt[kShadeWaves][RT_MAX_LIGHTS + 1];
  __shared__ uint32_t bbase[RT_MAX_LIGHTS + 1];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int q = depth & 1, nq = (depth + 1) & 1;
  const uint32_t total = depth == 0 ? uint32_t(a.path_count) : a.ctr->refl_count[depth];
  const int LS = a.lstride;
  uint32_t n_primary = 0;
  for (uint32_t base = blockIdx.x * kShadeBlock; base < total; base += gridDim.x * kShadeBlock) {  // block-uniform loop
    const uint32_t e = base + threadIdx.x;
    bool active = e < total;
    float4 ro = make_float4(0.f, 0.f, 0.f, __int_as_float(-1)), rd = make_float4(0.f, 0.f, 0.f, 0.f);
    float3 thr = make_float3(1.f, 1.f, 1.f);
    float2 hit = make_float2(INFINITY, __int_as_float(-1));
    if (active) {
      ro = a.ro[q][e];
      if (__float_as_int(ro.w) < 0) {
        active = false;
        a.resinfo[q][e] = make_uint2(0xffffffffu, 0u);
      } else {
        rd = a.rd[q][e];
        hit = a.hit[e];
        if (depth > 0) thr = f3(a.thr[q][e]);
      }
    }
    uint32_t mask = 0;
    bool spawn = false;
    float3 P = make_float3(0.f, 0.f, 0.f), N = P, V = P, rdir = P, kr3 = P;
    float4 m0 = make_float4(0.f, 0.f, 0.f, 0.f), m1 = m0;
    const float4* lights = nullptr;
    const int key = __float_as_int(hit.y);
    if (active) {
      const uint32_t lp = uint32_t(__float_as_int(ro.w));
      const int64_t p = a.path_begin + lp;
      const DevItem& it = item_ref<MULTI>(a, item_of<MULTI>(a, p));
      const DevScene& sc = it.sc;
      const int L = sc.L, D1 = it.cam.D + 1;
      lights = sc.lights;
      int eye, x, y;
      path_pixel(it.cam, p - it.path_offset, &eye, &x, &y);
      const int64_t pix = int64_t(y) * it.cam.W + x;
      float* rad = it.out.radiance[eye] + 3 * pix;
      const float3 o = f3(ro), d = f3(rd);
      if (depth == 0) {
        ++n_primary;
        if (it.out.hit_t[eye]) it.out.hit_t[eye][pix] = hit.x;
        if (it.out.hit_prim[eye]) it.out.hit_prim[eye][pix] = out_id(sc, key);
        if (PATH_IDS) {
          for (int k = 0; k < D1; ++k) it.out.path_prims[eye][pix * D1 + k] = -2;
          for (int k = 0; k < D1 * L; ++k) it.out.shadow_state[eye][pix * D1 * L + k] = 0;
        }
      }
      if (PATH_IDS) it.out.path_prims[eye][pix * D1 + depth] = out_id(sc, key);
      float3 add;
      if (key < 0) {
        add = mul(thr, make_float3(sc.background[0], sc.background[1], sc.background[2]));
      } else {
        P = o + hit.x * d;
        const float3 Ng = geometric_normal(sc, key, P);
        N = dot(Ng, d) > 0.0f ? -1.0f * Ng : Ng;
        V = -1.0f * d;
        float4 m2;
        material_of(sc, key, &m0, &m1, &m2);
        add = mul(thr, mul(make_float3(sc.ambient[0], sc.ambient[1], sc.ambient[2]), f3(m0)));
        for (int l = 0; l < L; ++l) {
          const float3 Lv = f3(lights[2 * l]) - P;
          const float dist = sqrtf(dot(Lv, Lv));
          const float ndl = dot(N, (1.0f / dist) * Lv);
          if (dist > kSecondaryTmin && ndl > 0.0f) mask |= 1u << l;
        }
        kr3 = f3(m2);
        if (depth < it.cam.D && (m2.x != 0.0f || m2.y != 0.0f || m2.z != 0.0f)) {
          spawn = true;
          rdir = normalize(d - (2.0f * dot(d, N)) * N);
        }
      }
      if (depth == 0) {
        rad[0] = add.x;
        rad[1] = add.y;
        rad[2] = add.z;
      } else {
        rad[0] += add.x;
        rad[1] += add.y;
        rad[2] += add.z;
      }
      a.resinfo[q][e] = make_uint2(lp, mask);
    }
    // per-wave counts of every queue (light queues 0..LS-1, mirror queue LS), then one atomic per
    // block and queue
    for (int l = 0; l <= LS; ++l) {
      const uint64_t bal = __ballot(l < LS ? ((mask >> l) & 1u) != 0 : spawn);
      if (lane == 0) wcnt[wave][l] = uint32_t(__popcll(bal));
    }
    __syncthreads();
    if (threadIdx.x <= uint32_t(LS)) {
      const int l = threadIdx.x;
      uint32_t run = 0;
      for (int w = 0; w < kShadeWaves; ++w) {
        const uint32_t c = wcnt[w][l];
        wcnt[w][l] = run;
        run += c;
      }
      uint32_t* ctr = l < LS ? &a.ctr->shadow_count[depth][l] : &a.ctr->refl_count[depth + 1];
      bbase[l] = run ? atomicAdd(ctr, run) : 0u;
    }
    __syncthreads();
    for (int l = 0; l < LS; ++l) {
      const bool mine = ((mask >> l) & 1u) != 0;
      const uint64_t bal = __ballot(mine);
      if (mine) {
        const uint32_t slot = bbase[l] + wcnt[wave][l] + uint32_t(__popcll(bal & lanemask_lt()));
        const float3 Lv = f3(lights[2 * l]) - P;
        const float dist = sqrtf(dot(Lv, Lv));
        const float3 Ld = (1.0f / dist) * Lv;
        const float ndl = dot(N, Ld);
        const float3 R = (2.0f * ndl) * N - Ld;
        const float rv = fmaxf(0.0f, dot(R, V));
        const float spec = powf(rv, m0.w);
        const float3 I = f3(lights[2 * l + 1]);
        const float3 term = mul(I, ndl * f3(m0) + spec * f3(m1));
        const size_t s = size_t(l) * a.cap + slot;
        a.srec[q][s] = make_float4(P.x, P.y, P.z, __int_as_float(key));
        a.sowner[q][s] = e;
        a.contrib[q][size_t(e) * LS + l] = make_float4(term.x * thr.x, term.y * thr.y, term.z * thr.z, 0.f);
      }
    }
    {
      const uint64_t bal = __ballot(spawn);
      if (spawn) {
        const uint32_t slot = bbase[LS] + wcnt[wave][LS] + uint32_t(__popcll(bal & lanemask_lt()));
        a.ro[nq][slot] = make_float4(P.x, P.y, P.z, ro.w);
        a.rd[nq][slot] = make_float4(rdir.x, rdir.y, rdir.z, __int_as_float(key));
        a.thr[nq][slot] = make_float4(thr.x * kr3.x, thr.y * kr3.y, thr.z * kr3.z, 0.f);
      }
    }
    __syncthreads();  // wcnt / bbase are reused by the next iteration
  }
  if (depth == 0) {  // one atomic per block: device-scope atomics on one address serialise
    for (int off = 32; off > 0; off >>= 1) n_primary += __shfl_xor(n_primary, off);
    if (lane == 0) wcnt[wave][0] = n_primary;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t sum = 0;
      for (int w = 0; w < kShadeWaves; ++w) sum += wcnt[w][0];
      if (sum) atomicAdd(&a.ctr->primary, sum);
    }
  }
}

// k_resolve: adds the unoccluded lights' terms of depth `depth` to each path's pixel, in light order.
template <bool PATH_IDS, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_resolve(KArgs a, int depth) {
  const int q = depth & 1;
  const uint32_t total = depth == 0 ? uint32_t(a.path_count) : a.ctr->refl_count[depth];
  const int LS = a.lstride;
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < total; e += gridDim.x * kBlock) {
    const uint2 ri = a.resinfo[q][e];
    if (ri.y == 0) continue;  // no shadow rays (also invalid paths)
    const int64_t p = a.path_begin + ri.x;
    const DevItem& it = item_ref<MULTI>(a, item_of<MULTI>(a, p));
    const int L = it.sc.L, D1 = it.cam.D + 1;
    int eye, x, y;
    path_pixel(it.cam, p - it.path_offset, &eye, &x, &y);
    const int64_t pix = int64_t(y) * it.cam.W + x;
    float3 sum = make_float3(0.f, 0.f, 0.f);
    for (int l = 0; l < L; ++l) {
      if (!((ri.y >> l) & 1u)) continue;
      const size_t k = size_t(e) * LS + l;
      const bool v = a.vis[q][k] != 0;
      if (v) sum = sum + f3(a.contrib[q][k]);
      if (PATH_IDS) it.out.shadow_state[eye][(pix * D1 + depth) * L + l] = v ? 2 : 1;
    }
    float* rad = it.out.radiance[eye] + 3 * pix;
    rad[0] += sum.x;
    rad[1] += sum.y;
    rad[2] += sum.z;
  }
}

__global__ void k_reset(Counters* ctr) {
  uint32_t* p = reinterpret_cast<uint32_t*>(ctr);
  for (int i = threadIdx.x; i < int(sizeof(Counters) / 4); i += blockDim.x) p[i] = 0;
}

__global__ void k_finish(const Counters* ctr, int D, int L, int64_t* out) {
  if (threadIdx.x != 0) return;
  int64_t refl = 0, shadow = 0;
  for (int d = 1; d <= D; ++d) refl += ctr->refl_count[d];
  for (int d = 0; d <= D; ++d)
    for (int l = 0; l < L; ++l) shadow += ctr->shadow_count[d][l];
  out[RT_COUNT_PRIMARY] += ctr->primary;
  out[RT_COUNT_REFLECTION] += refl;
  out[RT_COUNT_SHADOW] += shadow;
  out[RT_COUNT_CLOSEST_NODES] += int64_t(ctr->work[0]);
  out[RT_COUNT_CLOSEST_TRIS] += int64_t(ctr->work[1]);
  out[RT_COUNT_ANY_NODES] += int64_t(ctr->work[2]);
  out[RT_COUNT_ANY_TRIS] += int64_t(ctr->work[3]);
  out[RT_COUNT_ERRORS] += ctr->error;
}

// Readback: a grid of a few workgroups streams the radiance into mapped pinned host memory, so the
// copy leaves the compute units to the next frame's traversal.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_copy_to_host16(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                           size_t n) {
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
    __builtin_nontemporal_store(src[i], &dst[i]);
}

__global__ __launch_bounds__(kBlock) void k_copy_to_host4(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                          size_t n) {
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock)
    __builtin_nontemporal_store(src[i], &dst[i]);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename K>
hipError_t launch(K kernel, unsigned grid, const KArgs& a, int depth, hipStream_t s, TimerImpl* timer, int stage,
                  int block = kBlock) {
  if (timer) timer_begin(timer, stage, s);
  kernel<<<grid, block, 0, s>>>(a, depth);
  hipError_t e = hipGetLastError();
  if (timer) timer_end(timer, stage, s);
  return e;
}

}  // namespace

hipError_t copy_to_host(const void* src, void* host_dst_device_view, size_t bytes, int blocks, hipStream_t s) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(host_dst_device_view);
  if (((a | b) & 15u) == 0 && bytes % 16 == 0) {
    k_copy_to_host16<<<blocks, kBlock, 0, s>>>(static_cast<const u32x4*>(src),
                                               static_cast<u32x4*>(host_dst_device_view), bytes / 16);
  } else {
    k_copy_to_host4<<<blocks, kBlock, 0, s>>>(static_cast<const uint32_t*>(src),
                                              static_cast<uint32_t*>(host_dst_device_view), bytes / 4);
  }
  return hipGetLastError();
}

int trace_grid_size(int device, int blocks_per_cu, bool multi) {
  // per device (the current one, which the occupancy query reads): CUs and workgroups per CU of the
  // single-scene and batch traversal kernels, looked up once; renders may come from several threads
  static std::mutex lock;
  static int cached_cus[64] = {0}, cached_occ[64][2] = {{0}};
  if (device < 0 || device >= 64) return kMaxTraceBlocks;
  std::lock_guard<std::mutex> guard(lock);
  if (!cached_cus[device]) {
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) cus = prop.multiProcessorCount;
    int occ[2] = {0, 0};
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], k_trace<false, false>, kBlock, 0) != hipSuccess ||
        occ[0] <= 0)
      occ[0] = 4;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], k_trace<false, true>, kBlock, 0) != hipSuccess ||
        occ[1] <= 0)
      occ[1] = 4;
    cached_occ[device][0] = occ[0];
    cached_occ[device][1] = occ[1];
    cached_cus[device] = cus;
  }
  int per_cu = cached_occ[device][multi ? 1 : 0];
  if (blocks_per_cu > 0) per_cu = std::min(per_cu, blocks_per_cu);
  return std::min(kMaxTraceBlocks, cached_cus[device] * per_cu);
}

int spill_entries_for_depth(int32_t bvh_depth) {
  // at most (width - 1) = 3 entries wait per level of the tree; the newest kStackLds stay in LDS
  return std::min(kStackGlobal, std::max(1, 3 * bvh_depth - kStackLds + 1));
}

size_t plan_render(int64_t chunk, int32_t L, int grid_trace, RenderPlan* p, int stack_entries, int stack_threads) {
  if (stack_entries <= 0 || stack_entries > kStackGlobal) stack_entries = kStackGlobal;
  if (stack_threads <= 0) stack_threads = kMaxTraceBlocks * kBlock;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t n = size_t(chunk);
  const size_t ns = n * size_t(std::max(L, 1));
  p->chunk_paths = chunk;
  p->grid_trace = grid_trace;
  p->counters_off = take(sizeof(Counters));
  for (int k = 0; k < 2; ++k) {
    p->ro_off[k] = take(n * 16);
    p->rd_off[k] = take(n * 16);
    p->thr_off[k] = take(n * 16);
    p->resinfo_off[k] = take(n * 8);
    p->srec_off[k] = take(ns * 16);
    p->sowner_off[k] = take(ns * 4);
    p->contrib_off[k] = take(ns * 16);
    p->vis_off[k] = take(ns);
  }
  p->hit_off = take(n * 8);
  p->stack_entries = stack_entries;
  p->stack_threads = stack_threads;
  p->gstack_off = take(size_t(stack_threads) * size_t(stack_entries) * 4);
  p->bytes = off;
  return off;
}

hipError_t render_chunk(const RenderArgs& ra, hipStream_t s, TimerImpl* timer) {
  KArgs a{};
  const bool multi = ra.items != nullptr;
  a.one = ra.one;
  a.items = ra.items;
  a.num_items = multi ? ra.num_items : 1;
  a.lstride = std::max(ra.max_lights, 1);
  a.dmax = ra.max_depth;
  char* ws = ra.ws;
  const RenderPlan& p = ra.plan;
  a.ctr = reinterpret_cast<Counters*>(ws + p.counters_off);
  for (int k = 0; k < 2; ++k) {
    a.ro[k] = reinterpret_cast<float4*>(ws + p.ro_off[k]);
    a.rd[k] = reinterpret_cast<float4*>(ws + p.rd_off[k]);
    a.thr[k] = reinterpret_cast<float4*>(ws + p.thr_off[k]);
    a.resinfo[k] = reinterpret_cast<uint2*>(ws + p.resinfo_off[k]);
    a.srec[k] = reinterpret_cast<float4*>(ws + p.srec_off[k]);
    a.sowner[k] = reinterpret_cast<uint32_t*>(ws + p.sowner_off[k]);
    a.contrib[k] = reinterpret_cast<float4*>(ws + p.contrib_off[k]);
    a.vis[k] = reinterpret_cast<uint8_t*>(ws + p.vis_off[k]);
  }
  a.hit = reinterpret_cast<float2*>(ws + p.hit_off);
  a.gstack = reinterpret_cast<uint32_t*>(ws + p.gstack_off);
  const bool ids = (ra.flags & RT_FLAG_PATH_IDS) != 0;
  const bool count = (ra.flags & RT_FLAG_COUNT_WORK) != 0;
  a.path_begin = ra.path_begin;
  a.path_count = ra.path_count;
  a.cap = uint32_t(p.chunk_paths);
  a.brute = (ra.flags & RT_FLAG_BRUTE_FORCE) ? 1 : 0;
  a.trace_threads = p.grid_trace * kBlock;
  a.gstack_entries = p.stack_entries;
  if (a.trace_threads > p.stack_threads) return hipErrorInvalidValue;  // the spill area is per grid thread

  const unsigned gtrace = unsigned(p.grid_trace);
  const unsigned gstream =
      unsigned(std::max<int64_t>(1, std::min<int64_t>((ra.path_count + kBlock - 1) / kBlock, ra.stream_blocks)));
  const unsigned gshade = unsigned(std::max<int64_t>(
      1, std::min<int64_t>((ra.path_count + kShadeBlock - 1) / kShadeBlock, ra.stream_blocks * kBlock / kShadeBlock)));
  hipError_t e;
  if (timer) timer_begin(timer, RT_STAGE_SETUP, s);
  k_reset<<<1, 256, 0, s>>>(a.ctr);
  e = hipGetLastError();
  if (timer) timer_end(timer, RT_STAGE_SETUP, s);
  if (e != hipSuccess) return e;
  const int D = a.dmax;
  for (int d = 0; d <= D + 1; ++d) {
    if (multi)
      e = count ? launch(k_trace<true, true>, gtrace, a, d, s, timer, RT_STAGE_TRACE)
                : launch(k_trace<false, true>, gtrace, a, d, s, timer, RT_STAGE_TRACE);
    else
      e = count ? launch(k_trace<true, false>, gtrace, a, d, s, timer, RT_STAGE_TRACE)
                : launch(k_trace<false, false>, gtrace, a, d, s, timer, RT_STAGE_TRACE);
    if (e != hipSuccess) return e;
    if (d <= D) {
      if (multi)
        e = ids ? launch(k_shade<true, true>, gshade, a, d, s, timer, RT_STAGE_SHADE, kShadeBlock)
                : launch(k_shade<false, true>, gshade, a, d, s, timer, RT_STAGE_SHADE, kShadeBlock);
      else
        e = ids ? launch(k_shade<true, false>, gshade, a, d, s, timer, RT_STAGE_SHADE, kShadeBlock)
                : launch(k_shade<false, false>, gshade, a, d, s, timer, RT_STAGE_SHADE, kShadeBlock);
      if (e != hipSuccess) return e;
    }
    if (d >= 1) {
      if (multi)
        e = ids ? launch(k_resolve<true, true>, gstream, a, d - 1, s, timer, RT_STAGE_RESOLVE)
                : launch(k_resolve<false, true>, gstream, a, d - 1, s, timer, RT_STAGE_RESOLVE);
      else
        e = ids ? launch(k_resolve<true, false>, gstream, a, d - 1, s, timer, RT_STAGE_RESOLVE)
                : launch(k_resolve<false, false>, gstream, a, d - 1, s, timer, RT_STAGE_RESOLVE);
      if (e != hipSuccess) return e;
    }
  }
  if (ra.ray_counts) {
    k_finish<<<1, 64, 0, s>>>(a.ctr, D, a.lstride, ra.ray_counts);
    e = hipGetLastError();
  }
  return e;
}

// The item table is written by a kernel whose arguments carry up to kItemsPerUpload items, so a
// batch needs no host staging buffer and can be captured into a graph.
namespace {
constexpr int kItemsPerUpload = 8;
struct ItemUpload {
  DevItem items[kItemsPerUpload];
  int32_t n;
};
static_assert(sizeof(ItemUpload) <= 4000, "kernel argument block too large");
__global__ void k_upload_items(ItemUpload u, DevItem* dst) {
  const int i = threadIdx.x;
  if (i < u.n) dst[i] = u.items[i];
}
}  // namespace

hipError_t upload_items(const DevItem* items, int n, DevItem* dst, hipStream_t s) {
  for (int i = 0; i < n; i += kItemsPerUpload) {
    ItemUpload u{};
    u.n = std::min(kItemsPerUpload, n - i);
    for (int k = 0; k < u.n; ++k) u.items[k] = items[i + k];
    k_upload_items<<<1, kItemsPerUpload, 0, s>>>(u, dst + i);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace srt
