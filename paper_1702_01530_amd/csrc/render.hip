// Stereo Whitted ray tracing on gfx950: wavefront-persistent kernels.
//
// Per pass over a range of paths (a path = one pixel of one eye), for each ray
// depth d = 0..D:
//   k_closest<d==0>  persistent closest-hit traversal (primary rays generated
//                    in FP64 in-register for both eyes: the paper's parallel
//                    levels 1 and 2 share one launch and one queue)
//   k_shade          Phong shading, shadow-ray and mirror-ray spawning; wave
//                    ballots + prefix sums compact the new rays into queues
//   k_any            persistent any-hit traversal of the shadow queue
//   k_resolve        adds the unoccluded lights' terms in fixed light order
// Every pixel is owned by one queue entry per depth and its radiance is
// accumulated in a fixed order, so results are bitwise independent of queue
// order, pass size and what else shares the GPU.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "rt_internal.h"

namespace srt {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kStackLds = 32;                       // traversal stack entries per lane kept in LDS
constexpr int kStackGlobal = 96 - kStackLds;        // spill entries per lane in the workspace
constexpr int kMaxTraceBlocks = 2048;

// ---------------------------------------------------------------------------------------------
// Small vector helpers
// ---------------------------------------------------------------------------------------------

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

__device__ inline uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

// Next float above a non-negative x (+inf stays +inf): lets a `t < tmax` test admit t == x.
__device__ inline float next_up(float x) { return x == INFINITY ? x : __int_as_float(__float_as_int(x) + 1); }

// ---------------------------------------------------------------------------------------------
// Kernel arguments
// ---------------------------------------------------------------------------------------------

struct KArgs {
  DevScene sc;
  DevCamera cam;
  Counters* ctr;
  float4* ro[2];   // ray queues (ping-pong by depth parity): origin + path id bits
  float4* rd[2];   // direction + excluded primitive key bits
  float4* thr[2];  // throughput
  float2* hit;     // (t, key bits)
  uint2* resinfo;  // (first shadow record, light mask)
  float4* so;      // shadow origin + tmax
  float4* sd;      // shadow direction + excluded key bits
  float4* contrib; // light term x throughput
  uint8_t* vis;    // 1 = light visible
  uint32_t* gstack;
  float* radiance[2];
  float* hit_t[2];
  int32_t* hit_prim[2];
  int32_t* path_prims[2];
  uint8_t* shadow_state[2];
  int64_t path_begin, path_count;
  int32_t brute;
  int32_t trace_threads;  // threads in the persistent traversal grid (gstack stride)
};

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

// Slab test of one child box; returns entry distance, or +inf when missed.
__device__ inline float slab(float lox, float hix, float loy, float hiy, float loz, float hiz, float3 inv, float3 oi,
                             float tmin, float tmax) {
  const float x0 = fmaf(lox, inv.x, -oi.x), x1 = fmaf(hix, inv.x, -oi.x);
  const float y0 = fmaf(loy, inv.y, -oi.y), y1 = fmaf(hiy, inv.y, -oi.y);
  const float z0 = fmaf(loz, inv.z, -oi.z), z1 = fmaf(hiz, inv.z, -oi.z);
  const float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), tmin));
  const float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), tmax));
  return tn <= tf ? tn : INFINITY;
}

// ---------------------------------------------------------------------------------------------
// Traversal stack: kStackLds entries per lane in LDS (ring), older entries spilled to
// a lane-interleaved area of the workspace.
// ---------------------------------------------------------------------------------------------

struct Stack {
  uint32_t* lds;     // &lds_stack[0][threadIdx.x], stride kBlock
  uint32_t* global;  // &gstack[global thread], stride trace_threads
  int gstride;
  int sp;
  bool overflow;

  __device__ inline void push(int v) {
    if (sp >= kStackLds) {
      if (sp - kStackLds >= kStackGlobal) {  // cannot happen for trees of depth <= 97; never write out of bounds
        overflow = true;
        return;
      }
      global[size_t(sp - kStackLds) * gstride] = lds[(sp & (kStackLds - 1)) * kBlock];
    }
    lds[(sp & (kStackLds - 1)) * kBlock] = uint32_t(v);
    ++sp;
  }
  __device__ inline int pop() {
    --sp;
    int v = int(lds[(sp & (kStackLds - 1)) * kBlock]);
    if (sp >= kStackLds) lds[(sp & (kStackLds - 1)) * kBlock] = global[size_t(sp - kStackLds) * gstride];
    return v;
  }
};

struct Best {
  float t;
  int key;
  int id;
};

template <bool COUNT>
__device__ inline void test_leaf_closest(const DevScene& sc, int first, int count, float3 o, float3 d, float tmin,
                                         int exclude, Best& best, uint32_t& ntris) {
  for (int k = 0; k < count; ++k) {
    const int r = first + k;
    int id;
    const float t = tri_t(sc.tris, r, o, d, tmin, best.t, &id);
    if (COUNT) ++ntris;
    if (r != exclude && (t < best.t || (t == best.t && t < INFINITY && id < best.id))) {
      best.t = t;
      best.key = r;
      best.id = id;
    }
  }
}

// Closest hit: minimum t, exact ties to the smaller original id.
template <bool COUNT>
__device__ Best closest_hit(const DevScene& sc, float3 o, float3 d, float tmin, int exclude, bool brute, Stack& st,
                            uint32_t& nnodes, uint32_t& ntris) {
  Best best{INFINITY, -1, 0x7fffffff};
  // Candidates are tested against tmax = next_up(best.t) so that an exact tie in t reaches the
  // explicit (t, id) comparison; boxes entered exactly at best.t are not culled either.
  if (sc.T > 0) {
    if (brute || !sc.has_bvh) {
      for (int r = 0; r < sc.T; ++r) {
        int id;
        const float t = tri_t(sc.tris, r, o, d, tmin, next_up(best.t), &id);
        if (COUNT) ++ntris;
        if (r != exclude && (t < best.t || (t == best.t && t < INFINITY && id < best.id))) {
          best.t = t;
          best.key = r;
          best.id = id;
        }
      }
    } else {
      const float3 inv = make_float3(safe_rcp(d.x), safe_rcp(d.y), safe_rcp(d.z));
      const float3 oi = mul(o, inv);
      int node = sc.root;
      st.sp = 0;
      // A valid tree visits each node at most once; the cap only guards against a corrupt one.
      for (int64_t guard = 2 * int64_t(sc.T) + 64; guard > 0; --guard) {
        if (node >= 0) {
          if (node >= sc.num_nodes) {  // corrupt reference: stop this ray, never read out of bounds
            st.overflow = true;
            break;
          }
          const float4* n = sc.nodes + 4 * node;
          const float4 a = n[0], b = n[1], c = n[2], e = n[3];
          if (COUNT) ++nnodes;
          const float tmax = next_up(best.t);
          const float t0 = slab(a.x, a.y, a.z, a.w, c.x, c.y, inv, oi, tmin, tmax);
          const float t1 = slab(b.x, b.y, b.z, b.w, c.z, c.w, inv, oi, tmin, tmax);
          const int c0 = __float_as_int(e.x), c1 = __float_as_int(e.y);
          const bool h0 = t0 < INFINITY, h1 = t1 < INFINITY;
          if (h0 && h1) {
            const bool first0 = t0 <= t1;
            st.push(first0 ? c1 : c0);
            node = first0 ? c0 : c1;
          } else if (h0) {
            node = c0;
          } else if (h1) {
            node = c1;
          } else {
            if (st.sp == 0) break;
            node = st.pop();
          }
        } else {
          const int code = ~node;
          const int first = code >> 2, count = (code & 3) + 1;
          if (first + count > sc.T) {
            st.overflow = true;
            break;
          }
          for (int k = 0; k < count; ++k) {
            const int r = first + k;
            int id;
            const float t = tri_t(sc.tris, r, o, d, tmin, next_up(best.t), &id);
            if (COUNT) ++ntris;
            if (r != exclude && (t < best.t || (t == best.t && t < INFINITY && id < best.id))) {
              best.t = t;
              best.key = r;
              best.id = id;
            }
          }
          if (st.sp == 0) break;
          node = st.pop();
        }
      }
    }
  }
  for (int s = 0; s < sc.S; ++s) {
    const int key = sc.T + s;
    const float t = sphere_t(sc.spheres[s], o, d, tmin, next_up(best.t));
    if (key != exclude && (t < best.t || (t == best.t && t < INFINITY && key < best.id))) {
      best.t = t;
      best.key = key;
      best.id = key;
    }
  }
  for (int p = 0; p < sc.P; ++p) {
    const int key = sc.T + sc.S + p;
    const float t = plane_t(sc.planes[p], o, d, tmin, next_up(best.t));
    if (key != exclude && (t < best.t || (t == best.t && t < INFINITY && key < best.id))) {
      best.t = t;
      best.key = key;
      best.id = key;
    }
  }
  return best;
}

// Occlusion: any primitive other than `exclude` with t in (tmin, tmax).
template <bool COUNT>
__device__ bool any_hit(const DevScene& sc, float3 o, float3 d, float tmin, float tmax, int exclude, bool brute,
                        Stack& st, uint32_t& nnodes, uint32_t& ntris) {
  for (int s = 0; s < sc.S; ++s)
    if (sc.T + s != exclude && sphere_t(sc.spheres[s], o, d, tmin, tmax) < INFINITY) return true;
  for (int p = 0; p < sc.P; ++p)
    if (sc.T + sc.S + p != exclude && plane_t(sc.planes[p], o, d, tmin, tmax) < INFINITY) return true;
  if (sc.T == 0) return false;
  if (brute || !sc.has_bvh) {
    for (int r = 0; r < sc.T; ++r) {
      int id;
      if (COUNT) ++ntris;
      if (r != exclude && tri_t(sc.tris, r, o, d, tmin, tmax, &id) < INFINITY) return true;
    }
    return false;
  }
  const float3 inv = make_float3(safe_rcp(d.x), safe_rcp(d.y), safe_rcp(d.z));
  const float3 oi = mul(o, inv);
  int node = sc.root;
  st.sp = 0;
  for (int64_t guard = 2 * int64_t(sc.T) + 64; guard > 0; --guard) {
    if (node >= 0) {
      if (node >= sc.num_nodes) {
        st.overflow = true;
        return false;
      }
      const float4* n = sc.nodes + 4 * node;
      const float4 a = n[0], b = n[1], c = n[2], e = n[3];
      if (COUNT) ++nnodes;
      const float t0 = slab(a.x, a.y, a.z, a.w, c.x, c.y, inv, oi, tmin, tmax);
      const float t1 = slab(b.x, b.y, b.z, b.w, c.z, c.w, inv, oi, tmin, tmax);
      const int c0 = __float_as_int(e.x), c1 = __float_as_int(e.y);
      const bool h0 = t0 < INFINITY, h1 = t1 < INFINITY;
      if (h0 && h1) {
        const bool first0 = t0 <= t1;
        st.push(first0 ? c1 : c0);
        node = first0 ? c0 : c1;
      } else if (h0) {
        node = c0;
      } else if (h1) {
        node = c1;
      } else {
        if (st.sp == 0) return false;
        node = st.pop();
      }
    } else {
      const int code = ~node;
      const int first = code >> 2, count = (code & 3) + 1;
      if (first + count > sc.T) {
        st.overflow = true;
        return false;
      }
      for (int k = 0; k < count; ++k) {
        const int r = first + k;
        int id;
        if (COUNT) ++ntris;
        if (r != exclude && tri_t(sc.tris, r, o, d, tmin, tmax, &id) < INFINITY) return true;
      }
      if (st.sp == 0) return false;
      node = st.pop();
    }
  }
  st.overflow = true;
  return false;
}

__device__ inline void add_work(Counters* ctr, int slot, uint32_t v) {
  // wave reduction, one 64-bit atomic per wave
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane_id() == 0 && v) atomicAdd(&ctr->work[slot], (unsigned long long)v);
}

// ---------------------------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------------------------

template <bool PRIMARY, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_closest(KArgs a, int depth) {
  __shared__ uint32_t lstack[kStackLds * kBlock];
  const int lane = lane_id();
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  Stack st{&lstack[threadIdx.x], a.gstack + gtid, a.trace_threads, 0, false};
  const int q = depth & 1;
  const uint32_t total = PRIMARY ? uint32_t(a.path_count) : a.ctr->refl_count[depth];
  const float tmin = PRIMARY ? 0.0f : kSecondaryTmin;
  uint32_t nnodes = 0, ntris = 0;
  while (true) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->closest_work[depth], 64u);
    base = __shfl(base, 0);
    if (base >= total) break;
    const uint32_t e = base + lane;
    if (e < total) {
      float3 o, d;
      int exclude = -1;
      bool valid = true;
      if (PRIMARY) {
        int eye, x, y;
        const int64_t p = a.path_begin + e;
        valid = path_pixel(a.cam, p, &eye, &x, &y);
        if (valid) {
          primary_ray(a.cam, eye, x, y, &o, &d);
          a.ro[q][e] = make_float4(o.x, o.y, o.z, __int_as_float(int(p)));
          a.rd[q][e] = make_float4(d.x, d.y, d.z, __int_as_float(-1));
        } else {
          a.ro[q][e] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
        }
      } else {
        const float4 ro = a.ro[q][e], rd = a.rd[q][e];
        o = f3(ro);
        d = f3(rd);
        exclude = __float_as_int(rd.w);
      }
      if (valid) {
        Best b = closest_hit<COUNT>(a.sc, o, d, tmin, exclude, a.brute != 0, st, nnodes, ntris);
        a.hit[e] = make_float2(b.t, __int_as_float(b.key));
      }
    }
  }
  if (st.overflow) atomicOr(&a.ctr->pad[1], 1u);
  if (COUNT) {
    add_work(a.ctr, 0, nnodes);
    add_work(a.ctr, 1, ntris);
  }
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) void k_any(KArgs a, int depth) {
  __shared__ uint32_t lstack[kStackLds * kBlock];
  const int lane = lane_id();
  const int gtid = blockIdx.x * kBlock + threadIdx.x;
  Stack st{&lstack[threadIdx.x], a.gstack + gtid, a.trace_threads, 0, false};
  const uint32_t total = a.ctr->shadow_count[depth];
  uint32_t nnodes = 0, ntris = 0;
  while (true) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->any_work[depth], 64u);
    base = __shfl(base, 0);
    if (base >= total) break;
    const uint32_t e = base + lane;
    if (e < total) {
      const float4 so = a.so[e], sd = a.sd[e];
      const bool occ = any_hit<COUNT>(a.sc, f3(so), f3(sd), kSecondaryTmin, so.w, __float_as_int(sd.w),
                                      a.brute != 0, st, nnodes, ntris);
      a.vis[e] = occ ? 0 : 1;
    }
  }
  if (st.overflow) atomicOr(&a.ctr->pad[1], 1u);
  if (COUNT) {
    add_work(a.ctr, 2, nnodes);
    add_work(a.ctr, 3, ntris);
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

// Exclusive prefix sum over the wave; *total gets the wave sum.
__device__ inline uint32_t wave_exclusive_scan(uint32_t v, uint32_t* total) {
  const int lane = lane_id();
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  *total = __shfl(x, 63);
  return x - v;
}

template <bool PATH_IDS>
__global__ __launch_bounds__(kBlock) void k_shade(KArgs a, int depth) {
  const int lane = lane_id();
  const int q = depth & 1, nq = (depth + 1) & 1;
  const uint32_t total = depth == 0 ? uint32_t(a.path_count) : a.ctr->refl_count[depth];
  const int L = a.sc.L;
  const bool may_reflect = depth < a.cam.D;
  const int64_t HW = int64_t(a.cam.W) * a.cam.H;
  const int D1 = a.cam.D + 1;
  uint32_t n_primary = 0;
  for (uint32_t base = (blockIdx.x * kBlock + (threadIdx.x & ~63u)); base < total; base += gridDim.x * kBlock) {
    const uint32_t e = base + lane;
    bool active = e < total;
    float4 ro = make_float4(0.f, 0.f, 0.f, __int_as_float(-1)), rd = make_float4(0.f, 0.f, 0.f, 0.f);
    float3 thr = make_float3(1.f, 1.f, 1.f);
    float2 hit = make_float2(INFINITY, __int_as_float(-1));
    if (active) {
      ro = a.ro[q][e];
      if (__float_as_int(ro.w) < 0) {
        active = false;
      } else {
        rd = a.rd[q][e];
        hit = a.hit[e];
        if (depth > 0) thr = f3(a.thr[q][e]);
      }
    }
    int eye = 0, x = 0, y = 0;
    int64_t pix = 0;
    float* rad = nullptr;
    uint32_t mask = 0;
    bool spawn = false;
    float3 P = make_float3(0.f, 0.f, 0.f), N = P, V = P, rdir = P, kr3 = P;
    float4 m0 = make_float4(0.f, 0.f, 0.f, 0.f), m1 = m0;
    int key = -1;
    if (active) {
      path_pixel(a.cam, int64_t(__float_as_int(ro.w)), &eye, &x, &y);
      pix = int64_t(y) * a.cam.W + x;
      rad = a.radiance[eye] + 3 * pix;
      key = __float_as_int(hit.y);
      const float3 o = f3(ro), d = f3(rd);
      if (depth == 0) {
        ++n_primary;
        if (a.hit_t[eye]) a.hit_t[eye][pix] = hit.x;
        if (a.hit_prim[eye]) a.hit_prim[eye][pix] = out_id(a.sc, key);
        if (PATH_IDS) {
          for (int k = 0; k < D1; ++k) a.path_prims[eye][pix * D1 + k] = -2;
          for (int k = 0; k < D1 * L; ++k) a.shadow_state[eye][pix * D1 * L + k] = 0;
        }
      }
      if (PATH_IDS) a.path_prims[eye][pix * D1 + depth] = out_id(a.sc, key);
      float3 add;
      if (key < 0) {
        add = mul(thr, make_float3(a.sc.background[0], a.sc.background[1], a.sc.background[2]));
      } else {
        P = o + hit.x * d;
        const float3 Ng = geometric_normal(a.sc, key, P);
        N = dot(Ng, d) > 0.0f ? -1.0f * Ng : Ng;
        V = -1.0f * d;
        float4 m2;
        material_of(a.sc, key, &m0, &m1, &m2);
        add = mul(thr, mul(make_float3(a.sc.ambient[0], a.sc.ambient[1], a.sc.ambient[2]), f3(m0)));
        for (int l = 0; l < L; ++l) {
          const float3 Lv = f3(a.sc.lights[2 * l]) - P;
          const float dist = sqrtf(dot(Lv, Lv));
          const float ndl = dot(N, (1.0f / dist) * Lv);
          if (dist > kSecondaryTmin && ndl > 0.0f) mask |= 1u << l;
        }
        kr3 = f3(m2);
        if (may_reflect && (m2.x != 0.0f || m2.y != 0.0f || m2.z != 0.0f)) {
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
    }
    // compact shadow records
    uint32_t nsh = __popc(mask), wave_total;
    const uint32_t excl = wave_exclusive_scan(nsh, &wave_total);
    uint32_t sbase = 0;
    if (lane == 0 && wave_total) sbase = atomicAdd(&a.ctr->shadow_count[depth], wave_total);
    sbase = __shfl(sbase, 0) + excl;
    if (active) {
      a.resinfo[e] = make_uint2(sbase, mask);
      uint32_t k = sbase;
      for (int l = 0; l < L; ++l) {
        if (!(mask >> l & 1u)) continue;
        const float3 Lv = f3(a.sc.lights[2 * l]) - P;
        const float dist = sqrtf(dot(Lv, Lv));
        const float3 Ld = (1.0f / dist) * Lv;
        const float ndl = dot(N, Ld);
        const float3 R = (2.0f * ndl) * N - Ld;
        const float rv = fmaxf(0.0f, dot(R, V));
        const float spec = powf(rv, m0.w);
        const float3 I = f3(a.sc.lights[2 * l + 1]);
        const float3 term = mul(I, ndl * f3(m0) + spec * f3(m1));
        a.so[k] = make_float4(P.x, P.y, P.z, dist);
        a.sd[k] = make_float4(Ld.x, Ld.y, Ld.z, __int_as_float(key));
        a.contrib[k] = make_float4(term.x * thr.x, term.y * thr.y, term.z * thr.z, 0.f);
        ++k;
      }
    }
    // compact mirror rays into the next queue
    const uint64_t bal = __ballot(spawn);
    if (may_reflect && bal) {
      uint32_t rbase = 0;
      if (lane == 0) rbase = atomicAdd(&a.ctr->refl_count[depth + 1], uint32_t(__popcll(bal)));
      rbase = __shfl(rbase, 0);
      if (spawn) {
        const uint32_t slot = rbase + uint32_t(__popcll(bal & lanemask_lt()));
        a.ro[nq][slot] = make_float4(P.x, P.y, P.z, ro.w);
        a.rd[nq][slot] = make_float4(rdir.x, rdir.y, rdir.z, __int_as_float(key));
        a.thr[nq][slot] = make_float4(thr.x * kr3.x, thr.y * kr3.y, thr.z * kr3.z, 0.f);
      }
    }
  }
  if (depth == 0) {
    for (int off = 32; off > 0; off >>= 1) n_primary += __shfl_xor(n_primary, off);
    if (lane == 0 && n_primary) atomicAdd(&a.ctr->pad[0], n_primary);
  }
}

template <bool PATH_IDS>
__global__ __launch_bounds__(kBlock) void k_resolve(KArgs a, int depth) {
  const int q = depth & 1;
  const uint32_t total = depth == 0 ? uint32_t(a.path_count) : a.ctr->refl_count[depth];
  const int L = a.sc.L;
  const int D1 = a.cam.D + 1;
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < total; e += gridDim.x * kBlock) {
    const int path = __float_as_int(a.ro[q][e].w);
    if (path < 0) continue;
    const uint2 ri = a.resinfo[e];
    if (ri.y == 0 && !PATH_IDS) continue;
    int eye, x, y;
    path_pixel(a.cam, path, &eye, &x, &y);
    const int64_t pix = int64_t(y) * a.cam.W + x;
    float3 sum = make_float3(0.f, 0.f, 0.f);
    uint32_t k = ri.x;
    for (int l = 0; l < L; ++l) {
      uint8_t state = 0;
      if (ri.y >> l & 1u) {
        const bool v = a.vis[k] != 0;
        if (v) sum = sum + f3(a.contrib[k]);
        state = v ? 2 : 1;
        ++k;
      }
      if (PATH_IDS) a.shadow_state[eye][(pix * D1 + depth) * L + l] = state;
    }
    if (ri.y) {
      float* rad = a.radiance[eye] + 3 * pix;
      rad[0] += sum.x;
      rad[1] += sum.y;
      rad[2] += sum.z;
    }
  }
}

__global__ void k_reset(Counters* ctr) {
  uint32_t* p = reinterpret_cast<uint32_t*>(ctr);
  for (int i = threadIdx.x; i < int(sizeof(Counters) / 4); i += blockDim.x) p[i] = 0;
}

__global__ void k_finish(const Counters* ctr, int D, int64_t* out) {
  if (threadIdx.x != 0) return;
  int64_t refl = 0, shadow = 0;
  for (int d = 1; d <= D; ++d) refl += ctr->refl_count[d];
  for (int d = 0; d <= D; ++d) shadow += ctr->shadow_count[d];
  out[RT_COUNT_PRIMARY] += ctr->pad[0];
  out[RT_COUNT_REFLECTION] += refl;
  out[RT_COUNT_SHADOW] += shadow;
  out[RT_COUNT_CLOSEST_NODES] += int64_t(ctr->work[0]);
  out[RT_COUNT_CLOSEST_TRIS] += int64_t(ctr->work[1]);
  out[RT_COUNT_ANY_NODES] += int64_t(ctr->work[2]);
  out[RT_COUNT_ANY_TRIS] += int64_t(ctr->work[3]);
  out[RT_COUNT_ERRORS] += ctr->pad[1];
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename K>
hipError_t launch(K kernel, unsigned grid, const KArgs& a, int depth, hipStream_t s, TimerImpl* timer, int stage) {
  if (timer) timer_begin(timer, stage, s);
  kernel<<<grid, kBlock, 0, s>>>(a, depth);
  hipError_t e = hipGetLastError();
  if (timer) timer_end(timer, stage, s);
  return e;
}

}  // namespace

int trace_grid_size(int device) {
  static int cached[64] = {0};
  if (device < 0 || device >= 64) return kMaxTraceBlocks;
  if (cached[device]) return cached[device];
  hipDeviceProp_t prop;
  int grid = kMaxTraceBlocks;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_closest<false, false>, kBlock, 0) != hipSuccess ||
        per_cu <= 0)
      per_cu = 4;
    grid = std::min(kMaxTraceBlocks, prop.multiProcessorCount * per_cu);
  }
  cached[device] = grid;
  return grid;
}

size_t plan_render(int64_t chunk, int32_t L, int grid_trace, RenderPlan* p) {
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
  p->counters_off = take(sizeof(Counters) + 64);
  for (int k = 0; k < 2; ++k) {
    p->ro_off[k] = take(n * 16);
    p->rd_off[k] = take(n * 16);
    p->thr_off[k] = take(n * 16);
  }
  p->hit_off = take(n * 8);
  p->resinfo_off = take(n * 8);
  p->so_off = take(ns * 16);
  p->sd_off = take(ns * 16);
  p->contrib_off = take(ns * 16);
  p->vis_off = take(ns);
  p->gstack_off = take(size_t(kMaxTraceBlocks) * kBlock * kStackGlobal * 4);
  p->bytes = off;
  return off;
}

hipError_t render_chunk(const RenderArgs& ra, hipStream_t s, TimerImpl* timer) {
  KArgs a{};
  a.sc = ra.scene;
  a.cam = ra.cam;
  char* ws = ra.ws;
  const RenderPlan& p = ra.plan;
  a.ctr = reinterpret_cast<Counters*>(ws + p.counters_off);
  for (int k = 0; k < 2; ++k) {
    a.ro[k] = reinterpret_cast<float4*>(ws + p.ro_off[k]);
    a.rd[k] = reinterpret_cast<float4*>(ws + p.rd_off[k]);
    a.thr[k] = reinterpret_cast<float4*>(ws + p.thr_off[k]);
  }
  a.hit = reinterpret_cast<float2*>(ws + p.hit_off);
  a.resinfo = reinterpret_cast<uint2*>(ws + p.resinfo_off);
  a.so = reinterpret_cast<float4*>(ws + p.so_off);
  a.sd = reinterpret_cast<float4*>(ws + p.sd_off);
  a.contrib = reinterpret_cast<float4*>(ws + p.contrib_off);
  a.vis = reinterpret_cast<uint8_t*>(ws + p.vis_off);
  a.gstack = reinterpret_cast<uint32_t*>(ws + p.gstack_off);
  const rt_stereo_output* o = ra.out;
  const bool ids = (ra.flags & RT_FLAG_PATH_IDS) && o->path_prims[0] && o->path_prims[1] && o->shadow_state[0] &&
                   o->shadow_state[1];
  const bool count = (ra.flags & RT_FLAG_COUNT_WORK) != 0;
  for (int e = 0; e < 2; ++e) {
    a.radiance[e] = o->radiance[e];
    a.hit_t[e] = o->hit_t[e];
    a.hit_prim[e] = o->hit_prim[e];
    a.path_prims[e] = ids ? o->path_prims[e] : nullptr;
    a.shadow_state[e] = ids ? o->shadow_state[e] : nullptr;
  }
  a.path_begin = ra.path_begin;
  a.path_count = ra.path_count;
  a.brute = (ra.flags & RT_FLAG_BRUTE_FORCE) ? 1 : 0;
  a.trace_threads = p.grid_trace * kBlock;

  const unsigned gtrace = unsigned(p.grid_trace);
  const unsigned gstream = unsigned(std::min<int64_t>((ra.path_count + kBlock - 1) / kBlock, 256 * 8));
  hipError_t e;
  if (timer) timer_begin(timer, RT_STAGE_SETUP, s);
  k_reset<<<1, 256, 0, s>>>(a.ctr);
  e = hipGetLastError();
  if (timer) timer_end(timer, RT_STAGE_SETUP, s);
  if (e != hipSuccess) return e;
  for (int d = 0; d <= a.cam.D; ++d) {
    if (d == 0)
      e = count ? launch(k_closest<true, true>, gtrace, a, d, s, timer, RT_STAGE_TRACE_CLOSEST)
                : launch(k_closest<true, false>, gtrace, a, d, s, timer, RT_STAGE_TRACE_CLOSEST);
    else
      e = count ? launch(k_closest<false, true>, gtrace, a, d, s, timer, RT_STAGE_TRACE_CLOSEST)
                : launch(k_closest<false, false>, gtrace, a, d, s, timer, RT_STAGE_TRACE_CLOSEST);
    if (e != hipSuccess) return e;
    e = ids ? launch(k_shade<true>, gstream, a, d, s, timer, RT_STAGE_SHADE)
            : launch(k_shade<false>, gstream, a, d, s, timer, RT_STAGE_SHADE);
    if (e != hipSuccess) return e;
    e = count ? launch(k_any<true>, gtrace, a, d, s, timer, RT_STAGE_TRACE_ANY)
              : launch(k_any<false>, gtrace, a, d, s, timer, RT_STAGE_TRACE_ANY);
    if (e != hipSuccess) return e;
    e = ids ? launch(k_resolve<true>, gstream, a, d, s, timer, RT_STAGE_RESOLVE)
            : launch(k_resolve<false>, gstream, a, d, s, timer, RT_STAGE_RESOLVE);
    if (e != hipSuccess) return e;
  }
  if (o->ray_counts) {
    k_finish<<<1, 64, 0, s>>>(a.ctr, a.cam.D, o->ray_counts);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace srt
