// Linear BVH build on the device (gfx950).
//
// The paper (Section 3, Table 1) lists BVH trees as fast to construct, simple to
// traverse and well suited to GPUs.  The tree here is built from the Morton order:
//   1. per triangle: bounding box and centroid, input validation;
//   2. reduction of the centroid and scene bounds;
//   3. 63-bit Morton code of the centroid quantised to 2^21 cells per axis;
//   4. stable LSD radix sort of (code, triangle id), 8 passes of 8 bits;
//   5. binary tree over the sorted leaves: by default locally-ordered clustering
//      (PLOC: neighbours in the Morton order merge by smallest surface area, so
//      node boxes come with the merges); with RT_ACCEL_KARRAS, Karras (2012)
//      emission (split at the highest differing bit; equal codes split by index) and
//   6. a bottom-up box refit (an atomic arrival counter per node, the second
//      child to arrive unions both boxes and climbs on);
//   7. a bottom-up surface-area cost table that picks the cheapest way to cut the
//      binary tree into a 4-wide one (filled during the refit, or one launch per
//      clustering round);
//   8. top-down collapse into that 4-wide tree, one level per launch, with the
//      children's boxes quantised to 8 bits on each node's own grid (64-byte
//      nodes), and 48-byte triangle records in leaf order.
// Every step is deterministic, so a scene always builds the same tree.

#include <hip/hip_runtime.h>


#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

#include "rt_internal.h"
#define SRT_HD __host__ __device__
#include "ploc_rule.h"


namespace srt {

int leaf_size() { return 1; }  // every leaf of the collapsed tree is one triangle

namespace {

constexpr int kBlock = 256;
constexpr int kSortItems = 16;                      // keys per thread per sort tile
constexpr int kSortTile = kBlock * kSortItems;      // 4096 keys per block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__device__ inline bool finite3(float a, float b, float c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// ---------------------------------------------------------------------------------------------
// 1-2. Triangle boxes, validation, bounds
// ---------------------------------------------------------------------------------------------

struct Bounds6 {
  float clo[3], chi[3];  // centroid bounds
  float blo[3], bhi[3];  // scene box
};

__global__ __launch_bounds__(kBlock) void k_tri_prep(const float* __restrict__ tris,
                                                     const uint32_t* __restrict__ mat, int64_t T, int32_t M,
                                                     float4* __restrict__ lo_out, float4* __restrict__ hi_out,
                                                     Bounds6* __restrict__ partial, uint32_t* __restrict__ status) {
  __shared__ float red[12][kBlock];
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  float c[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (i < T) {
    const float* p = tris + 9 * i;
    float v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = p[k];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 9; ++k) ok = ok && fabsf(v[k]) <= RT_MAX_COORD;  // false for NaN and inf too
    if (!ok) atomicOr(status, 1u);
    if (mat[i] >= uint32_t(M)) atomicOr(status, 2u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(v[a], fminf(v[3 + a], v[6 + a]));
      hi[a] = fmaxf(v[a], fmaxf(v[3 + a], v[6 + a]));
      c[a] = 0.5f * lo[a] + 0.5f * hi[a];
      cmax[a] = c[a];
    }
    lo_out[i] = make_float4(lo[0], lo[1], lo[2], 0.f);
    hi_out[i] = make_float4(hi[0], hi[1], hi[2], 0.f);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = c[a];
    red[3 + a][threadIdx.x] = cmax[a];
    red[6 + a][threadIdx.x] = lo[a];
    red[9 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
        red[6 + a][threadIdx.x] = fminf(red[6 + a][threadIdx.x], red[6 + a][threadIdx.x + s]);
        red[9 + a][threadIdx.x] = fmaxf(red[9 + a][threadIdx.x], red[9 + a][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Bounds6 b;
    for (int a = 0; a < 3; ++a) {
      b.clo[a] = red[a][0];
      b.chi[a] = red[3 + a][0];
      b.blo[a] = red[6 + a][0];
      b.bhi[a] = red[9 + a][0];
    }
    partial[blockIdx.x] = b;
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce_bounds(Bounds6* __restrict__ partial, int64_t n) {
  __shared__ float red[12][kBlock];
  float v[12];
  for (int a = 0; a < 3; ++a) {
    v[a] = INFINITY;
    v[3 + a] = -INFINITY;
    v[6 + a] = INFINITY;
    v[9 + a] = -INFINITY;
  }
  for (int64_t i = threadIdx.x; i < n; i += kBlock) {
    Bounds6 b = partial[i];
    for (int a = 0; a < 3; ++a) {
      v[a] = fminf(v[a], b.clo[a]);
      v[3 + a] = fmaxf(v[3 + a], b.chi[a]);
      v[6 + a] = fminf(v[6 + a], b.blo[a]);
      v[9 + a] = fmaxf(v[9 + a], b.bhi[a]);
    }
  }
  for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
        red[6 + a][threadIdx.x] = fminf(red[6 + a][threadIdx.x], red[6 + a][threadIdx.x + s]);
        red[9 + a][threadIdx.x] = fmaxf(red[9 + a][threadIdx.x], red[9 + a][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Bounds6 b;
    for (int a = 0; a < 3; ++a) {
      b.clo[a] = red[a][0];
      b.chi[a] = red[3 + a][0];
      b.blo[a] = red[6 + a][0];
      b.bhi[a] = red[9 + a][0];
    }
    partial[0] = b;
  }
}

__global__ __launch_bounds__(kBlock) void k_check_spheres_planes(const float* __restrict__ spheres,
                                                                 const uint32_t* __restrict__ smat, int32_t S,
                                                                 const float* __restrict__ planes,
                                                                 const uint32_t* __restrict__ pmat, int32_t P,
                                                                 int32_t M, uint32_t* __restrict__ status) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < S) {
    const float* s = spheres + 4 * i;
    if (!(finite3(s[0], s[1], s[2]) && isfinite(s[3]) && s[3] > 0.f) || smat[i] >= uint32_t(M)) atomicOr(status, 4u);
  } else if (i < S + P) {
    int k = i - S;
    const float* p = planes + 4 * k;
    bool ok = finite3(p[0], p[1], p[2]) && isfinite(p[3]) && (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) > 0.f;
    if (!ok || pmat[k] >= uint32_t(M)) atomicOr(status, 8u);
  }
}

// ---------------------------------------------------------------------------------------------
// 3. Morton codes
// ---------------------------------------------------------------------------------------------

__device__ inline uint64_t spread21(uint32_t x) {
  uint64_t v = x & 0x1fffffu;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__global__ __launch_bounds__(kBlock) void k_morton(const float4* __restrict__ lo, const float4* __restrict__ hi,
                                                   const Bounds6* __restrict__ bounds, int64_t T,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ ids) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= T) return;
  Bounds6 b = bounds[0];
  float4 l = lo[i], h = hi[i];
  float c[3] = {0.5f * l.x + 0.5f * h.x, 0.5f * l.y + 0.5f * h.y, 0.5f * l.z + 0.5f * h.z};
  uint32_t q[3];
  const float cells = 2097152.0f;  // 2^21
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float ext = b.chi[a] - b.clo[a];
    float s = ext > 0.f ? (c[a] - b.clo[a]) / ext * cells : 0.f;
    s = fminf(fmaxf(s, 0.f), cells - 1.f);
    q[a] = uint32_t(s);
  }
  keys[i] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
  ids[i] = uint32_t(i);
}

// ---------------------------------------------------------------------------------------------
// 4. Stable LSD radix sort, 8 bits per pass
// ---------------------------------------------------------------------------------------------

// Per-block digit histogram, stored digit-major: hist[digit * nblocks + block].
__global__ __launch_bounds__(kBlock) void k_digit_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                       uint32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = int64_t(blockIdx.x) * kSortTile;
#pragma unroll 4
  for (int k = 0; k < kSortItems; ++k) {
    int64_t i = base + int64_t(k) * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of hist (length m) in place, one block.
__global__ __launch_bounds__(1024) void k_scan_exclusive(uint32_t* __restrict__ data, int64_t m,
                                                          uint32_t* __restrict__ total_out) {
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  int64_t per = (m + 1023) / 1024;
  int64_t begin = tid * per, end = begin + per < m ? begin + per : m;
  uint32_t s = 0;
  for (int64_t i = begin; i < end; ++i) s += data[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = part[tid] - s;
  for (int64_t i = begin; i < end; ++i) {
    uint32_t x = data[i];
    data[i] = run;
    run += x;
  }
  if (total_out && tid == 1023) *total_out = part[1023];
}

// Multi-block exclusive scan for long arrays: per-tile sums, a scan of the sums, then each tile
// scans itself from its offset.  Tiles are kScanTile consecutive elements, 4 per thread.
constexpr int kScanThreads = 1024, kScanPer = 4, kScanTile = kScanThreads * kScanPer;

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const uint32_t* __restrict__ data, int64_t m,
                                                             uint32_t* __restrict__ sums) {
  __shared__ uint32_t red[kScanThreads / 64];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = base + threadIdx.x + int64_t(k) * kScanThreads;
    if (i < m) s += data[i];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(uint32_t* __restrict__ data, int64_t m,
                                                             const uint32_t* __restrict__ offsets) {
  __shared__ uint32_t part[kScanThreads];
  const int tid = threadIdx.x;
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(tid) * kScanPer;
  uint32_t v[kScanPer];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < m ? data[base + k] : 0u;
    s += v[k];
  }
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t x = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += x;
    __syncthreads();
  }
  uint32_t run = offsets[blockIdx.x] + part[tid] - s;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < m) data[base + k] = run;
    run += v[k];
  }
}

__device__ inline uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Stable scatter: element order inside the tile is (round, thread), i.e. index order.
__global__ __launch_bounds__(kBlock) void k_scatter(const uint64_t* __restrict__ keys_in,
                                                    const uint32_t* __restrict__ ids_in, int64_t n, int shift,
                                                    const uint32_t* __restrict__ offsets, int64_t nblocks,
                                                    uint64_t* __restrict__ keys_out, uint32_t* __restrict__ ids_out) {
  __shared__ uint32_t running[kRadix];
  __shared__ uint32_t wave_cnt[kBlock / 64][kRadix];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  running[tid] = offsets[int64_t(tid) * nblocks + blockIdx.x];
  for (int w = 0; w < kBlock / 64; ++w) wave_cnt[w][tid] = 0;
  __syncthreads();
  int64_t base = int64_t(blockIdx.x) * kSortTile;
  for (int k = 0; k < kSortItems; ++k) {
    int64_t i = base + int64_t(k) * kBlock + tid;
    bool valid = i < n;
    uint64_t key = valid ? keys_in[i] : 0;
    uint32_t id = valid ? ids_in[i] : 0;
    uint32_t digit = uint32_t((key >> shift) & (kRadix - 1));
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      uint64_t bal = __ballot((digit >> b) & 1u);
      peers &= ((digit >> b) & 1u) ? bal : ~bal;
    }
    uint32_t rank = __popcll(peers & lanemask_lt());
    bool leader = valid && rank == 0;
    if (leader) wave_cnt[wave][digit] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[digit] + rank;
      for (int w = 0; w < wave; ++w) pos += wave_cnt[w][digit];
      if (pos < uint64_t(n)) {
        keys_out[pos] = key;
        ids_out[pos] = id;
      }
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      add += wave_cnt[w][tid];
      wave_cnt[w][tid] = 0;
    }
    running[tid] += add;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// 5. Karras (2012) hierarchy emission
// ---------------------------------------------------------------------------------------------

__device__ inline int delta(const uint64_t* __restrict__ k, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = k[i], b = k[j];
  if (a != b) return __clzll(a ^ b);
  return 64 + __clz(uint32_t(i) ^ uint32_t(j));
}

// children[i] = (left, right) references, parents of internal nodes at parent[0..T-2],
// parents of leaves at parent[T-1 + leaf]; range[i] = (first, last) sorted leaf indices.
__global__ __launch_bounds__(kBlock) void k_karras(const uint64_t* __restrict__ keys, int64_t n,
                                                   int2* __restrict__ children, int32_t* __restrict__ parent,
                                                   int2* __restrict__ range) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n - 1) return;
  int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
  int dmin = delta(keys, n, i, i - d);
  int64_t lmax = 2;
  while (delta(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
  int64_t l = 0;
  for (int64_t t = lmax / 2; t >= 1; t /= 2)
    if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
  int64_t j = i + l * d;
  int dnode = delta(keys, n, i, j);
  int64_t s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
  int64_t first = i < j ? i : j, last = i < j ? j : i;
  int left = (first == gamma) ? ~int(gamma) : int(gamma);           // leaf refs as ~index here
  int right = (last == gamma + 1) ? ~int(gamma + 1) : int(gamma + 1);
  children[i] = make_int2(left, right);
  range[i] = make_int2(int(first), int(last));
  if (gamma < 0 || gamma + 1 >= n) return;  // cannot happen for a valid split; never write out of bounds
  if (left < 0) parent[n - 1 + ~left] = int(i); else parent[left] = int(i);
  if (right < 0) parent[n - 1 + ~right] = int(i); else parent[right] = int(i);
}

// ---------------------------------------------------------------------------------------------
// 6./7. Bottom-up refit and cost table
// ---------------------------------------------------------------------------------------------

__device__ inline float half_area(float4 lo, float4 hi) {
  const float dx = hi.x - lo.x, dy = hi.y - lo.y, dz = hi.z - lo.z;
  return dx * dy + dy * dz + dz * dx;
}

#ifndef SRT_DP_TRI_COST
#define SRT_DP_TRI_COST 0.5f
#endif
// Cost-optimal cut of the binary tree into the 4-wide tree (surface-area model, as in Ylitie et al.
// 2017): C(n, j) is the least expected cost of binary subtree n when it may take j slots of its BVH4
// parent.  C(n, 1) = A(n) + D_n(4) (n becomes a BVH4 node whose four slots its two children share),
// D_n(j) = min over k of C(a, k) + C(b, j - k), and C(n, j) = min(C(n, 1), D_n(j)) for j > 1 (n kept
// whole, or opened across j slots).  A leaf costs its area times the relative cost of a triangle test,
// whatever its slot count.  Choice bits per node, for j = 2, 3, 4 at bit 3 (j - 2): the split k
// (2 bits) and whether opening wins.
__device__ inline void dp_child_costs(int r, const float4* dp_cost, const float4* leaf_lo, const float4* leaf_hi,
                                      const uint32_t* sorted_ids, float (&c)[4]) {
  if (r < 0) {
    const uint32_t id = sorted_ids[~r];
    const float a = SRT_DP_TRI_COST * half_area(leaf_lo[id], leaf_hi[id]);
    c[0] = c[1] = c[2] = c[3] = a;
  } else {
    const float4 v = dp_cost[r];
    c[0] = v.x, c[1] = v.y, c[2] = v.z, c[3] = v.w;
  }
}

// Fills the cost table entry of binary node n, whose box and children's entries are final.
__device__ inline void dp_node(int64_t n, const int2* children, const float4* nodebox, const float4* leaf_lo,
                               const float4* leaf_hi, const uint32_t* sorted_ids, float4* dp_cost,
                               uint32_t* dp_choice) {
  const int2 ch = children[n];
  float ca[4], cb[4];
  dp_child_costs(ch.x, dp_cost, leaf_lo, leaf_hi, sorted_ids, ca);
  dp_child_costs(ch.y, dp_cost, leaf_lo, leaf_hi, sorted_ids, cb);
  float D[5];
  int K[5];
  for (int j = 2; j <= 4; ++j) {
    D[j] = INFINITY;
    K[j] = 1;
    for (int k = 1; k < j; ++k) {
      const float c = ca[k - 1] + cb[j - k - 1];
      if (c < D[j]) {
        D[j] = c;
        K[j] = k;
      }
    }
  }
  const float c1 = half_area(nodebox[2 * n], nodebox[2 * n + 1]) + D[4];
  dp_cost[n] = make_float4(c1, fminf(c1, D[2]), fminf(c1, D[3]), fminf(c1, D[4]));
  uint32_t choice = 0;
  for (int j = 2; j <= 4; ++j) choice |= (uint32_t(K[j]) | (D[j] < c1 ? 4u : 0u)) << (3 * (j - 2));
  dp_choice[n] = choice;
}

// The clustering tree's nodes of one round (children were made in earlier rounds).
__global__ __launch_bounds__(kBlock) void k_wide_dp(const int2* __restrict__ children, const float4* nodebox,
                                                    const float4* leaf_lo, const float4* leaf_hi,
                                                    const uint32_t* sorted_ids, float4* dp_cost,
                                                    uint32_t* dp_choice, int64_t first, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= count) return;
  dp_node(first + i, children, nodebox, leaf_lo, leaf_hi, sorted_ids, dp_cost, dp_choice);
}

__global__ __launch_bounds__(kBlock) void k_refit(const int2* __restrict__ children,
                                                  const int32_t* __restrict__ parent,
                                                  const float4* __restrict__ leaf_lo, const float4* __restrict__ leaf_hi,
                                                  const uint32_t* __restrict__ sorted_ids, float4* nodebox,
                                                  uint32_t* flags, int64_t n, int32_t* __restrict__ max_depth,
                                                  uint32_t* __restrict__ status, float4* dp_cost,
                                                  uint32_t* dp_choice) {
  int64_t leaf = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (leaf >= n) return;
  int node = parent[n - 1 + leaf];
  int depth = 1;
  for (int guard = 0; guard < 256; ++guard) {
    if (node < 0 || node >= n - 1) {  // corrupt parent link: report instead of reading out of bounds
      atomicOr(status, 16u);
      return;
    }
    uint32_t old = __hip_atomic_fetch_add(&flags[node], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 0) break;  // the sibling subtree is still being built; its thread climbs on
    int2 ch = children[node];
    float4 lo[2], hi[2];
    int c[2] = {ch.x, ch.y};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (c[k] < 0) {
        uint32_t id = sorted_ids[~c[k]];
        lo[k] = leaf_lo[id];
        hi[k] = leaf_hi[id];
      } else {
        lo[k] = nodebox[2 * c[k]];
        hi[k] = nodebox[2 * c[k] + 1];
      }
    }
    nodebox[2 * node] = make_float4(fminf(lo[0].x, lo[1].x), fminf(lo[0].y, lo[1].y), fminf(lo[0].z, lo[1].z), 0.f);
    nodebox[2 * node + 1] =
        make_float4(fmaxf(hi[0].x, hi[1].x), fmaxf(hi[0].y, hi[1].y), fmaxf(hi[0].z, hi[1].z), 0.f);
    dp_node(node, children, nodebox, leaf_lo, leaf_hi, sorted_ids, dp_cost, dp_choice);
    if (node == 0) break;
    node = parent[node];
  }
  // depth of this leaf: count ancestors (read-only walk over the parent links)
  int nd = parent[n - 1 + leaf];
  while (nd != 0 && depth < 256) {
    nd = parent[nd];
    if (nd < 0 || nd >= n - 1) {
      atomicOr(status, 16u);
      return;
    }
    ++depth;
  }
  atomicMax(max_depth, depth);
}

// ---------------------------------------------------------------------------------------------
// 5'-6'. PLOC: parallel locally-ordered clustering over the Morton order (Meister and Bittner
// 2018), an alternative to steps 5-6.  Clusters start as the sorted leaves.  Each round, every
// cluster finds the neighbour within kPlocRadius positions whose merged box has the smallest
// surface area (ties to the smaller position); mutual pairs merge into a new internal node, and
// the survivors are compacted in order.  The globally best pair is always mutual, so every round
// merges.  Node indices are handed out from T-2 downwards by prefix sums, so the root is node 0 and
// the tree is the same on every run.
// ---------------------------------------------------------------------------------------------

// Search radius: with the cost-table collapse, 32 gives the fewest node visits per frame on the
// benchmark scene (8, 16, 24, 48 and 64 were measured).
#ifndef SRT_PLOC_RADIUS
#define SRT_PLOC_RADIUS 32
#endif
constexpr int kPlocRadius = SRT_PLOC_RADIUS;

__global__ __launch_bounds__(kBlock) void k_ploc_init(const uint32_t* __restrict__ sorted_ids,
                                                      const float4* __restrict__ leaf_lo,
                                                      const float4* __restrict__ leaf_hi, int64_t n,
                                                      float4* __restrict__ c_lo, float4* __restrict__ c_hi,
                                                      int32_t* __restrict__ c_ref) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t id = sorted_ids[i];
  c_lo[i] = leaf_lo[id];
  c_hi[i] = leaf_hi[id];
  c_ref[i] = ~int32_t(i);
}

// nn[i] = the best merge partner of cluster i among positions i-R..i+R (n >= 2).
__global__ __launch_bounds__(kBlock) void k_ploc_nn(const float4* __restrict__ c_lo, const float4* __restrict__ c_hi,
                                                    int64_t n, int32_t* __restrict__ nn) {
  __shared__ float4 s_lo[kBlock + 2 * kPlocRadius], s_hi[kBlock + 2 * kPlocRadius];
  const int64_t start = int64_t(blockIdx.x) * kBlock;
  for (int k = threadIdx.x; k < kBlock + 2 * kPlocRadius; k += kBlock) {
    const int64_t g = start - kPlocRadius + k;
    if (g >= 0 && g < n) {
      s_lo[k] = c_lo[g];
      s_hi[k] = c_hi[g];
    }
  }
  __syncthreads();
  const int64_t i = start + threadIdx.x;
  if (i >= n) return;
  // the LDS arrays hold positions start - R .. start + kBlock + R - 1
  nn[i] = int32_t(ploc_partner(s_lo, s_hi, start - kPlocRadius, i, n, kPlocRadius));
}

__global__ __launch_bounds__(kBlock) void k_ploc_flags(const int32_t* __restrict__ nn, int64_t n,
                                                       uint32_t* __restrict__ keep, uint32_t* __restrict__ merge) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t j = nn[i];
  const bool mutual = nn[j] == int32_t(i);
  merge[i] = (mutual && int64_t(j) > i) ? 1u : 0u;  // the lower position of a mutual pair makes the node
  keep[i] = (mutual && int64_t(j) < i) ? 0u : 1u;   // the higher one is absorbed
}

struct PlocCompactArgs {
  const float4* c_lo;
  const float4* c_hi;
  const int32_t* c_ref;
  const int32_t* nn;
  const uint32_t* keep_pos;   // exclusive prefix sums of the keep flags
  const uint32_t* merge_pos;  // ... and of the merge flags
  int64_t n;
  int64_t node_base;  // index of this round's first new node
  float4* o_lo;
  float4* o_hi;
  int32_t* o_ref;
  int2* children;
  float4* nodebox;
};

__global__ __launch_bounds__(kBlock) void k_ploc_compact(PlocCompactArgs a) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int32_t j = a.nn[i];
  const bool mutual = a.nn[j] == int32_t(i);
  if (mutual && int64_t(j) < i) return;  // absorbed by cluster j
  const uint32_t p = a.keep_pos[i];
  if (mutual) {
    const int64_t node = a.node_base + a.merge_pos[i];
    const float4 alo = a.c_lo[i], ahi = a.c_hi[i], blo = a.c_lo[j], bhi = a.c_hi[j];
    const float4 ulo = make_float4(fminf(alo.x, blo.x), fminf(alo.y, blo.y), fminf(alo.z, blo.z), 0.f);
    const float4 uhi = make_float4(fmaxf(ahi.x, bhi.x), fmaxf(ahi.y, bhi.y), fmaxf(ahi.z, bhi.z), 0.f);
    a.children[node] = make_int2(a.c_ref[i], a.c_ref[j]);
    a.nodebox[2 * node] = ulo;
    a.nodebox[2 * node + 1] = uhi;
    a.o_lo[p] = ulo;
    a.o_hi[p] = uhi;
    a.o_ref[p] = int32_t(node);
  } else {
    a.o_lo[p] = a.c_lo[i];
    a.o_hi[p] = a.c_hi[i];
    a.o_ref[p] = a.c_ref[i];
  }
}

// ---------------------------------------------------------------------------------------------
// 8. Collapse into a 4-wide BVH, top-down one level at a time.  A BVH4 node takes a binary node's two
// children and opens some of them into their own children (keeping left-to-right order) where the
// cost table says, so it holds up to four.  Internal children become the next level's nodes; their
// indices come from a prefix sum, so the layout is deterministic and each level's nodes are
// contiguous.
// ---------------------------------------------------------------------------------------------

constexpr int kWideEmpty = INT32_MIN;

struct WideArgs {
  const int2* children;
  const float4* nodebox;
  const float4* leaf_lo;
  const float4* leaf_hi;
  const uint32_t* sorted_ids;
  const int2* frontier;  // (binary node, BVH4 index)
  int64_t m;
  int4* sel;             // chosen binary-tree references per frontier item
  uint32_t* nint;        // internal children per item -> exclusive offsets (+ total at [m])
  int2* next;            // next frontier
  float4* nodes;         // 8 float4 per BVH4 node
  int64_t level_base;    // BVH4 index of the next level's first node
  float pad;
  const uint32_t* dp_choice;  // per binary node: the cost-optimal cut
};


__global__ __launch_bounds__(kBlock) void k_wide_select(WideArgs a) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= a.m) return;
  const int2 ch = a.children[a.frontier[i].x];
  int r[4] = {ch.x, ch.y, kWideEmpty, kWideEmpty};
  int cnt = 2;
  // follow the cost-optimal cut: the node's four slots split k : 4 - k between its children, and a
  // child with j > 1 slots is opened when that is cheaper
  int js[4] = {int((a.dp_choice[a.frontier[i].x] >> 6) & 3u), 0, 0, 0};
  js[1] = 4 - js[0];
  for (int step = 0; step < 2; ++step) {
    int p = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (p < 0 && k < cnt && r[k] >= 0 && js[k] > 1 && ((a.dp_choice[r[k]] >> (3 * (js[k] - 2) + 2)) & 1u)) p = k;
    if (p < 0) break;
    const int2 c = a.children[r[p]];
    const int kk = int((a.dp_choice[r[p]] >> (3 * (js[p] - 2))) & 3u);
    const int jj = js[p];
#pragma unroll
    for (int k = 3; k > 0; --k)
      if (k > p + 1 && k <= cnt) {
        r[k] = r[k - 1];
        js[k] = js[k - 1];
      }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k == p) {
        r[k] = c.x;
        js[k] = kk;
      }
      if (k == p + 1) {
        r[k] = c.y;
        js[k] = jj - kk;
      }
    }
    ++cnt;
  }
  a.sel[i] = make_int4(r[0], r[1], r[2], r[3]);
  uint32_t n = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) n += (r[k] >= 0) ? 1u : 0u;
  a.nint[i] = n;
}

__global__ __launch_bounds__(kBlock) void k_wide_emit(WideArgs a) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= a.m) return;
  const int b4 = a.frontier[i].y;
  const int4 s4 = a.sel[i];
  const int r[4] = {s4.x, s4.y, s4.z, s4.w};
  const uint32_t off = a.nint[i];
  float lo[3][4], hi[3][4];
  int ref[4];
  uint32_t k_int = 0;
  const float p = a.pad;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float4 l, h;
    if (r[k] == kWideEmpty) {
      // an empty slot: a box at +inf on every axis misses every ray in the slab test
      l = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
      h = l;
      ref[k] = 0;
    } else if (r[k] < 0) {
      const uint32_t id = a.sorted_ids[~r[k]];
      l = a.leaf_lo[id];
      h = a.leaf_hi[id];
      l = make_float4(l.x - p, l.y - p, l.z - p, 0.f);
      h = make_float4(h.x + p, h.y + p, h.z + p, 0.f);
      ref[k] = ~((~r[k]) << 2);
    } else {
      l = a.nodebox[2 * r[k]];
      h = a.nodebox[2 * r[k] + 1];
      l = make_float4(l.x - p, l.y - p, l.z - p, 0.f);
      h = make_float4(h.x + p, h.y + p, h.z + p, 0.f);
      const int idx = int(a.level_base + off + k_int);
      a.next[off + k_int] = make_int2(r[k], idx);
      ++k_int;
      ref[k] = idx;
    }
    lo[0][k] = l.x, lo[1][k] = l.y, lo[2][k] = l.z;
    hi[0][k] = h.x, hi[1][k] = h.y, hi[2][k] = h.z;
  }
#if SRT_QNODE
  // Quantise the children's boxes on the node's own grid: per axis a power-of-two step s with
  // 255 s >= the node's extent, lower corners rounded down and upper corners rounded up.  The
  // differences are formed in FP64 and nudged outwards by one FP64 ulp, so the exact grid box always
  // contains the padded FP32 box.  The node stores 2^24 s (the traversal reads each grid byte as the
  // FP16 value q 2^-24); s >= 2^-126 and, with vertices within RT_MAX_COORD, s <= 2^34, so 2^24 s
  // is a normal float.
  float plo[3], phi[3];
  for (int ax = 0; ax < 3; ++ax) {
    plo[ax] = INFINITY;
    phi[ax] = -INFINITY;
    for (int k = 0; k < 4; ++k)
      if (r[k] != kWideEmpty) {
        plo[ax] = fminf(plo[ax], lo[ax][k]);
        phi[ax] = fmaxf(phi[ax], hi[ax][k]);
      }
  }
  uint32_t qlo[3] = {0u, 0u, 0u}, qhi[3] = {0u, 0u, 0u};
  float steps[3];
  for (int ax = 0; ax < 3; ++ax) {
    const double base = double(plo[ax]);
    const double ext = nextafter(double(phi[ax]) - base, INFINITY);
    int e = -126;
    if (ext > 0.0) {
      int k2;
      frexp(ext / 255.0, &k2);
      e = k2;
      while (e > -126 && ldexp(255.0, e - 1) >= ext) --e;
      while (ldexp(255.0, e) < ext) ++e;
    }
    const double step = ldexp(1.0, e);
    steps[ax] = __uint_as_float(uint32_t(e + 24 + 127) << 23);  // 2^(e + 24)
    for (int k = 0; k < 4; ++k) {
      uint32_t ql = 255u, qh = 0u;
      if (r[k] != kWideEmpty) {
        const double dl = nextafter(double(lo[ax][k]) - base, -INFINITY);
        const double dh = nextafter(double(hi[ax][k]) - base, INFINITY);
        ql = uint32_t(fmin(fmax(floor(dl / step), 0.0), 255.0));
        qh = uint32_t(fmin(fmax(ceil(dh / step), 0.0), 255.0));
      }
      qlo[ax] |= ql << (8 * k);
      qhi[ax] |= qh << (8 * k);
    }
  }
  for (int k = 1; k < 4; ++k)
    if (r[k] == kWideEmpty) ref[k] = ref[0];
  float4* out = a.nodes + 4 * int64_t(b4);
  out[0] = make_float4(plo[0], plo[1], plo[2], steps[0]);
  out[1] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), __int_as_float(ref[2]), __int_as_float(ref[3]));
  out[2] = make_float4(__uint_as_float(qlo[0]), __uint_as_float(qhi[0]), __uint_as_float(qlo[1]), __uint_as_float(qhi[1]));
  out[3] = make_float4(__uint_as_float(qlo[2]), __uint_as_float(qhi[2]), steps[1], steps[2]);
#else
  float4* out = a.nodes + 8 * int64_t(b4);
  out[0] = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
  out[1] = make_float4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
  out[2] = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
  out[3] = make_float4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
  out[4] = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
  out[5] = make_float4(hi[2][0], hi[2][1], hi[2][2], hi[2][3]);
  out[6] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), __int_as_float(ref[2]), __int_as_float(ref[3]));
  out[7] = make_float4(0.f, 0.f, 0.f, 0.f);
#endif
}

__global__ void k_set_int2(int2* p, int2 v) { *p = v; }

__global__ __launch_bounds__(kBlock) void k_pack_tris(const float* __restrict__ tris, const uint32_t* __restrict__ mat,
                                                      const uint32_t* __restrict__ order, int64_t T,
                                                      float4* __restrict__ recs) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= T) return;
  uint32_t id = order ? order[i] : uint32_t(i);
  const float* p = tris + 9 * int64_t(id);
  float v0x = p[0], v0y = p[1], v0z = p[2];
  recs[3 * i + 0] = make_float4(v0x, v0y, v0z, __int_as_float(int(id)));
  recs[3 * i + 1] = make_float4(p[3] - v0x, p[4] - v0y, p[5] - v0z, __int_as_float(int(mat[id])));
  recs[3 * i + 2] = make_float4(p[6] - v0x, p[7] - v0y, p[8] - v0z, 0.f);
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n, int b = kBlock) { return unsigned((n + b - 1) / b); }

}  // namespace

// In-place exclusive scan of data[0, m); the total goes to *total_out if it is not null.  `tmp`
// holds scan_tmp_entries(m) words.
int64_t scan_tmp_entries(int64_t m) { return m / kScanTile + 2; }

hipError_t scan_exclusive(uint32_t* data, int64_t m, uint32_t* total_out, uint32_t* tmp, hipStream_t s) {
  if (m <= 2 * kScanTile) {
    k_scan_exclusive<<<1, 1024, 0, s>>>(data, m, total_out);
    return hipGetLastError();
  }
  const int64_t nb = (m + kScanTile - 1) / kScanTile;
  k_tile_sums<<<unsigned(nb), kScanThreads, 0, s>>>(data, m, tmp);
  k_scan_exclusive<<<1, 1024, 0, s>>>(tmp, nb, total_out);
  k_tile_scan<<<unsigned(nb), kScanThreads, 0, s>>>(data, m, tmp);
  return hipGetLastError();
}

BuildPlan plan_build(int64_t T, int64_t S, int64_t P, int64_t M, int64_t L, bool bvh, bool ploc) {
  BuildPlan p{};
  p.T = T;
  p.bvh = bvh && T >= 2;
  p.ploc = ploc;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  int64_t num_nodes = p.bvh ? T - 1 : 0;  // an upper bound for the 4-wide tree
  p.nodes_off = take(size_t(num_nodes) * kNodeBytes);
  p.tris_off = take(size_t(T) * 48);
  p.spheres_off = take(size_t(S) * 16);
  p.sphere_mat_off = take(size_t(S) * 4);
  p.planes_off = take(size_t(P) * 16);
  p.plane_mat_off = take(size_t(P) * 4);
  p.mats_off = take(size_t(M) * 48);
  p.lights_off = take(size_t(L) * 32 + 32);
  p.storage_bytes = off;

  off = 0;
  p.num_blocks_prep = (T + kBlock - 1) / kBlock;
  p.num_sort_blocks = (T + kSortTile - 1) / kSortTile;
  p.status_off = take(64);
  p.partial_off = take(size_t(p.num_blocks_prep > 0 ? p.num_blocks_prep : 1) * sizeof(Bounds6));
  if (T > 0) {
    p.lo_off = take(size_t(T) * 16);
    p.hi_off = take(size_t(T) * 16);
  }
  if (p.bvh) {
    p.keys0_off = take(size_t(T) * 8);
    p.keys1_off = take(size_t(T) * 8);
    p.ids0_off = take(size_t(T) * 4);
    p.ids1_off = take(size_t(T) * 4);
    p.hist_off = take(size_t(p.num_sort_blocks) * kRadix * 4);
    p.children_off = take(size_t(T) * 8);
    p.nodebox_off = take(size_t(T) * 32);
    if (!ploc) {
      p.range_off = take(size_t(T) * 8);
      p.parent_off = take(size_t(2 * T) * 4);
      p.flags_off = take(size_t(T) * 4);
    }
    p.dp_cost_off = take(size_t(T) * 16);
    p.dp_choice_off = take(size_t(T) * 4);
    p.frontier_off[0] = take(size_t(T) * 8);
    p.frontier_off[1] = take(size_t(T) * 8);
    p.sel_off = take(size_t(T) * 16);
    p.nint_off = take(size_t(T + 1) * 4);
    p.scan_tmp_off = take(size_t(scan_tmp_entries(std::max<int64_t>(T + 1, p.num_sort_blocks * kRadix))) * 4);
    if (ploc) {
      for (int k = 0; k < 2; ++k) {
        p.ploc_lo_off[k] = take(size_t(T) * 16);
        p.ploc_hi_off[k] = take(size_t(T) * 16);
        p.ploc_ref_off[k] = take(size_t(T) * 4);
      }
      p.ploc_nn_off = take(size_t(T) * 4);
      p.ploc_keep_off = take(size_t(T + 1) * 4);
      p.ploc_merge_off = take(size_t(T + 1) * 4);
    }
  }
  p.scratch_bytes = off;
  return p;
}

hipError_t build_scene_device(const rt_scene_desc* desc, const BuildPlan& plan, char* storage, char* scratch,
                              hipStream_t stream, BuildResult* result) {
  const int64_t T = desc->num_triangles;
  const int S = desc->num_spheres, P = desc->num_planes, M = desc->num_materials, L = desc->num_lights;
  uint32_t* status = reinterpret_cast<uint32_t*>(scratch + plan.status_off);
  hipError_t e;
#define SRT_CHECK(x)                   \
  do {                                 \
    e = (x);                           \
    if (e != hipSuccess) return e;     \
  } while (0)
#define SRT_LAUNCH_CHECK() SRT_CHECK(hipGetLastError())

  k_fill<uint32_t><<<1, 64, 0, stream>>>(status, 0u, 16);
  SRT_LAUNCH_CHECK();

  // spheres, planes, materials, lights
  if (S > 0) {
    SRT_CHECK(hipMemcpyAsync(storage + plan.spheres_off, desc->spheres, size_t(S) * 16, hipMemcpyDeviceToDevice, stream));
    SRT_CHECK(hipMemcpyAsync(storage + plan.sphere_mat_off, desc->sphere_material, size_t(S) * 4,
                             hipMemcpyDeviceToDevice, stream));
  }
  if (P > 0) {
    SRT_CHECK(hipMemcpyAsync(storage + plan.planes_off, desc->planes, size_t(P) * 16, hipMemcpyDeviceToDevice, stream));
    SRT_CHECK(hipMemcpyAsync(storage + plan.plane_mat_off, desc->plane_material, size_t(P) * 4,
                             hipMemcpyDeviceToDevice, stream));
  }
  if (S + P > 0) {
    k_check_spheres_planes<<<blocks_for(S + P), kBlock, 0, stream>>>(desc->spheres, desc->sphere_material, S,
                                                                     desc->planes, desc->plane_material, P, M, status);
    SRT_LAUNCH_CHECK();
  }
  {
    // materials: (kd, n), (ks, 0), (kr, 0); lights: (pos, 0), (I, 0)
    size_t mb = size_t(M) * 48, lb = size_t(L) * 32;
    float* host = static_cast<float*>(std::malloc(mb + lb + 16));
    if (!host) return hipErrorOutOfMemory;
    for (int i = 0; i < M; ++i) {
      const rt_material& m = desc->materials[i];
      float* o = host + 12 * i;
      o[0] = m.albedo[0], o[1] = m.albedo[1], o[2] = m.albedo[2], o[3] = m.shininess;
      o[4] = m.specular[0], o[5] = m.specular[1], o[6] = m.specular[2], o[7] = 0.f;
      o[8] = m.reflectance[0], o[9] = m.reflectance[1], o[10] = m.reflectance[2], o[11] = 0.f;
    }
    for (int i = 0; i < L; ++i) {
      const rt_light& l = desc->lights[i];
      float* o = host + 12 * M + 8 * i;
      o[0] = l.position[0], o[1] = l.position[1], o[2] = l.position[2], o[3] = 0.f;
      o[4] = l.intensity[0], o[5] = l.intensity[1], o[6] = l.intensity[2], o[7] = 0.f;
    }
    e = hipMemcpyAsync(storage + plan.mats_off, host, mb, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && lb)
      e = hipMemcpyAsync(storage + plan.lights_off, reinterpret_cast<char*>(host) + mb, lb, hipMemcpyHostToDevice,
                         stream);
    // pageable source: wait before freeing it
    hipError_t e2 = hipStreamSynchronize(stream);
    std::free(host);
    SRT_CHECK(e);
    SRT_CHECK(e2);
  }

  result->depth = 0;
  result->max_leaf = T > 0 ? 1 : 0;
  result->num_nodes = 0;
  result->root = 0;
  for (int a = 0; a < 3; ++a) result->lo[a] = result->hi[a] = 0.f;

  float4* recs = reinterpret_cast<float4*>(storage + plan.tris_off);
  Bounds6 bounds{};
  int32_t depth = 0;
  if (T > 0) {
    float4* lo = reinterpret_cast<float4*>(scratch + plan.lo_off);
    float4* hi = reinterpret_cast<float4*>(scratch + plan.hi_off);
    Bounds6* partial = reinterpret_cast<Bounds6*>(scratch + plan.partial_off);
    k_tri_prep<<<blocks_for(T), kBlock, 0, stream>>>(desc->triangles, desc->tri_material, T, M, lo, hi, partial,
                                                     status);
    SRT_LAUNCH_CHECK();
    k_reduce_bounds<<<1, kBlock, 0, stream>>>(partial, plan.num_blocks_prep);
    SRT_LAUNCH_CHECK();

    if (plan.bvh) {
      uint64_t* k0 = reinterpret_cast<uint64_t*>(scratch + plan.keys0_off);
      uint64_t* k1 = reinterpret_cast<uint64_t*>(scratch + plan.keys1_off);
      uint32_t* i0 = reinterpret_cast<uint32_t*>(scratch + plan.ids0_off);
      uint32_t* i1 = reinterpret_cast<uint32_t*>(scratch + plan.ids1_off);
      uint32_t* hist = reinterpret_cast<uint32_t*>(scratch + plan.hist_off);
      uint32_t* scan_tmp = reinterpret_cast<uint32_t*>(scratch + plan.scan_tmp_off);
      k_morton<<<blocks_for(T), kBlock, 0, stream>>>(lo, hi, partial, T, k0, i0);
      SRT_LAUNCH_CHECK();
      const int64_t nb = plan.num_sort_blocks;
      for (int pass = 0; pass < 8; ++pass) {
        int shift = pass * kRadixBits;
        k_digit_hist<<<unsigned(nb), kBlock, 0, stream>>>(k0, T, shift, hist, nb);
        SRT_LAUNCH_CHECK();
        SRT_CHECK(scan_exclusive(hist, nb * kRadix, nullptr, scan_tmp, stream));
        k_scatter<<<unsigned(nb), kBlock, 0, stream>>>(k0, i0, T, shift, hist, nb, k1, i1);
        SRT_LAUNCH_CHECK();
        std::swap(k0, k1);
        std::swap(i0, i1);
      }
      // after 8 passes the sorted data is back in the *0 buffers
      int2* children = reinterpret_cast<int2*>(scratch + plan.children_off);
      int2* range = reinterpret_cast<int2*>(scratch + plan.range_off);
      int32_t* parent = reinterpret_cast<int32_t*>(scratch + plan.parent_off);
      uint32_t* flags = reinterpret_cast<uint32_t*>(scratch + plan.flags_off);
      float4* nodebox = reinterpret_cast<float4*>(scratch + plan.nodebox_off);
      float4* dp_cost = reinterpret_cast<float4*>(scratch + plan.dp_cost_off);
      uint32_t* dp_choice = reinterpret_cast<uint32_t*>(scratch + plan.dp_choice_off);
      if (plan.ploc) {
        float4* c_lo[2] = {reinterpret_cast<float4*>(scratch + plan.ploc_lo_off[0]),
                           reinterpret_cast<float4*>(scratch + plan.ploc_lo_off[1])};
        float4* c_hi[2] = {reinterpret_cast<float4*>(scratch + plan.ploc_hi_off[0]),
                           reinterpret_cast<float4*>(scratch + plan.ploc_hi_off[1])};
        int32_t* c_ref[2] = {reinterpret_cast<int32_t*>(scratch + plan.ploc_ref_off[0]),
                             reinterpret_cast<int32_t*>(scratch + plan.ploc_ref_off[1])};
        int32_t* nn = reinterpret_cast<int32_t*>(scratch + plan.ploc_nn_off);
        uint32_t* keep = reinterpret_cast<uint32_t*>(scratch + plan.ploc_keep_off);
        uint32_t* merge = reinterpret_cast<uint32_t*>(scratch + plan.ploc_merge_off);
        k_ploc_init<<<blocks_for(T), kBlock, 0, stream>>>(i0, lo, hi, T, c_lo[0], c_hi[0], c_ref[0]);
        SRT_LAUNCH_CHECK();
        std::vector<std::pair<int64_t, int64_t>> round_nodes;  // nodes each round created, in merge order
        int64_t n = T, next = T - 1;
        int cur = 0;
        for (int round = 0; n > 1; ++round) {
          if (round >= T) return hipErrorUnknown;  // every round merges at least one pair
          k_ploc_nn<<<blocks_for(n), kBlock, 0, stream>>>(c_lo[cur], c_hi[cur], n, nn);
          SRT_LAUNCH_CHECK();
          k_ploc_flags<<<blocks_for(n), kBlock, 0, stream>>>(nn, n, keep, merge);
          SRT_LAUNCH_CHECK();
          SRT_CHECK(scan_exclusive(keep, n, keep + n, scan_tmp, stream));
          SRT_CHECK(scan_exclusive(merge, n, merge + n, scan_tmp, stream));
          uint32_t totals[2] = {0u, 0u};
          SRT_CHECK(hipMemcpyAsync(&totals[0], keep + n, 4, hipMemcpyDeviceToHost, stream));
          SRT_CHECK(hipMemcpyAsync(&totals[1], merge + n, 4, hipMemcpyDeviceToHost, stream));
          SRT_CHECK(hipStreamSynchronize(stream));
          const int64_t merges = totals[1];
          if (merges < 1 || merges > next || int64_t(totals[0]) != n - merges) return hipErrorUnknown;
          PlocCompactArgs ca;
          ca.c_lo = c_lo[cur];
          ca.c_hi = c_hi[cur];
          ca.c_ref = c_ref[cur];
          ca.nn = nn;
          ca.keep_pos = keep;
          ca.merge_pos = merge;
          ca.n = n;
          ca.node_base = next - merges;
          ca.o_lo = c_lo[cur ^ 1];
          ca.o_hi = c_hi[cur ^ 1];
          ca.o_ref = c_ref[cur ^ 1];
          ca.children = children;
          ca.nodebox = nodebox;
          k_ploc_compact<<<blocks_for(n), kBlock, 0, stream>>>(ca);
          SRT_LAUNCH_CHECK();
          round_nodes.emplace_back(next - merges, merges);
          next -= merges;
          n -= merges;
          cur ^= 1;
        }
        if (next != 0) return hipErrorUnknown;  // T - 1 merges make a binary tree rooted at node 0
        for (const auto& rn : round_nodes) {  // children were created in earlier rounds
          k_wide_dp<<<blocks_for(rn.second), kBlock, 0, stream>>>(children, nodebox, lo, hi, i0, dp_cost, dp_choice,
                                                                  rn.first, rn.second);
          SRT_LAUNCH_CHECK();
        }
        SRT_CHECK(hipMemcpyAsync(&bounds, partial, sizeof(bounds), hipMemcpyDeviceToHost, stream));
        SRT_CHECK(hipStreamSynchronize(stream));
      } else {
        int32_t* dmax = reinterpret_cast<int32_t*>(status + 4);
        k_karras<<<blocks_for(T - 1), kBlock, 0, stream>>>(k0, T, children, parent, range);
        SRT_LAUNCH_CHECK();
        k_fill<uint32_t><<<blocks_for(T - 1), kBlock, 0, stream>>>(flags, 0u, T - 1);
        SRT_LAUNCH_CHECK();
        k_refit<<<blocks_for(T), kBlock, 0, stream>>>(children, parent, lo, hi, i0, nodebox, flags, T, dmax, status,
                                                      dp_cost, dp_choice);
        SRT_LAUNCH_CHECK();
        // read back the scene bounds for the padding
        SRT_CHECK(hipMemcpyAsync(&bounds, partial, sizeof(bounds), hipMemcpyDeviceToHost, stream));
        SRT_CHECK(hipMemcpyAsync(&depth, dmax, sizeof(depth), hipMemcpyDeviceToHost, stream));
        SRT_CHECK(hipStreamSynchronize(stream));
      }
      float coord_max = 0.f;
      for (int a = 0; a < 3; ++a)
        coord_max = std::max(coord_max, std::max(std::fabs(bounds.blo[a]), std::fabs(bounds.bhi[a])));
      WideArgs wa;
      wa.children = children;
      wa.nodebox = nodebox;
      wa.leaf_lo = lo;
      wa.leaf_hi = hi;
      wa.sorted_ids = i0;
      wa.sel = reinterpret_cast<int4*>(scratch + plan.sel_off);
      wa.nint = reinterpret_cast<uint32_t*>(scratch + plan.nint_off);
      wa.nodes = reinterpret_cast<float4*>(storage + plan.nodes_off);
      wa.pad = coord_max * 0x1p-18f + 1e-20f;  // conservative box growth (slab and triangle-test rounding)
      wa.dp_choice = dp_choice;
      int2* fr[2] = {reinterpret_cast<int2*>(scratch + plan.frontier_off[0]),
                     reinterpret_cast<int2*>(scratch + plan.frontier_off[1])};
      k_set_int2<<<1, 1, 0, stream>>>(fr[0], make_int2(0, 0));
      SRT_LAUNCH_CHECK();
      int64_t m = 1, allocated = 1;
      int levels = 0;
      while (m > 0) {
        wa.frontier = fr[levels & 1];
        wa.next = fr[(levels + 1) & 1];
        wa.m = m;
        wa.level_base = allocated;
        k_wide_select<<<blocks_for(m), kBlock, 0, stream>>>(wa);
        SRT_LAUNCH_CHECK();
        SRT_CHECK(scan_exclusive(wa.nint, m, wa.nint + m, scan_tmp, stream));
        k_wide_emit<<<blocks_for(m), kBlock, 0, stream>>>(wa);
        SRT_LAUNCH_CHECK();
        uint32_t next_m = 0;
        SRT_CHECK(hipMemcpyAsync(&next_m, wa.nint + m, sizeof(next_m), hipMemcpyDeviceToHost, stream));
        SRT_CHECK(hipStreamSynchronize(stream));
        allocated += next_m;
        m = next_m;
        ++levels;
        if (allocated > T - 1) return hipErrorUnknown;  // every level adds nodes: impossible for a valid hierarchy
      }
      result->num_nodes = allocated;
      depth = levels;
      k_pack_tris<<<blocks_for(T), kBlock, 0, stream>>>(desc->triangles, desc->tri_material, i0, T, recs);
      SRT_LAUNCH_CHECK();
      result->root = 0;
    } else {
      k_pack_tris<<<blocks_for(T), kBlock, 0, stream>>>(desc->triangles, desc->tri_material, nullptr, T, recs);
      SRT_LAUNCH_CHECK();
      SRT_CHECK(hipMemcpyAsync(&bounds, partial, sizeof(bounds), hipMemcpyDeviceToHost, stream));
      result->root = ~0;  // a single leaf holding record 0 (used only when T == 1)
    }
  }
  uint32_t st = 0;
  SRT_CHECK(hipMemcpyAsync(&st, status, sizeof(st), hipMemcpyDeviceToHost, stream));
  SRT_CHECK(hipStreamSynchronize(stream));
  result->status_bits = st;
  result->depth = depth;
  for (int a = 0; a < 3; ++a) {
    result->lo[a] = T > 0 ? bounds.blo[a] : 0.f;
    result->hi[a] = T > 0 ? bounds.bhi[a] : 0.f;
  }
  return hipSuccess;
#undef SRT_CHECK
#undef SRT_LAUNCH_CHECK
}

}  // namespace srt
