// The merge-partner rule of the clustering tree builder (locally-ordered clustering over the Morton
// order, Meister and Bittner 2018), shared by the build kernel and a host-side check of its rounds.
//
// Plain C++: the including translation unit defines SRT_HD (e.g. `__host__ __device__`) before the
// include to make the functions callable from kernels; a host-only build leaves it empty.  V is any
// type with float members x, y, z (float4 in the kernels).
#pragma once

#include <math.h>
#include <stdint.h>

#ifndef SRT_HD
#define SRT_HD
#endif

namespace srt {

// Surface area (up to the factor 2) of the union of boxes a and b.  Symmetric in a and b, and never
// below either box's own area (max/min are exact and correctly rounded sums and products of
// non-negative values are monotone), which the mutual-pair argument below relies on.
template <class V>
SRT_HD inline float merged_area(V alo, V ahi, V blo, V bhi) {
  const float dx = fmaxf(ahi.x, bhi.x) - fminf(alo.x, blo.x);
  const float dy = fmaxf(ahi.y, bhi.y) - fminf(alo.y, blo.y);
  const float dz = fmaxf(ahi.z, bhi.z) - fminf(alo.z, blo.z);
  return dx * dy + dy * dz + dz * dx;
}

// Merge partner of cluster i among positions i-R .. i+R of n clusters (n >= 2): the one whose
// merged box has the smallest area, ties to the smaller position.  lo/hi hold the boxes of
// positions base, base+1, ... (lo[j - base] is position j).
//
// Exception: when i and its parity partner p = i ^ 1 have the same area and merging them does not
// grow it (coincident or identical boxes), i takes p.  Runs of coincident triangles then pair up as
// (0,1), (2,3), ... and halve every round instead of all choosing one cluster and growing a chain.
// The exception applies only when the equalities hold from both sides, so p takes i back: p's best
// is at most merged(p, i) = area(p) and at least area(p) (no merge shrinks a box), so p's own
// exception fires.  Without exceptions, the smallest position of any globally cheapest pair picks
// its smallest cheapest partner, which picks it back.  Either way every round has a mutual pair
// and merges.
template <class V>
SRT_HD inline int64_t ploc_partner(const V* lo, const V* hi, int64_t base, int64_t i, int64_t n, int radius) {
  const V alo = lo[i - base], ahi = hi[i - base];
  float best = __builtin_huge_valf();
  int64_t bj = i > 0 ? i - 1 : i + 1;
  for (int k = -radius; k <= radius; ++k) {  // ascending positions: ties keep the smaller one
    const int64_t j = i + k;
    if (k == 0 || j < 0 || j >= n) continue;
    const float ar = merged_area(alo, ahi, lo[j - base], hi[j - base]);
    if (ar < best) {
      best = ar;
      bj = j;
    }
  }
  const int64_t p = i ^ 1;
  if (p < n) {
    const V plo = lo[p - base], phi = hi[p - base];
    if (best == merged_area(alo, ahi, alo, ahi) && best == merged_area(plo, phi, plo, phi) &&
        best == merged_area(alo, ahi, plo, phi))
      bj = p;
  }
  return bj;
}

}  // namespace srt
