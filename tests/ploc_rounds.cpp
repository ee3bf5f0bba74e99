// Host-side check of the clustering builder's merge rounds, built with the kernel's own partner rule
// (paper_1702_01530_amd/csrc/ploc_rule.h).  Each round every cluster picks its partner, mutual pairs
// merge in place of their lower position and the survivors keep their order, as the device rounds
// do.  Checks that every round merges at least one pair on inputs full of exact ties: the case of a
// distant box, a box B and two boxes at B's low and high corners, boxes snapped to a coarse grid,
// nested and coincident boxes.  Prints one line per case and exits non-zero on a failure.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_1702_01530_amd/csrc/ploc_rule.h"

struct V4 {
  float x, y, z, w;
};

struct Result {
  bool ok;
  int rounds;
  int depth;
};

// Runs rounds until one cluster is left; returns whether every round merged and the tree depth.
static Result build(std::vector<V4> lo, std::vector<V4> hi, int radius, std::vector<int64_t>* first_nn) {
  int64_t n = int64_t(lo.size());
  std::vector<int> depth(size_t(n), 0);
  int rounds = 0;
  while (n > 1) {
    std::vector<int64_t> nn(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) nn[size_t(i)] = srt::ploc_partner(lo.data(), hi.data(), 0, i, n, radius);
    if (first_nn && rounds == 0) *first_nn = nn;
    std::vector<V4> nlo, nhi;
    std::vector<int> ndepth;
    int64_t merges = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t j = nn[size_t(i)];
      const bool mutual = nn[size_t(j)] == i;
      if (mutual && j < i) continue;  // absorbed by the lower position
      if (mutual) {
        ++merges;
        const V4 a = lo[size_t(i)], b = lo[size_t(j)], c = hi[size_t(i)], d = hi[size_t(j)];
        nlo.push_back({std::min(a.x, b.x), std::min(a.y, b.y), std::min(a.z, b.z), 0.f});
        nhi.push_back({std::max(c.x, d.x), std::max(c.y, d.y), std::max(c.z, d.z), 0.f});
        ndepth.push_back(1 + std::max(depth[size_t(i)], depth[size_t(j)]));
      } else {
        nlo.push_back(lo[size_t(i)]);
        nhi.push_back(hi[size_t(i)]);
        ndepth.push_back(depth[size_t(i)]);
      }
    }
    ++rounds;
    if (merges < 1) return {false, rounds, 0};
    lo.swap(nlo);
    hi.swap(nhi);
    depth.swap(ndepth);
    n = int64_t(lo.size());
  }
  return {true, rounds, depth[0]};
}

static int failures = 0;

static void report(const char* name, bool ok, const char* detail) {
  std::printf("%s %s %s\n", ok ? "OK" : "FAIL", name, detail);
  if (!ok) ++failures;
}

int main() {
  char buf[256];
  {
    // a distant box, B's low corner, B = [0,2]^3, B's high corner, in Morton order: every merge with
    // B or between the corners gives B's area exactly
    std::vector<V4> lo = {{-50, -50, -50, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {1.99f, 1.99f, 1.99f, 0}};
    std::vector<V4> hi = {{-49, -49, -49, 0}, {0.01f, 0.01f, 0.01f, 0}, {2, 2, 2, 0}, {2, 2, 2, 0}};
    std::vector<int64_t> nn;
    Result r = build(lo, hi, 32, &nn);
    std::snprintf(buf, sizeof buf, "nn=[%lld,%lld,%lld,%lld] rounds=%d", (long long)nn[0], (long long)nn[1],
                  (long long)nn[2], (long long)nn[3], r.rounds);
    report("corners_of_a_box", r.ok && nn[1] == 2 && nn[2] == 1, buf);
  }
  {
    // coincident boxes: pairs (0,1), (2,3), ... every round, so the depth is ceil(log2 n)
    for (int n : {2, 3, 7, 300, 1025}) {
      std::vector<V4> lo(size_t(n), V4{0, 0, 0, 0}), hi(size_t(n), V4{1, 2, 0, 0});
      Result r = build(lo, hi, 32, nullptr);
      int expect = 0;
      while ((1 << expect) < n) ++expect;
      std::snprintf(buf, sizeof buf, "n=%d rounds=%d depth=%d (log2 bound %d)", n, r.rounds, r.depth, expect);
      report("coincident", r.ok && r.depth == expect, buf);
    }
  }
  {
    // nested boxes of growing size in Morton order merge one pair per round into a chain as deep as
    // the input is long: the rounds still all merge, and the build falls back to the Karras tree when
    // such a chain is too deep for the traversal stack
    const int n = 200;
    std::vector<V4> lo(static_cast<size_t>(n), V4{0, 0, 0, 0}), hi;
    float s = 1.0f;
    for (int i = 0; i < n; ++i, s *= 1.2f) hi.push_back(V4{s, s, s, 0});
    Result r = build(lo, hi, 32, nullptr);
    std::snprintf(buf, sizeof buf, "n=%d rounds=%d depth=%d", n, r.rounds, r.depth);
    report("nested_chain", r.ok && r.depth == n - 1, buf);
  }
  {
    // random boxes on a coarse integer grid (many exact ties), points, nested boxes, duplicates
    std::mt19937 rng(12345);
    for (int trial = 0; trial < 400; ++trial) {
      const int n = 2 + int(rng() % 700), g = 1 + int(rng() % 4);
      std::vector<V4> lo(static_cast<size_t>(n)), hi(static_cast<size_t>(n));
      for (int i = 0; i < n; ++i) {
        float a[3], b[3];
        for (int k = 0; k < 3; ++k) {
          a[k] = float(int(rng() % 5) * g);
          b[k] = a[k] + float(int(rng() % 3) * g);  // zero extent is common
        }
        if (i > 0 && rng() % 4 == 0) {  // a copy of, or a box inside, the previous one
          lo[size_t(i)] = lo[size_t(i - 1)];
          hi[size_t(i)] = rng() % 2 ? hi[size_t(i - 1)] : lo[size_t(i - 1)];
          continue;
        }
        lo[size_t(i)] = {a[0], a[1], a[2], 0};
        hi[size_t(i)] = {b[0], b[1], b[2], 0};
      }
      // order by a coarse key so that equal boxes are neighbours, as the Morton order makes them
      std::vector<int> idx(static_cast<size_t>(n));
      for (int i = 0; i < n; ++i) idx[size_t(i)] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](int p, int q) {
        const V4 &u = lo[size_t(p)], &v = lo[size_t(q)];
        return u.x + 7 * u.y + 49 * u.z < v.x + 7 * v.y + 49 * v.z;
      });
      std::vector<V4> slo, shi;
      for (int i : idx) {
        slo.push_back(lo[size_t(i)]);
        shi.push_back(hi[size_t(i)]);
      }
      const int radius = trial % 3 == 0 ? 1 : (trial % 3 == 1 ? 8 : 32);
      Result r = build(slo, shi, radius, nullptr);
      if (!r.ok) {
        std::snprintf(buf, sizeof buf, "trial=%d n=%d grid=%d radius=%d round %d merged nothing", trial, n, g, radius,
                      r.rounds);
        report("grid_ties", false, buf);
      }
    }
    report("grid_ties", failures == 0, "400 trials");
  }
  return failures ? 1 : 0;
}
