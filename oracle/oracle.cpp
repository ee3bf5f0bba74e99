// Stereo Whitted ray-tracing oracle: plain, slow, FP64, brute force.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this library.  It shares no code, header
// or constant with the GPU library, and the GPU library never calls it.
//
// What it computes (the paper, Sections 2-3): a stereo pair is two projections
// of one scene, one from each of the observer's eyes ("double rendering"), each
// synthesised by backward ray tracing, with every pixel's rays independent of
// every other pixel's.  The paper names no camera, shading model or recursion;
// the readings taken here are:
//   * an off-axis stereo pair: eyes at C -+ (B/2) r, pixel-centre rays, image
//     centres converging at distance Z0 along the forward axis;
//   * Whitted recursion without refraction: a closest hit, Phong lighting
//     (kd N.L + ks max(0, R.V)^n, R = 2(N.L)N - L, no distance falloff) from
//     every point light that a shadow ray finds unoccluded, an ambient term
//     ambient*kd, and a mirror ray weighted by kr up to a reflection depth D;
//   * every closest-hit and shadow query answered by testing EVERY primitive
//     (Moller-Trumbore triangles, spheres, planes); ties in t go to the smaller
//     primitive id; secondary rays start at t > 1e-4 and skip the primitive
//     they leave.
// All arithmetic is IEEE binary64, round-to-nearest, built without
// contraction or fast-math.  Inputs are the FP32 scene arrays and camera
// fields, widened exactly.
//
// Besides radiance the oracle returns the ray-tree signature (closest-hit id
// per depth, shadow state per depth and light) and, for each decision, a
// margin: how far the inputs sit from flipping it.  Tests use the margins to
// certify pixels where FP32 and FP64 legitimately choose differently.  Near-miss
// margins of 1e-2 and above are not recorded (reported as +inf): certification
// only ever uses margins below 1e-3.  A shifted render moves chosen hit points
// along their rays before the path goes on, so that a test can ask whether a
// different choice further down a path is the exact answer for a hit point a
// stated distance from the exact one (a backward-error check).

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline V3 mul(V3 a, V3 b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double length(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return (1.0 / length(a)) * a; }
inline V3 load3f(const float* p) { return {double(p[0]), double(p[1]), double(p[2])}; }

const double kInf = std::numeric_limits<double>::infinity();
const double kSecondaryTmin = 1e-4;  // self-intersection offset for spawned rays (scene units)
const double kNearMiss = 1e-2;       // margins above this are not recorded

}  // namespace

extern "C" {

typedef struct {
  int64_t num_triangles;
  const float* triangles;  // [T][3][3]
  const uint32_t* tri_material;
  int32_t num_spheres;
  const float* spheres;  // [S][4] centre, radius
  const uint32_t* sphere_material;
  int32_t num_planes;
  const float* planes;  // [P][4] normal, offset (n.x = d)
  const uint32_t* plane_material;
  int32_t num_materials;
  const float* materials;  // [M][10] kd, ks, kr, shininess
  int32_t num_lights;
  const float* lights;  // [L][6] position, intensity
  float ambient[3];
  float background[3];
} orc_scene;

typedef struct {
  float center[3], forward[3], up[3];
  float hfov_deg, baseline, convergence;
  int32_t width, height, max_depth;
} orc_camera;

typedef struct {
  double* radiance;         // [n][3]
  double* hit_t;            // [n] primary t, +inf on a miss
  int32_t* hit_prim;        // [n] primary id, -1 on a miss
  int32_t* path_prims;      // [n][D+1] closest-hit id per depth; -1 miss, -2 ray not spawned
  uint8_t* shadow_state;    // [n][D+1][L] 0 not cast, 1 occluded, 2 visible
  double* hit_margin;       // [n][D+1] closest-hit decision margin (inf when not spawned)
  double* shadow_margin;    // [n][D+1][L] cast and occlusion decision margin
  double* shadow_contrib;   // [n][D+1][L] radiance the light's decision is worth at the pixel
  double* path_t;           // [n][D+1] closest-hit distance per depth; +inf on a miss or not spawned
  double* hit_cos;          // [n] |cos| of the angle between the primary ray and the hit's normal; NaN on a miss
  int64_t ray_counts[3];    // out: primary, reflection, shadow rays traced
  double seconds[2];        // out: wall time of the tree build (0 in brute force) and of the tracing
} orc_output;

}  // extern "C"

namespace {

struct Tri {
  V3 v0, e1, e2;
};

struct Scene {
  std::vector<Tri> tris;
  std::vector<uint32_t> tri_mat;
  std::vector<V3> sph_c;
  std::vector<double> sph_r;
  std::vector<uint32_t> sph_mat;
  std::vector<V3> pl_n;
  std::vector<double> pl_d;
  std::vector<uint32_t> pl_mat;
  struct Mat {
    V3 kd, ks, kr;
    double n;
  };
  std::vector<Mat> mats;
  struct Light {
    V3 pos, I;
  };
  std::vector<Light> lights;
  V3 ambient, background;
  int64_t T = 0, S = 0, P = 0;
};

Scene load_scene(const orc_scene* s) {
  Scene sc;
  sc.T = s->num_triangles;
  sc.S = s->num_spheres;
  sc.P = s->num_planes;
  sc.tris.resize(size_t(sc.T));
  for (int64_t i = 0; i < sc.T; ++i) {
    const float* p = s->triangles + 9 * i;
    V3 a = load3f(p), b = load3f(p + 3), c = load3f(p + 6);
    sc.tris[size_t(i)] = {a, b - a, c - a};
  }
  sc.tri_mat.assign(s->tri_material, s->tri_material + sc.T);
  for (int64_t i = 0; i < sc.S; ++i) {
    sc.sph_c.push_back(load3f(s->spheres + 4 * i));
    sc.sph_r.push_back(double(s->spheres[4 * i + 3]));
    sc.sph_mat.push_back(s->sphere_material[i]);
  }
  for (int64_t i = 0; i < sc.P; ++i) {
    sc.pl_n.push_back(load3f(s->planes + 4 * i));
    sc.pl_d.push_back(double(s->planes[4 * i + 3]));
    sc.pl_mat.push_back(s->plane_material[i]);
  }
  for (int i = 0; i < s->num_materials; ++i) {
    const float* m = s->materials + 10 * i;
    sc.mats.push_back({load3f(m), load3f(m + 3), load3f(m + 6), double(m[9])});
  }
  for (int i = 0; i < s->num_lights; ++i) {
    const float* l = s->lights + 6 * i;
    sc.lights.push_back({load3f(l), load3f(l + 3)});
  }
  sc.ambient = load3f(s->ambient);
  sc.background = load3f(s->background);
  return sc;
}

// ---------------------------------------------------------------------------------------------
// Ray-primitive tests.  Each returns the parametric distance of the candidate
// intersection in *t and whether it is accepted for t in (tmin, tmax).
// ---------------------------------------------------------------------------------------------

// Moller & Trumbore (1997): solve O + t d = v0 + u e1 + v e2 by Cramer's rule.
// Closed triangle (inclusive edges); only det == 0 is rejected.
// *margin gets the signed barycentric distance to the nearest edge, min(u, v, 1-u-v),
// times the sine of the ray's angle to the plane (how far, in relative terms,
// the ray passes from flipping the inside/outside decision).
inline bool hit_triangle(const Tri& tr, V3 O, V3 d, double tmin, double tmax, double* t, double* u_out,
                         double* v_out, double* margin) {
  V3 Tv = O - tr.v0;
  V3 P = cross(d, tr.e2);
  double det = dot(tr.e1, P);
  *margin = kInf;
  if (det == 0.0) return false;
  double u = dot(Tv, P) / det;
  V3 Q = cross(Tv, tr.e1);
  double v = dot(d, Q) / det;
  double tt = dot(tr.e2, Q) / det;
  *t = tt;
  *u_out = u;
  *v_out = v;
  double m = std::fmin(u, std::fmin(v, 1.0 - u - v));
  double sin_angle = std::fabs(det) / (length(cross(tr.e1, tr.e2)) * length(d));
  *margin = m * sin_angle;
  return u >= 0.0 && v >= 0.0 && u + v <= 1.0 && tt > tmin && tt < tmax;
}

// Sphere with unit-length d: b = -oc.d is the foot of the perpendicular from the
// centre, h^2 = |oc + b d|^2 its squared distance, disc = r^2 - h^2; roots b -+ sqrt(disc).
inline bool hit_sphere(V3 c, double r, V3 O, V3 d, double tmin, double tmax, double* t, double* margin) {
  V3 oc = O - c;
  double b = -dot(oc, d);
  V3 foot = oc + b * d;
  double h2 = dot(foot, foot);
  double disc = r * r - h2;
  *margin = disc / (r * r);
  if (disc < 0.0) {
    *t = b;  // closest approach, so that a near miss in front is seen as one
    return false;
  }
  double s = std::sqrt(disc);
  double t0 = b - s, t1 = b + s;
  if (t0 > tmin && t0 < tmax) {
    *t = t0;
    return true;
  }
  if (t1 > tmin && t1 < tmax) {
    *t = t1;
    return true;
  }
  return false;
}

inline bool hit_plane(V3 n, double dist, V3 O, V3 d, double tmin, double tmax, double* t, double* margin) {
  double nd = dot(n, d);
  *margin = std::fabs(nd) / (length(n) * length(d));
  if (nd == 0.0) return false;
  double tt = (dist - dot(n, O)) / nd;
  *t = tt;
  return tt > tmin && tt < tmax;
}

struct Hit {
  double t = kInf;
  int64_t prim = -1;
  double margin = kInf;
};

// Relative distance of a candidate t from an interval end point.
inline double t_margin(double t, double edge) {
  if (edge == 0.0 || !std::isfinite(edge)) return kInf;
  return std::fabs(t - edge) / std::fabs(edge);
}

// Closest hit over every primitive: minimum t, exact ties to the smaller id.
// The decision margin is the smallest of: the winner's inside margin, the
// outside margin of every near-missed primitive lying in front of the winner,
// the relative t gap to the runner-up, and the distance of any candidate t from tmin.
Hit closest_hit(const Scene& sc, V3 O, V3 d, double tmin, int64_t exclude) {
  Hit best;
  double second_t = kInf;
  struct Near {
    double t, m;
  };
  std::vector<Near> near;
  auto consider = [&](int64_t id, bool hit, double t, double m) {
    if (std::fabs(m) < kNearMiss && t > tmin * (1.0 - kNearMiss)) near.push_back({t, std::fabs(m)});
    if (tmin > 0.0 && std::isfinite(t) && t_margin(t, tmin) < kNearMiss) near.push_back({t, t_margin(t, tmin)});
    if (!hit) return;
    if (t < best.t || (t == best.t && id < best.prim)) {
      if (best.prim >= 0) second_t = std::fmin(second_t, best.t);
      best.t = t;
      best.prim = id;
    } else {
      second_t = std::fmin(second_t, t);
    }
  };
  for (int64_t i = 0; i < sc.T; ++i) {
    if (i == exclude) continue;
    double t = kInf, u, v, m;
    bool h = hit_triangle(sc.tris[size_t(i)], O, d, tmin, kInf, &t, &u, &v, &m);
    consider(i, h, t, m);
  }
  for (int64_t i = 0; i < sc.S; ++i) {
    int64_t id = sc.T + i;
    if (id == exclude) continue;
    double t = kInf, m;
    bool h = hit_sphere(sc.sph_c[size_t(i)], sc.sph_r[size_t(i)], O, d, tmin, kInf, &t, &m);
    consider(id, h, t, m);
  }
  for (int64_t i = 0; i < sc.P; ++i) {
    int64_t id = sc.T + sc.S + i;
    if (id == exclude) continue;
    double t = kInf, m;
    bool h = hit_plane(sc.pl_n[size_t(i)], sc.pl_d[size_t(i)], O, d, tmin, kInf, &t, &m);
    consider(id, h, t, m);
  }
  double margin = kInf;
  double limit = std::isfinite(best.t) ? best.t * (1.0 + kNearMiss) : kInf;
  for (const Near& n : near)
    if (n.t <= limit) margin = std::fmin(margin, n.m);
  if (best.prim >= 0 && std::isfinite(second_t)) margin = std::fmin(margin, (second_t - best.t) / best.t);
  best.margin = margin;
  return best;
}

// Occlusion: does any primitive other than `exclude` intersect for t in (tmin, tmax)?
// Tests every primitive (no early exit) so that the decision margin is complete.
bool any_hit(const Scene& sc, V3 O, V3 d, double tmin, double tmax, int64_t exclude, double* margin_out) {
  bool occluded = false;
  double margin = kInf;
  auto consider = [&](bool hit, double t, double m) {
    bool in_range = t > tmin * (1.0 - kNearMiss) && t < tmax * (1.0 + kNearMiss);
    if (in_range) margin = std::fmin(margin, std::fabs(m));
    if (std::isfinite(t)) {
      if (t_margin(t, tmin) < kNearMiss) margin = std::fmin(margin, t_margin(t, tmin));
      if (t_margin(t, tmax) < kNearMiss) margin = std::fmin(margin, t_margin(t, tmax));
    }
    occluded = occluded || hit;
  };
  for (int64_t i = 0; i < sc.T; ++i) {
    if (i == exclude) continue;
    double t = kInf, u, v, m;
    bool h = hit_triangle(sc.tris[size_t(i)], O, d, tmin, tmax, &t, &u, &v, &m);
    consider(h, t, m);
  }
  for (int64_t i = 0; i < sc.S; ++i) {
    int64_t id = sc.T + i;
    if (id == exclude) continue;
    double t = kInf, m;
    bool h = hit_sphere(sc.sph_c[size_t(i)], sc.sph_r[size_t(i)], O, d, tmin, tmax, &t, &m);
    consider(h, t, m);
  }
  for (int64_t i = 0; i < sc.P; ++i) {
    int64_t id = sc.T + sc.S + i;
    if (id == exclude) continue;
    double t = kInf, m;
    bool h = hit_plane(sc.pl_n[size_t(i)], sc.pl_d[size_t(i)], O, d, tmin, tmax, &t, &m);
    consider(h, t, m);
  }
  *margin_out = margin;
  return occluded;
}

// ---------------------------------------------------------------------------------------------
// Triangle hierarchy for the second mode: a binary tree built top-down by splitting the triangles
// at the median centroid on the longest axis of the centroid bounds, at most four triangles per
// leaf.  Node boxes bound the triangles' vertices (exact in FP64, the inputs being FP32) and are
// padded outwards by kBvhPad times the scene's largest coordinate, far more than the rounding of
// the slab and triangle arithmetic, so a ray that hits a triangle at t enters every box above it at
// or before t.
// ---------------------------------------------------------------------------------------------

const double kBvhPad = 1e-9;

struct Bvh {
  struct Node {
    double lo[3], hi[3];
    int64_t left;   // inner node: left child; leaf: position of its first triangle in `order`
    int32_t count;  // triangles in a leaf, 0 for an inner node
    int64_t right;  // inner node: right child
  };
  std::vector<Node> nodes;
  std::vector<int64_t> order;  // triangle ids in leaf order
};

Bvh build_bvh(const Scene& sc) {
  Bvh b;
  const int64_t T = sc.T;
  if (T == 0) return b;
  std::vector<V3> cen(static_cast<size_t>(T));
  double big = 0.0;
  for (int64_t i = 0; i < T; ++i) {
    const Tri& t = sc.tris[size_t(i)];
    V3 v1 = t.v0 + t.e1, v2 = t.v0 + t.e2;
    cen[size_t(i)] = (1.0 / 3.0) * (t.v0 + v1 + v2);
    for (V3 v : {t.v0, v1, v2})
      big = std::fmax(big, std::fmax(std::fabs(v.x), std::fmax(std::fabs(v.y), std::fabs(v.z))));
  }
  const double pad = kBvhPad * (1.0 + big);
  b.order.resize(size_t(T));
  for (int64_t i = 0; i < T; ++i) b.order[size_t(i)] = i;
  struct Task {
    int64_t node, begin, end;
  };
  b.nodes.push_back({});
  std::vector<Task> todo{{0, 0, T}};
  while (!todo.empty()) {
    Task k = todo.back();
    todo.pop_back();
    Bvh::Node nd;
    for (int a = 0; a < 3; ++a) nd.lo[a] = kInf, nd.hi[a] = -kInf;
    double clo[3] = {kInf, kInf, kInf}, chi[3] = {-kInf, -kInf, -kInf};
    for (int64_t i = k.begin; i < k.end; ++i) {
      const int64_t id = b.order[size_t(i)];
      const Tri& t = sc.tris[size_t(id)];
      for (V3 v : {t.v0, t.v0 + t.e1, t.v0 + t.e2}) {
        const double c[3] = {v.x, v.y, v.z};
        for (int a = 0; a < 3; ++a) nd.lo[a] = std::fmin(nd.lo[a], c[a]), nd.hi[a] = std::fmax(nd.hi[a], c[a]);
      }
      const double c[3] = {cen[size_t(id)].x, cen[size_t(id)].y, cen[size_t(id)].z};
      for (int a = 0; a < 3; ++a) clo[a] = std::fmin(clo[a], c[a]), chi[a] = std::fmax(chi[a], c[a]);
    }
    for (int a = 0; a < 3; ++a) nd.lo[a] -= pad, nd.hi[a] += pad;
    if (k.end - k.begin <= 4) {
      nd.left = k.begin;
      nd.count = int32_t(k.end - k.begin);
      nd.right = -1;
      b.nodes[size_t(k.node)] = nd;
      continue;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    const int64_t mid = (k.begin + k.end) / 2;
    auto key = [&](int64_t id) {
      const V3& c = cen[size_t(id)];
      return axis == 0 ? c.x : (axis == 1 ? c.y : c.z);
    };
    std::nth_element(b.order.begin() + k.begin, b.order.begin() + mid, b.order.begin() + k.end,
                     [&](int64_t x, int64_t y) { return key(x) < key(y) || (key(x) == key(y) && x < y); });
    nd.count = 0;
    nd.left = int64_t(b.nodes.size());
    nd.right = nd.left + 1;
    b.nodes[size_t(k.node)] = nd;
    b.nodes.push_back({});
    b.nodes.push_back({});
    todo.push_back({nd.left, k.begin, mid});
    todo.push_back({nd.right, mid, k.end});
  }
  return b;
}

// Parametric interval where the ray is inside the box, clipped to [tmin, tmax]; false if empty.
inline bool enter_box(const Bvh::Node& n, V3 O, V3 d, double tmin, double tmax, double* t_enter) {
  const double o[3] = {O.x, O.y, O.z}, dd[3] = {d.x, d.y, d.z};
  double t0 = tmin, t1 = tmax;
  for (int a = 0; a < 3; ++a) {
    if (dd[a] == 0.0) {
      if (o[a] < n.lo[a] || o[a] > n.hi[a]) return false;
      continue;
    }
    double ta = (n.lo[a] - o[a]) / dd[a], tb = (n.hi[a] - o[a]) / dd[a];
    if (ta > tb) std::swap(ta, tb);
    t0 = std::fmax(t0, ta);
    t1 = std::fmin(t1, tb);
  }
  *t_enter = t0;
  return t0 <= t1;
}

// Closest hit through the tree: the same candidates and tie rule as closest_hit, no margin.
Hit closest_hit_bvh(const Scene& sc, const Bvh& b, V3 O, V3 d, double tmin, int64_t exclude) {
  Hit best;
  auto consider = [&](int64_t id, bool hit, double t) {
    if (hit && (t < best.t || (t == best.t && id < best.prim))) best.t = t, best.prim = id;
  };
  if (!b.nodes.empty()) {
    std::vector<int64_t> stack{0};
    while (!stack.empty()) {
      const Bvh::Node& n = b.nodes[size_t(stack.back())];
      stack.pop_back();
      double te;
      if (!enter_box(n, O, d, tmin, best.t, &te)) continue;
      if (n.count > 0) {
        for (int64_t i = n.left; i < n.left + n.count; ++i) {
          const int64_t id = b.order[size_t(i)];
          if (id == exclude) continue;
          double t = kInf, u, v, m;
          bool h = hit_triangle(sc.tris[size_t(id)], O, d, tmin, kInf, &t, &u, &v, &m);
          consider(id, h, t);
        }
        continue;
      }
      double tl = 0.0, tr = 0.0;
      const bool hl = enter_box(b.nodes[size_t(n.left)], O, d, tmin, best.t, &tl);
      const bool hr = enter_box(b.nodes[size_t(n.right)], O, d, tmin, best.t, &tr);
      if (hl && hr) {  // nearer child on top
        stack.push_back(tl <= tr ? n.right : n.left);
        stack.push_back(tl <= tr ? n.left : n.right);
      } else if (hl) {
        stack.push_back(n.left);
      } else if (hr) {
        stack.push_back(n.right);
      }
    }
  }
  for (int64_t i = 0; i < sc.S; ++i) {
    int64_t id = sc.T + i;
    if (id == exclude) continue;
    double t = kInf, m;
    bool h = hit_sphere(sc.sph_c[size_t(i)], sc.sph_r[size_t(i)], O, d, tmin, kInf, &t, &m);
    consider(id, h, t);
  }
  for (int64_t i = 0; i < sc.P; ++i) {
    int64_t id = sc.T + sc.S + i;
    if (id == exclude) continue;
    double t = kInf, m;
    bool h = hit_plane(sc.pl_n[size_t(i)], sc.pl_d[size_t(i)], O, d, tmin, kInf, &t, &m);
    consider(id, h, t);
  }
  best.margin = std::numeric_limits<double>::quiet_NaN();
  return best;
}

// Occlusion through the tree: the same yes/no as any_hit, no margin.
bool any_hit_bvh(const Scene& sc, const Bvh& b, V3 O, V3 d, double tmin, double tmax, int64_t exclude) {
  for (int64_t i = 0; i < sc.S; ++i) {
    int64_t id = sc.T + i;
    double t = kInf, m;
    if (id != exclude && hit_sphere(sc.sph_c[size_t(i)], sc.sph_r[size_t(i)], O, d, tmin, tmax, &t, &m)) return true;
  }
  for (int64_t i = 0; i < sc.P; ++i) {
    int64_t id = sc.T + sc.S + i;
    double t = kInf, m;
    if (id != exclude && hit_plane(sc.pl_n[size_t(i)], sc.pl_d[size_t(i)], O, d, tmin, tmax, &t, &m)) return true;
  }
  if (b.nodes.empty()) return false;
  std::vector<int64_t> stack{0};
  while (!stack.empty()) {
    const Bvh::Node& n = b.nodes[size_t(stack.back())];
    stack.pop_back();
    double te;
    if (!enter_box(n, O, d, tmin, tmax, &te)) continue;
    if (n.count > 0) {
      for (int64_t i = n.left; i < n.left + n.count; ++i) {
        const int64_t id = b.order[size_t(i)];
        if (id == exclude) continue;
        double t = kInf, u, v, m;
        if (hit_triangle(sc.tris[size_t(id)], O, d, tmin, tmax, &t, &u, &v, &m)) return true;
      }
      continue;
    }
    stack.push_back(n.right);
    stack.push_back(n.left);
  }
  return false;
}

// ---------------------------------------------------------------------------------------------
// Stereo camera (off-axis pair)
// ---------------------------------------------------------------------------------------------

struct Camera {
  V3 C, f, r, u;
  double fpx, cx, cy, B, Z0;
  int W, H, D;
};

Camera make_camera(const orc_camera* c) {
  Camera cam;
  cam.C = load3f(c->center);
  cam.f = normalize(load3f(c->forward));
  cam.r = normalize(cross(load3f(c->up), cam.f));
  cam.u = cross(cam.f, cam.r);
  double half = 0.5 * double(c->hfov_deg) * M_PI / 180.0;
  cam.W = c->width;
  cam.H = c->height;
  cam.D = c->max_depth;
  cam.fpx = (0.5 * double(cam.W)) / std::tan(half);
  cam.cx = 0.5 * double(cam.W);
  cam.cy = 0.5 * double(cam.H);
  cam.B = double(c->baseline);
  cam.Z0 = double(c->convergence);
  return cam;
}

// Eye e (0 left, 1 right) sits at C + s_e r with s = -+B/2; the ray through the
// centre of pixel (i, j) (column left to right, row top to bottom).  With a
// positive convergence distance the frustum is sheared by -s_e/Z0 so that the
// image centres of both eyes meet at C + Z0 f.
void primary_ray(const Camera& cam, int eye, int i, int j, V3* O, V3* d) {
  double s = (eye == 0 ? -0.5 : 0.5) * cam.B;
  *O = cam.C + s * cam.r;
  double a = (double(i) + 0.5 - cam.cx) / cam.fpx;
  if (cam.Z0 > 0.0) a -= s / cam.Z0;
  double b = -(double(j) + 0.5 - cam.cy) / cam.fpx;
  *d = normalize(cam.f + a * cam.r + b * cam.u);
}

// ---------------------------------------------------------------------------------------------
// Whitted recursion
// ---------------------------------------------------------------------------------------------

struct PathRecord {
  V3 radiance;
  double hit_t;
  double hit_cos = std::numeric_limits<double>::quiet_NaN();
  int32_t hit_prim;
  int32_t* path_prims;
  uint8_t* shadow_state;
  double* hit_margin;
  double* shadow_margin;
  double* shadow_contrib;
  double* path_t;
  const double* t_shift;  // null, or [D+1] distances added to each depth's hit distance
  int64_t n_refl = 0, n_shadow = 0;
};

struct Tracer {
  const Scene& sc;
  int D;
  int L;
  const Bvh* bvh;  // null: brute force with margins

  uint32_t material_of(int64_t prim) const {
    if (prim < sc.T) return sc.tri_mat[size_t(prim)];
    if (prim < sc.T + sc.S) return sc.sph_mat[size_t(prim - sc.T)];
    return sc.pl_mat[size_t(prim - sc.T - sc.S)];
  }

  V3 geometric_normal(int64_t prim, V3 P) const {
    if (prim < sc.T) {
      const Tri& t = sc.tris[size_t(prim)];
      return normalize(cross(t.e1, t.e2));
    }
    if (prim < sc.T + sc.S) {
      size_t k = size_t(prim - sc.T);
      return (1.0 / sc.sph_r[k]) * (P - sc.sph_c[k]);
    }
    return normalize(sc.pl_n[size_t(prim - sc.T - sc.S)]);
  }

  // Radiance arriving along ray (O, d) at recursion depth `depth`.
  V3 trace(V3 O, V3 d, int depth, double tmin, int64_t exclude, V3 throughput, PathRecord& rec) const {
    Hit h = bvh ? closest_hit_bvh(sc, *bvh, O, d, tmin, exclude) : closest_hit(sc, O, d, tmin, exclude);
    rec.path_prims[depth] = int32_t(h.prim);
    rec.hit_margin[depth] = h.margin;
    rec.path_t[depth] = h.t;
    if (depth == 0) {
      rec.hit_t = h.t;
      rec.hit_prim = int32_t(h.prim);
    }
    if (h.prim < 0) return sc.background;

    // A shifted hit point (for backward-error checks) moves along the ray; the primitive stays.
    double th = rec.t_shift ? h.t + rec.t_shift[depth] : h.t;
    V3 P = O + th * d;
    V3 Ng = geometric_normal(h.prim, P);
    if (depth == 0) rec.hit_cos = std::fabs(dot(Ng, d)) / (length(Ng) * length(d));
    V3 N = dot(Ng, d) > 0.0 ? -1.0 * Ng : Ng;
    V3 V = -1.0 * d;
    const Scene::Mat& m = sc.mats[material_of(h.prim)];

    V3 Lo = mul(sc.ambient, m.kd);
    for (int l = 0; l < L; ++l) {
      const Scene::Light& lt = sc.lights[size_t(l)];
      V3 Lv = lt.pos - P;
      double dist = length(Lv);
      V3 Ld = (1.0 / dist) * Lv;
      double ndl = dot(N, Ld);
      size_t k = size_t(depth) * size_t(L) + size_t(l);
      double cast_margin = std::fabs(ndl);
      if (dist > kSecondaryTmin && ndl > 0.0) {
        V3 R = (2.0 * ndl) * N - Ld;
        double rv = std::fmax(0.0, dot(R, V));
        double spec = std::pow(rv, m.n);
        V3 term = mul(lt.I, ndl * m.kd + spec * m.ks);
        V3 w = mul(term, throughput);
        rec.shadow_contrib[k] = std::fmax(std::fabs(w.x), std::fmax(std::fabs(w.y), std::fabs(w.z)));
        double occ_margin = std::numeric_limits<double>::quiet_NaN();
        bool occ = bvh ? any_hit_bvh(sc, *bvh, P, Ld, kSecondaryTmin, dist, h.prim)
                       : any_hit(sc, P, Ld, kSecondaryTmin, dist, h.prim, &occ_margin);
        rec.n_shadow++;
        rec.shadow_margin[k] = std::fmin(cast_margin, occ_margin);
        rec.shadow_state[k] = occ ? 1 : 2;
        if (!occ) Lo = Lo + term;
      } else {
        // Not cast.  Its worth is the jump the Phong term makes at N.L = 0.
        double rv = std::fmax(0.0, dot(-1.0 * Ld, V));
        V3 w = mul(mul(lt.I, std::pow(rv, m.n) * m.ks), throughput);
        rec.shadow_contrib[k] = std::fmax(std::fabs(w.x), std::fmax(std::fabs(w.y), std::fabs(w.z)));
        rec.shadow_margin[k] = cast_margin;
        rec.shadow_state[k] = 0;
      }
    }
    bool reflective = m.kr.x != 0.0 || m.kr.y != 0.0 || m.kr.z != 0.0;
    if (depth < D && reflective) {
      V3 r = normalize(d - (2.0 * dot(d, N)) * N);
      rec.n_refl++;
      V3 Li = trace(P, r, depth + 1, kSecondaryTmin, h.prim, mul(throughput, m.kr), rec);
      Lo = Lo + mul(m.kr, Li);
    }
    return Lo;
  }
};

int render_paths(const orc_scene* scene_in, const orc_camera* cam_in, const int64_t* samples, int64_t n,
                 int32_t nthreads, bool use_bvh, const double* t_shift, orc_output* out) {
  if (!scene_in || !cam_in || !out || cam_in->width <= 0 || cam_in->height <= 0 || cam_in->max_depth < 0)
    return -1;
  Scene sc = load_scene(scene_in);
  Camera cam = make_camera(cam_in);
  const auto t_build = std::chrono::steady_clock::now();
  Bvh bvh;
  if (use_bvh) bvh = build_bvh(sc);
  const auto t_trace = std::chrono::steady_clock::now();
  const int64_t HW = int64_t(cam.W) * cam.H;
  const int64_t total = samples ? n : 2 * HW;
  const int D = cam.D;
  const int L = int(sc.lights.size());
  Tracer tracer{sc, D, L, use_bvh ? &bvh : nullptr};
  std::atomic<int64_t> next{0}, n_refl{0}, n_shadow{0};
  const int64_t chunk = 4;
  auto worker = [&]() {
    int64_t my_refl = 0, my_shadow = 0;
    for (;;) {
      int64_t start = next.fetch_add(chunk);
      if (start >= total) break;
      int64_t end = std::min(total, start + chunk);
      for (int64_t s = start; s < end; ++s) {
        int64_t pid = samples ? samples[s] : s;
        int eye = int(pid / HW);
        int64_t px = pid % HW;
        int row = int(px / cam.W), col = int(px % cam.W);
        PathRecord rec;
        rec.path_prims = out->path_prims + s * (D + 1);
        rec.shadow_state = out->shadow_state + s * (D + 1) * L;
        rec.hit_margin = out->hit_margin + s * (D + 1);
        rec.shadow_margin = out->shadow_margin + s * (D + 1) * L;
        rec.shadow_contrib = out->shadow_contrib + s * (D + 1) * L;
        rec.path_t = out->path_t + s * (D + 1);
        rec.t_shift = t_shift ? t_shift + s * (D + 1) : nullptr;
        for (int k = 0; k <= D; ++k) {
          rec.path_prims[k] = -2;
          rec.hit_margin[k] = kInf;
          rec.path_t[k] = kInf;
        }
        for (int k = 0; k < (D + 1) * L; ++k) {
          rec.shadow_state[k] = 0;
          rec.shadow_margin[k] = kInf;
          rec.shadow_contrib[k] = 0.0;
        }
        V3 O, d;
        primary_ray(cam, eye, col, row, &O, &d);
        V3 Lr = tracer.trace(O, d, 0, 0.0, -1, V3{1.0, 1.0, 1.0}, rec);
        out->radiance[3 * s + 0] = Lr.x;
        out->radiance[3 * s + 1] = Lr.y;
        out->radiance[3 * s + 2] = Lr.z;
        out->hit_t[s] = rec.hit_t;
        out->hit_cos[s] = rec.hit_cos;
        out->hit_prim[s] = rec.hit_prim;
        my_refl += rec.n_refl;
        my_shadow += rec.n_shadow;
      }
    }
    n_refl += my_refl;
    n_shadow += my_shadow;
  };
  int nt = nthreads > 0 ? nthreads : 1;
  std::vector<std::thread> pool;
  for (int i = 1; i < nt; ++i) pool.emplace_back(worker);
  worker();
  for (auto& t : pool) t.join();
  const auto t_end = std::chrono::steady_clock::now();
  out->seconds[0] = std::chrono::duration<double>(t_trace - t_build).count();
  out->seconds[1] = std::chrono::duration<double>(t_end - t_trace).count();
  out->ray_counts[0] = total;
  out->ray_counts[1] = n_refl.load();
  out->ray_counts[2] = n_shadow.load();
  return 0;
}

}  // namespace

extern "C" {

// Renders the sampled paths (path id = eye*H*W + row*W + col; NULL = all 2*H*W of them) with
// `nthreads` worker threads pulling rows of work dynamically, testing every primitive for every
// query.  Returns 0 on success, -1 on invalid arguments.
int orc_render(const orc_scene* scene_in, const orc_camera* cam_in, const int64_t* samples, int64_t n,
               int32_t nthreads, orc_output* out) {
  return render_paths(scene_in, cam_in, samples, n, nthreads, false, nullptr, out);
}

// The same render through the triangle hierarchy: the same radiance and ray-tree signature; the
// margins are NaN (not computed).
int orc_render_bvh(const orc_scene* scene_in, const orc_camera* cam_in, const int64_t* samples, int64_t n,
                   int32_t nthreads, orc_output* out) {
  return render_paths(scene_in, cam_in, samples, n, nthreads, true, nullptr, out);
}

// Either render with the hit point of sampled path s at depth k moved along its ray by
// t_shift[s*(D+1) + k] (a signed distance; the primitive hit is kept).  Used to ask whether a
// different choice further down the path is what exact arithmetic gives for a hit point within a
// stated distance of the exact one.  accel: 0 brute force (with margins), 1 hierarchy.
int orc_render_shifted(const orc_scene* scene_in, const orc_camera* cam_in, const int64_t* samples, int64_t n,
                       int32_t nthreads, int32_t accel, const double* t_shift, orc_output* out) {
  if ((accel != 0 && accel != 1) || !t_shift) return -1;
  return render_paths(scene_in, cam_in, samples, n, nthreads, accel == 1, t_shift, out);
}

// Single primary ray, for camera checks.
void orc_primary_ray(const orc_camera* c, int32_t eye, int32_t col, int32_t row, double* O, double* d) {
  Camera cam = make_camera(c);
  V3 o, dd;
  primary_ray(cam, eye, col, row, &o, &dd);
  O[0] = o.x, O[1] = o.y, O[2] = o.z;
  d[0] = dd.x, d[1] = dd.y, d[2] = dd.z;
}

// Single ray-primitive tests, for the pins.  *margin (may be NULL) gets the decision margin the
// renderer records for the primitive: the triangle's barycentric edge margin times the sine of the
// ray's angle to its plane, disc/r^2 for a sphere (unit d), the sine of the grazing angle for a plane.
int32_t orc_intersect_triangle(const double* O, const double* d, const double* v0, const double* v1,
                               const double* v2, double tmin, double tmax, double* t, double* u, double* v,
                               double* margin) {
  V3 a{v0[0], v0[1], v0[2]}, b{v1[0], v1[1], v1[2]}, c{v2[0], v2[1], v2[2]};
  Tri tr{a, b - a, c - a};
  double m;
  *t = kInf;
  bool hit = hit_triangle(tr, V3{O[0], O[1], O[2]}, V3{d[0], d[1], d[2]}, tmin, tmax, t, u, v, &m);
  if (margin) *margin = m;
  return hit ? 1 : 0;
}

int32_t orc_intersect_sphere(const double* O, const double* d, const double* c, double r, double tmin, double tmax,
                             double* t, double* margin) {
  double m;
  *t = kInf;
  bool hit = hit_sphere(V3{c[0], c[1], c[2]}, r, V3{O[0], O[1], O[2]}, V3{d[0], d[1], d[2]}, tmin, tmax, t, &m);
  if (margin) *margin = m;
  if (hit) return 1;
  *t = kInf;
  return 0;
}

int32_t orc_intersect_plane(const double* O, const double* d, const double* n, double dist, double tmin, double tmax,
                            double* t, double* margin) {
  double m;
  *t = kInf;
  bool hit = hit_plane(V3{n[0], n[1], n[2]}, dist, V3{O[0], O[1], O[2]}, V3{d[0], d[1], d[2]}, tmin, tmax, t, &m);
  if (margin) *margin = m;
  return hit ? 1 : 0;
}

// Closest hit (t, id, decision margin) of explicit rays against a scene, for the pins.  d need not
// be unit length for triangles and planes; spheres require unit d.  exclude may be NULL.
int32_t orc_closest_hits(const orc_scene* scene_in, const double* O, const double* d, int64_t n, double tmin,
                         const int64_t* exclude, double* t_out, int64_t* prim_out, double* margin_out) {
  Scene sc = load_scene(scene_in);
  for (int64_t i = 0; i < n; ++i) {
    Hit h = closest_hit(sc, V3{O[3 * i], O[3 * i + 1], O[3 * i + 2]}, V3{d[3 * i], d[3 * i + 1], d[3 * i + 2]}, tmin,
                        exclude ? exclude[i] : -1);
    t_out[i] = h.t;
    prim_out[i] = h.prim;
    if (margin_out) margin_out[i] = h.margin;
  }
  return 0;
}

// Occlusion of explicit segments (t in (tmin, tmax)) and its decision margin, for the pins.
int32_t orc_occluded(const orc_scene* scene_in, const double* O, const double* d, int64_t n, double tmin,
                     const double* tmax, const int64_t* exclude, int32_t* occluded_out, double* margin_out) {
  Scene sc = load_scene(scene_in);
  for (int64_t i = 0; i < n; ++i) {
    double m;
    occluded_out[i] = any_hit(sc, V3{O[3 * i], O[3 * i + 1], O[3 * i + 2]}, V3{d[3 * i], d[3 * i + 1], d[3 * i + 2]},
                              tmin, tmax[i], exclude ? exclude[i] : -1, &m)
                          ? 1
                          : 0;
    if (margin_out) margin_out[i] = m;
  }
  return 0;
}

}  // extern "C"
