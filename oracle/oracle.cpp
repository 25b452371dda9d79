// FP64 oracle for closest-hit ray intersection with bicubic Bezier and Gregory
// patches by hierarchical parametric subdivision (Binder & Keller, "Massively
// Parallel Stackless Ray Tracing of Catmull-Clark Subdivision Surfaces").
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP
// library is checked against.  It shares no code, header, table or constant
// generator with the library; only tests, the smoke check and the CPU-baseline
// leg of the benchmark may load it.
//
// Conventions (readings of the paper, all documented with the project design):
//   * grid slot(i, j) = 4*j + i, i along u, j along v; f = sum B_i(u) B_j(v) p_ij
//     (Sec. 2.1; Alg. 1 evaluates q_{3,0} at (u1, v0)).
//   * Gregory inner point (i, j): (du P^u + dv P^v)/(du + dv), du = u or 1-u,
//     dv = v or 1-v (the weighting of Alg. 2); P^u in slots 5, 6, 9, 10 and P^v
//     in slots 16..19.
//   * domains are integer (pos, size) in units of 2^-23 (Alg. 3); splits
//     alternate u, v, u, ... (Sec. 3); a node is a leaf at per-axis depth L.
//   * child box = [min, max + d] of the de Casteljau half of the current lower
//     bound grid, d the parent's displacement (Sec. 3.3 and Alg. 3).
//   * the reported hit is the entry distance into the closest leaf box and the
//     leaf-domain centre (Sec. 3: bounding boxes alone give the intersection).
//
// Everything is IEEE double, compiled without fast-math and without contraction.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace orc {

struct V3 {
  double x, y, z;
};
static inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
static inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
static inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
static inline V3 vmin(V3 a, V3 b) { return {std::min(a.x, b.x), std::min(a.y, b.y), std::min(a.z, b.z)}; }
static inline V3 vmax(V3 a, V3 b) { return {std::max(a.x, b.x), std::max(a.y, b.y), std::max(a.z, b.z)}; }
static inline V3 vabs(V3 a) { return {std::fabs(a.x), std::fabs(a.y), std::fabs(a.z)}; }
static inline double at(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
static inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
static inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

static const int kInner[4] = {5, 6, 9, 10};  // (1,1) (2,1) (1,2) (2,2): P^u
static const int kInnerV[4] = {16, 17, 18, 19};  // P^v, same order
static const double kUnit = 1.0 / 8388608.0;  // 2^-23
static const uint32_t kFull = 1u << 23;
static const uint32_t kNoHit = 0xFFFFFFFFu;

struct Grid {
  V3 p[16];
};

struct Patch {
  V3 cp[20];
  bool gregory;
  V3 lo, hi;  // hull of the 16 (Bezier) or 20 (Gregory) points
  double pad = 0.0;  // every subdivision box grown by this on all sides (patch-local frames)
};

struct Ray {
  V3 o, d;
  double tmin, tmax;
};

struct Best {
  double t;
  uint32_t id;
  double u, v;
};

struct Counters {  // per ray
  uint32_t node, cand, split, backtrack, greg, leaf, crop, cand_greg;
};

// ------------------------------------------------------------------ evaluation
static void bernstein(double t, double b[4]) {
  double s = 1.0 - t;
  b[0] = s * s * s;
  b[1] = 3.0 * t * s * s;
  b[2] = 3.0 * t * t * s;
  b[3] = t * t * t;
}

// d/dt B_k^3(t) = 3 (B_{k-1}^2(t) - B_k^2(t))
static void bernstein_d(double t, double b[4]) {
  double s = 1.0 - t;
  b[0] = -3.0 * s * s;
  b[1] = 3.0 * s * s - 6.0 * t * s;
  b[2] = 6.0 * t * s - 3.0 * t * t;
  b[3] = 3.0 * t * t;
}

// Tensor-product Bernstein sum and its first and mixed partial derivatives.
static void bezier_eval(const Grid& g, double u, double v, V3* f, V3* fu, V3* fv, V3* fuv) {
  double bu[4], bv[4], du[4], dv[4];
  bernstein(u, bu);
  bernstein(v, bv);
  bernstein_d(u, du);
  bernstein_d(v, dv);
  V3 a = {0, 0, 0}, b = {0, 0, 0}, c = {0, 0, 0}, e = {0, 0, 0};
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) {
      V3 p = g.p[4 * j + i];
      a = a + (bu[i] * bv[j]) * p;
      b = b + (du[i] * bv[j]) * p;
      c = c + (bu[i] * dv[j]) * p;
      e = e + (du[i] * dv[j]) * p;
    }
  if (f) *f = a;
  if (fu) *fu = b;
  if (fv) *fv = c;
  if (fuv) *fuv = e;
}

// Blend parameters of inner point k: du = u or 1-u, dv = v or 1-v.
static inline bool inner_first_u(int k) { return (k & 1) == 0; }  // i == 1
static inline bool inner_first_v(int k) { return (k & 2) == 0; }  // j == 1

// Surface point and first partials of a Bezier or Gregory patch (Sec. 2.2): the
// Gregory patch is the Bezier patch whose inner points are the (u, v)-dependent
// blends; the partials include the derivative of the blend weights.
static void patch_eval(const Patch& P, double u, double v, V3* f, V3* fu, V3* fv) {
  Grid g;
  for (int s = 0; s < 16; ++s) g.p[s] = P.cp[s];
  double lu[4] = {0, 0, 0, 0}, lv[4] = {0, 0, 0, 0};  // d(lambda)/du, d(lambda)/dv
  if (P.gregory) {
    for (int k = 0; k < 4; ++k) {
      double du = inner_first_u(k) ? u : 1.0 - u;
      double dv = inner_first_v(k) ? v : 1.0 - v;
      double den = du + dv;
      V3 pu = P.cp[kInner[k]], pv = P.cp[kInnerV[k]];
      if (den > 0.0) {
        double lam = du / den;
        g.p[kInner[k]] = lam * pu + (1.0 - lam) * pv;
        double sdu = inner_first_u(k) ? 1.0 : -1.0, sdv = inner_first_v(k) ? 1.0 : -1.0;
        lu[k] = sdu * dv / (den * den);
        lv[k] = -sdv * du / (den * den);
      } else {
        g.p[kInner[k]] = 0.5 * (pu + pv);
      }
    }
  }
  V3 a, b, c;
  bezier_eval(g, u, v, &a, &b, &c, nullptr);
  if (P.gregory) {
    double bu[4], bv[4];
    bernstein(u, bu);
    bernstein(v, bv);
    for (int k = 0; k < 4; ++k) {
      int i = inner_first_u(k) ? 1 : 2, j = inner_first_v(k) ? 1 : 2;
      V3 diff = P.cp[kInner[k]] - P.cp[kInnerV[k]];
      b = b + (bu[i] * bv[j] * lu[k]) * diff;
      c = c + (bu[i] * bv[j] * lv[k]) * diff;
    }
  }
  if (f) *f = a;
  if (fu) *fu = b;
  if (fv) *fv = c;
}

// --------------------------------------------------------- de Casteljau, crop
// Split four points of a cubic at parameter t into the two halves.
static void casteljau(const V3 in[4], double t, V3 left[4], V3 right[4]) {
  double s = 1.0 - t;
  V3 ab = s * in[0] + t * in[1];
  V3 bc = s * in[1] + t * in[2];
  V3 cd = s * in[2] + t * in[3];
  V3 abc = s * ab + t * bc;
  V3 bcd = s * bc + t * cd;
  V3 abcd = s * abc + t * bcd;
  left[0] = in[0]; left[1] = ab; left[2] = abc; left[3] = abcd;
  right[0] = abcd; right[1] = bcd; right[2] = cd; right[3] = in[3];
}

static inline int slot(int i, int j) { return 4 * j + i; }

static void gather(const Grid& g, int axis, int line, V3 out[4]) {
  for (int k = 0; k < 4; ++k) out[k] = axis == 0 ? g.p[slot(k, line)] : g.p[slot(line, k)];
}
static void scatter(Grid& g, int axis, int line, const V3 in[4]) {
  for (int k = 0; k < 4; ++k) (axis == 0 ? g.p[slot(k, line)] : g.p[slot(line, k)]) = in[k];
}

// Halves of a grid split at parameter 1/2 along axis (0: u, 1: v).
static void split_half(const Grid& g, int axis, Grid* L, Grid* R) {
  for (int line = 0; line < 4; ++line) {
    V3 in[4], l[4], r[4];
    gather(g, axis, line, in);
    casteljau(in, 0.5, l, r);
    scatter(*L, axis, line, l);
    scatter(*R, axis, line, r);
  }
}

// Restriction of a cubic to [t0, t1] by two de Casteljau subdivisions.
static void crop1(const V3 in[4], double t0, double t1, V3 out[4]) {
  V3 cur[4], l[4], r[4];
  for (int k = 0; k < 4; ++k) cur[k] = in[k];
  if (t1 < 1.0) {
    casteljau(cur, t1, l, r);
    for (int k = 0; k < 4; ++k) cur[k] = l[k];
  }
  if (t0 > 0.0) {
    casteljau(cur, t0 / t1, l, r);
    for (int k = 0; k < 4; ++k) cur[k] = r[k];
  }
  for (int k = 0; k < 4; ++k) out[k] = cur[k];
}

// Control points of the patch restricted to [u0,u1] x [v0,v1], cropping one
// parametric direction after the other (the route Sec. 2.1 calls mathematically
// equivalent to Alg. 1).
static Grid crop(const Grid& g, double u0, double u1, double v0, double v1) {
  Grid a = g, b;
  for (int line = 0; line < 4; ++line) {
    V3 in[4], out[4];
    gather(a, 0, line, in);
    crop1(in, u0, u1, out);
    scatter(b, 0, line, out);
  }
  for (int line = 0; line < 4; ++line) {
    V3 in[4], out[4];
    gather(b, 1, line, in);
    crop1(in, v0, v1, out);
    scatter(a, 1, line, out);
  }
  return a;
}

// ----------------------------------------------------------- Gregory bounds
// Maximum of the Bernstein weight B_1 (k = 1) or B_2 (k = 2) of degree 3 over
// [t0, t1]: the weight at the peak (1/3 resp. 2/3) clamped into the interval (Alg. 2).
static double wbar(int k, double t0, double t1) {
  double peak = k == 1 ? 1.0 / 3.0 : 2.0 / 3.0;
  double t = std::min(std::max(peak, t0), t1);
  return k == 1 ? 3.0 * t * (1.0 - t) * (1.0 - t) : 3.0 * t * t * (1.0 - t);
}

struct Bound {
  Grid q;  // lower bounding Bezier patch restricted to the domain
  V3 d;    // displacement of the upper bound
};

// Extreme blends of inner point k over a domain: A at the smallest weight on
// P^u, B at the largest (Sec. 2.2, weight bounds; Alg. 2).
static void inner_extremes(const Patch& P, int k, double u0, double u1, double v0, double v1,
                           V3* A, V3* B) {
  double dul = inner_first_u(k) ? u0 : 1.0 - u1, duh = inner_first_u(k) ? u1 : 1.0 - u0;
  double dvl = inner_first_v(k) ? v0 : 1.0 - v1, dvh = inner_first_v(k) ? v1 : 1.0 - v0;
  V3 pu = P.cp[kInner[k]], pv = P.cp[kInnerV[k]];
  // (a P^u + b P^v) / (a + b) written as P^v + a/(a+b) (P^u - P^v): the same
  // value, exact when the pair coincides (a Bezier patch as a Gregory patch)
  double lam_lo = dul / (dul + dvh), lam_hi = duh / (duh + dvl);
  *A = pv + lam_lo * (pu - pv);
  *B = pv + lam_hi * (pu - pv);
}

// calcPointsAndD (Alg. 2): the lower bounding Bezier patch restricted to D and
// the displacement d(D) = sum_ij wbar_i(u-range) wbar_j(v-range) |A_ij - B_ij|.
// A Bezier patch returns its own restriction and d = 0.
static Bound calc_points_and_d(const Patch& P, double u0, double u1, double v0, double v1) {
  Grid g;
  for (int s = 0; s < 16; ++s) g.p[s] = P.cp[s];
  V3 d = {0, 0, 0};
  if (P.gregory) {
    for (int k = 0; k < 4; ++k) {
      V3 A, B;
      inner_extremes(P, k, u0, u1, v0, v1, &A, &B);
      g.p[kInner[k]] = vmin(A, B);
      int i = inner_first_u(k) ? 1 : 2, j = inner_first_v(k) ? 1 : 2;
      d = d + (wbar(i, u0, u1) * wbar(j, v0, v1)) * vabs(A - B);
    }
  }
  Bound b;
  b.q = crop(g, u0, u1, v0, v1);
  b.d = d;
  return b;
}

static Bound calc_points_and_d_int(const Patch& P, uint32_t pu, uint32_t pv, uint32_t su, uint32_t sv) {
  return calc_points_and_d(P, pu * kUnit, (pu + su) * kUnit, pv * kUnit, (pv + sv) * kUnit);
}

static void grid_box(const Grid& g, V3 d, double pad, V3* lo, V3* hi) {
  V3 a = g.p[0], b = g.p[0];
  for (int s = 1; s < 16; ++s) {
    a = vmin(a, g.p[s]);
    b = vmax(b, g.p[s]);
  }
  const V3 e = {pad, pad, pad};
  *lo = a - e;
  *hi = (b + d) + e;
}

// ------------------------------------------------------------------ slab test
// Closed slab test on [tmin, cap]; a zero direction component keeps the slab
// unbounded when the origin lies between the planes and misses otherwise.
static bool slab(const Ray& r, V3 lo, V3 hi, double cap, double* entry) {
  double near = r.tmin, far = cap;
  for (int a = 0; a < 3; ++a) {
    double o = at(r.o, a), d = at(r.d, a), l = at(lo, a), h = at(hi, a);
    if (d == 0.0) {
      if (o < l || o > h) return false;
      continue;
    }
    double t0 = (l - o) / d, t1 = (h - o) / d;
    near = std::max(near, std::min(t0, t1));
    far = std::min(far, std::max(t0, t1));
  }
  if (!(near <= far)) return false;
  *entry = near;
  return true;
}

static bool ray_valid(const Ray& r) {
  double v[8] = {r.o.x, r.o.y, r.o.z, r.d.x, r.d.y, r.d.z, r.tmin, r.tmax};
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(v[k])) return false;
  if (std::isnan(r.tmin) || std::isnan(r.tmax)) return false;
  if (r.d.x == 0.0 && r.d.y == 0.0 && r.d.z == 0.0) return false;
  return r.tmin <= r.tmax;
}

static inline bool better(double t, uint32_t id, const Best& b) {
  return t < b.t || (t == b.t && id < b.id);
}

// ---------------------------------------------------- per-patch subdivision
struct Split {
  uint32_t pu, pv, su, sv;
};

// Orders other than closest-first, for measurement only (what a learned child order
// could save at best); wherever both halves of a split are hit and they are not the
// leaf pair:
//   kHindsight: on the patch of the ray's known closest hit (id, leaf corner pu, pv
//               in units of 2^-23), the half holding that leaf is visited first: the
//               order a perfect predictor of the final leaf gives;
//   kLookahead: on every patch, the half whose first visit costs fewer split steps
//               over the node's subtree (both orders tried, closest-first below):
//               the order a perfect predictor of that work label gives.
//   kSingleBox: not an order but the alternative Sec. 3.3 measures its two-box test
//               against: every node tests only its own box (its grid bounded on its
//               own domain by Alg. 2, with its own displacement); a hit node above
//               the leaf depth has both halves visited, the lower one first, and a
//               hit leaf is recorded at its own entry distance.
//   kRetest:    closest-first, and a pending sibling is skipped when it is resumed if its
//               box (tested when its parent was split) is entered beyond the best distance
//               found since (Alg. 3 does not re-test it; measurement of what that would save).
enum OrderMode { kHindsight = 0, kLookahead = 1, kSingleBox = 2, kRetest = 3 };
struct OrderHint {
  int mode;
  uint32_t id, pu, pv;
};

// One patch against one ray: depth-first closest-first traversal of the binary
// tree of subdomains, processed with an explicit stack (Sec. 3.3, Alg. 3).
//   * each visited node splits its grid at 1/2 along its axis and tests both
//     child boxes with the current best distance as cap;
//   * the closer child that was hit is visited first (ties: the lower half);
//   * when the children are leaves, the first of them is recorded if closer
//     than the best hit so far; its sibling cannot be closer (Sec. 3.3);
//   * the second child is visited after the first one's subtree without being
//     re-tested, as Alg. 3 resumes it from the bit trail;
//   * a Gregory node's grid and displacement are recomputed for its own domain
//     (Alg. 3 recomputes at every Gregory step); a Bezier child takes the split half.
struct Frame {
  uint32_t pu, pv, su, sv;
  int axis, depth;
  bool second;
  double entry;  // entry distance of the frame's box, tested when its parent was split
  Grid g;
  V3 d;
};

static void run_frames(const Patch& P, uint32_t id, const Ray& r, int L, Best& best, Counters& c,
                       std::vector<Split>* trace, const OrderHint* hint, std::vector<Frame>& stack);

// The two children of frame f (first = ch[0]) in the order first_r gives; the first
// one gets its Gregory grid (the recompute of Alg. 3), the second is pushed for later.
static void push_children(const Patch& P, const Frame& f, const Grid& gl, const Grid& gr, bool hl, bool hr,
                          bool first_r, uint32_t rpu, uint32_t rpv, uint32_t csu, uint32_t csv, double tl, double tr,
                          Counters& c, std::vector<Frame>& stack) {
  Frame ch[2];
  for (int k = 0; k < 2; ++k) {
    bool is_r = (k == 0) ? first_r : !first_r;
    Frame& n = ch[k];
    n.pu = is_r ? rpu : f.pu;
    n.pv = is_r ? rpv : f.pv;
    n.su = csu;
    n.sv = csv;
    n.axis = 1 - f.axis;
    n.depth = f.depth + 1;
    n.second = (k == 1);
    n.entry = is_r ? tr : tl;
    n.g = is_r ? gr : gl;
    n.d = {0, 0, 0};
  }
  if (hl && hr) stack.push_back(ch[1]);
  if (P.gregory) {  // the chosen child gets its own lower grid and displacement
    Bound b = calc_points_and_d_int(P, ch[0].pu, ch[0].pv, ch[0].su, ch[0].sv);
    c.greg++;
    ch[0].g = b.q;
    ch[0].d = b.d;
  }
  stack.push_back(ch[0]);
}

static void intersect_patch_single_box(const Patch& P, uint32_t id, const Ray& r, int L, Best& best,
                                       Counters& c) {
  struct Dom {
    uint32_t pu, pv, su, sv;
    int depth;
  };
  std::vector<Dom> stack;
  stack.reserve(2 * L + 2);
  stack.push_back({0, 0, kFull, kFull, 0});
  while (!stack.empty()) {
    const Dom f = stack.back();
    stack.pop_back();
    const Bound b = calc_points_and_d_int(P, f.pu, f.pv, f.su, f.sv);  // a Bezier patch: its crop, d = 0
    c.split++;
    V3 lo, hi;
    grid_box(b.q, b.d, P.pad, &lo, &hi);
    double t = 0.0;
    if (!slab(r, lo, hi, best.t, &t)) continue;
    if (f.depth == 2 * L) {
      if (better(t, id, best)) {
        best.t = t;
        best.id = id;
        best.u = (f.pu + f.su / 2) * kUnit;
        best.v = (f.pv + f.sv / 2) * kUnit;
        c.leaf++;
      }
      continue;
    }
    const int axis = f.depth & 1;
    const uint32_t csu = axis == 0 ? f.su / 2 : f.su, csv = axis == 1 ? f.sv / 2 : f.sv;
    stack.push_back({axis == 0 ? f.pu + csu : f.pu, axis == 1 ? f.pv + csv : f.pv, csu, csv, f.depth + 1});
    stack.push_back({f.pu, f.pv, csu, csv, f.depth + 1});  // the lower half first
  }
}

static void intersect_patch(const Patch& P, uint32_t id, const Ray& r, int L, Best& best,
                            Counters& c, std::vector<Split>* trace, const OrderHint* hint = nullptr) {
  if (hint && hint->mode == kSingleBox) {
    intersect_patch_single_box(P, id, r, L, best, c);
    return;
  }
  std::vector<Frame> stack;
  stack.reserve(4 * L + 4);  // at most one pending sibling per level
  Frame root;
  root.pu = root.pv = 0;
  root.su = root.sv = kFull;
  root.axis = 0;
  root.depth = 0;
  root.second = false;
  root.entry = 0.0;
  if (P.gregory) {
    Bound b = calc_points_and_d_int(P, 0, 0, kFull, kFull);
    c.greg++;
    root.g = b.q;
    root.d = b.d;
  } else {
    for (int s = 0; s < 16; ++s) root.g.p[s] = P.cp[s];
    root.d = {0, 0, 0};
  }
  stack.push_back(root);
  run_frames(P, id, r, L, best, c, trace, hint, stack);
}

static void run_frames(const Patch& P, uint32_t id, const Ray& r, int L, Best& best, Counters& c,
                       std::vector<Split>* trace, const OrderHint* hint, std::vector<Frame>& stack) {
  const int leaf_depth = 2 * L;
  while (!stack.empty()) {
    Frame f = stack.back();
    stack.pop_back();
    if (f.second && hint && hint->mode == kRetest && f.entry > best.t) continue;  // behind the best hit
    if (f.second) {
      c.backtrack++;
      if (!P.gregory) c.crop++;  // Alg. 3 re-crops a Bezier grid after backtracking
      if (P.gregory) {
        Bound b = calc_points_and_d_int(P, f.pu, f.pv, f.su, f.sv);
        c.greg++;
        f.g = b.q;
        f.d = b.d;
      }
    }
    c.split++;
    if (trace) trace->push_back({f.pu, f.pv, f.su, f.sv});
    Grid gl, gr;
    split_half(f.g, f.axis, &gl, &gr);
    V3 lol, hil, lor, hir;
    grid_box(gl, f.d, P.pad, &lol, &hil);
    grid_box(gr, f.d, P.pad, &lor, &hir);
    double tl = 0, tr = 0;
    bool hl = slab(r, lol, hil, best.t, &tl);
    bool hr = slab(r, lor, hir, best.t, &tr);
    if (!hl && !hr) continue;
    uint32_t csu = f.axis == 0 ? f.su / 2 : f.su, csv = f.axis == 1 ? f.sv / 2 : f.sv;
    uint32_t rpu = f.axis == 0 ? f.pu + csu : f.pu, rpv = f.axis == 1 ? f.pv + csv : f.pv;
    bool first_r = hr && (!hl || tr < tl);
    if (hint && hint->mode == kHindsight && hint->id == id && hl && hr && f.depth + 1 != leaf_depth)
      first_r = f.axis == 0 ? hint->pu >= rpu : hint->pv >= rpv;
    if (hint && hint->mode == kLookahead && hl && hr && f.depth + 1 != leaf_depth) {
      uint32_t steps[2];
      for (int o = 0; o < 2; ++o) {  // o = 0: closest first; o = 1: the other half first
        std::vector<Frame> sub;
        Best b2 = best;
        Counters c2 = {0, 0, 0, 0, 0, 0, 0, 0};
        push_children(P, f, gl, gr, hl, hr, o == 0 ? first_r : !first_r, rpu, rpv, csu, csv, tl, tr, c2, sub);
        run_frames(P, id, r, L, b2, c2, nullptr, nullptr, sub);
        steps[o] = c2.split;
      }
      if (steps[1] < steps[0]) first_r = !first_r;
    }
    if (f.depth + 1 == leaf_depth) {
      double t = first_r ? tr : tl;
      if (better(t, id, best)) {
        uint32_t lpu = first_r ? rpu : f.pu, lpv = first_r ? rpv : f.pv;
        best.t = t;
        best.id = id;
        best.u = (lpu + csu / 2) * kUnit;
        best.v = (lpv + csv / 2) * kUnit;
        c.leaf++;
      }
      continue;
    }
    push_children(P, f, gl, gr, hl, hr, first_r, rpu, rpv, csu, csv, tl, tr, c, stack);
  }
}

// ------------------------------------------------------------------- scene/BVH
struct Node {
  V3 lo, hi;
  int32_t left, right;  // children, or -1
  uint32_t first, count;  // leaf range into order[]
};

// Patch-local frame (Sec. 3.4: intersecting in local frames tightens the boxes):
// rows r0 = unit(p30 - p00), r1 = unit of (p03 - p00) with its r0 part removed,
// r2 = r0 x r1; the identity for a patch whose u or v edge is degenerate.  A
// point x maps to (r0.x, r1.x, r2.x), applied to both patch and ray, so ray
// parameters are unchanged and only the boxes (now in the patch's frame) differ.
struct Frame3 {
  V3 r0, r1, r2;
};

struct Scene {
  std::vector<Patch> patches;
  std::vector<Node> nodes;
  std::vector<uint32_t> order;
  int L;
  bool use_bvh;
  bool local = false;               // subdivide each patch in its local frame
  std::vector<Frame3> frames;       // per patch, when local
  std::vector<Patch> local_patches;  // patches mapped into their frames, when local
};

static Frame3 local_frame(const Patch& P) {
  const Frame3 id = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  V3 eu = P.cp[3] - P.cp[0], ev = P.cp[12] - P.cp[0];
  double lu = std::sqrt(dot(eu, eu)), lv = std::sqrt(dot(ev, ev));
  if (!(lu > 0.0) || !(lv > 0.0)) return id;
  V3 r0 = (1.0 / lu) * eu;
  V3 w = ev - dot(ev, r0) * r0;
  double lw = std::sqrt(dot(w, w));
  if (!(lw > 1e-9 * lv)) return id;
  V3 r1 = (1.0 / lw) * w;
  return {r0, r1, cross(r0, r1)};
}

static inline V3 to_frame(const Frame3& F, V3 x) { return {dot(F.r0, x), dot(F.r1, x), dot(F.r2, x)}; }

// The patch and ray that subdivision works on: world ones, or both in the patch's frame.
static inline const Patch& work_patch(const Scene& S, uint32_t k) {
  return S.local ? S.local_patches[k] : S.patches[k];
}
static inline Ray work_ray(const Scene& S, uint32_t k, const Ray& r) {
  if (!S.local) return r;
  const Frame3& F = S.frames[k];
  return {to_frame(F, r.o), to_frame(F, r.d), r.tmin, r.tmax};
}

static void load_patch(Patch& P, const float* cp, uint8_t type) {
  P.gregory = type == 1;
  for (int s = 0; s < 20; ++s) P.cp[s] = {cp[3 * s], cp[3 * s + 1], cp[3 * s + 2]};
  int n = P.gregory ? 20 : 16;
  P.lo = P.hi = P.cp[0];
  for (int s = 1; s < n; ++s) {
    P.lo = vmin(P.lo, P.cp[s]);
    P.hi = vmax(P.hi, P.cp[s]);
  }
}

// Median-split BVH over patch boxes (independent of the library's binned SAH).
static int build_node(Scene& S, uint32_t first, uint32_t count) {
  Node n;
  n.lo = S.patches[S.order[first]].lo;
  n.hi = S.patches[S.order[first]].hi;
  V3 clo = 0.5 * (n.lo + n.hi), chi = clo;
  for (uint32_t k = first; k < first + count; ++k) {
    const Patch& P = S.patches[S.order[k]];
    n.lo = vmin(n.lo, P.lo);
    n.hi = vmax(n.hi, P.hi);
    V3 c = 0.5 * (P.lo + P.hi);
    clo = vmin(clo, c);
    chi = vmax(chi, c);
  }
  n.left = n.right = -1;
  n.first = first;
  n.count = count;
  int idx = (int)S.nodes.size();
  S.nodes.push_back(n);
  if (count <= 4) return idx;
  V3 ext = chi - clo;
  int axis = (ext.x >= ext.y && ext.x >= ext.z) ? 0 : (ext.y >= ext.z ? 1 : 2);
  uint32_t mid = first + count / 2;
  std::nth_element(S.order.begin() + first, S.order.begin() + mid, S.order.begin() + first + count,
                   [&](uint32_t a, uint32_t b) {
                     double ca = at(S.patches[a].lo, axis) + at(S.patches[a].hi, axis);
                     double cb = at(S.patches[b].lo, axis) + at(S.patches[b].hi, axis);
                     return ca < cb || (ca == cb && a < b);
                   });
  int l = build_node(S, first, mid - first);
  int r = build_node(S, mid, first + count - mid);
  S.nodes[idx].left = l;
  S.nodes[idx].right = r;
  return idx;
}

static void trace_ray(const Scene& S, const Ray& r, Best& best, Counters& c, const OrderHint* hint = nullptr) {
  best.t = r.tmax;
  best.id = kNoHit;
  best.u = best.v = 0.0;
  if (!ray_valid(r)) return;
  if (!S.use_bvh) {
    for (uint32_t k = 0; k < S.patches.size(); ++k) {
      double e;
      if (!slab(r, S.patches[k].lo, S.patches[k].hi, best.t, &e)) continue;
      c.cand++;
      c.cand_greg += S.patches[k].gregory;
      intersect_patch(work_patch(S, k), k, work_ray(S, k, r), S.L, best, c, nullptr, hint);
    }
    return;
  }
  double e;
  if (S.nodes.empty() || !slab(r, S.nodes[0].lo, S.nodes[0].hi, best.t, &e)) return;
  std::vector<int> stack;
  stack.push_back(0);
  while (!stack.empty()) {
    const Node& n = S.nodes[stack.back()];
    stack.pop_back();
    c.node++;
    if (n.left < 0) {
      for (uint32_t k = n.first; k < n.first + n.count; ++k) {
        uint32_t id = S.order[k];
        if (!slab(r, S.patches[id].lo, S.patches[id].hi, best.t, &e)) continue;
        c.cand++;
        c.cand_greg += S.patches[id].gregory;
        intersect_patch(work_patch(S, id), id, work_ray(S, id, r), S.L, best, c, nullptr, hint);
      }
      continue;
    }
    double tl = 0, tr = 0;
    bool hl = slab(r, S.nodes[n.left].lo, S.nodes[n.left].hi, best.t, &tl);
    bool hr = slab(r, S.nodes[n.right].lo, S.nodes[n.right].hi, best.t, &tr);
    if (hl && hr) {
      if (tr < tl) {
        stack.push_back(n.left);
        stack.push_back(n.right);
      } else {
        stack.push_back(n.right);
        stack.push_back(n.left);
      }
    } else if (hl) {
      stack.push_back(n.left);
    } else if (hr) {
      stack.push_back(n.right);
    }
  }
}

static Ray load_ray(const float* r8) {
  Ray r;
  r.o = {r8[0], r8[1], r8[2]};
  r.tmin = r8[3];
  r.d = {r8[4], r8[5], r8[6]};
  r.tmax = r8[7];
  return r;
}

template <class F>
static void parallel_for(uint32_t n, int nthreads, F fn) {
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  std::atomic<uint32_t> next(0);
  const uint32_t chunk = 256;
  auto work = [&]() {
    for (;;) {
      uint32_t b = next.fetch_add(chunk);
      if (b >= n) break;
      uint32_t e = std::min(n, b + chunk);
      for (uint32_t i = b; i < e; ++i) fn(i);
    }
  };
  if (nthreads == 1) {
    work();
    return;
  }
  std::vector<std::thread> th;
  for (int k = 0; k < nthreads; ++k) th.emplace_back(work);
  for (auto& t : th) t.join();
}

// ------------------------------------------------------- brute-force reference
// Dense tessellation of every candidate patch into res x res cells (two
// triangles each) with a min/max pyramid for pruning, intersected with the
// watertight ray/triangle test of Woop, Benthin and Wald (2013) in double.
struct Tess {
  int res;
  std::vector<V3> pts;  // (res+1)^2
  std::vector<std::vector<V3>> lo, hi;  // levels: 0 = cells, then halved
};

static void tessellate(const Patch& P, int res, Tess& T) {
  T.res = res;
  T.pts.resize((size_t)(res + 1) * (res + 1));
  for (int y = 0; y <= res; ++y)
    for (int x = 0; x <= res; ++x) patch_eval(P, (double)x / res, (double)y / res, &T.pts[y * (res + 1) + x], nullptr, nullptr);
  T.lo.clear();
  T.hi.clear();
  int n = res;
  std::vector<V3> lo((size_t)n * n), hi((size_t)n * n);
  for (int y = 0; y < n; ++y)
    for (int x = 0; x < n; ++x) {
      V3 a = T.pts[y * (res + 1) + x], b = T.pts[y * (res + 1) + x + 1];
      V3 c = T.pts[(y + 1) * (res + 1) + x], d = T.pts[(y + 1) * (res + 1) + x + 1];
      lo[y * n + x] = vmin(vmin(a, b), vmin(c, d));
      hi[y * n + x] = vmax(vmax(a, b), vmax(c, d));
    }
  T.lo.push_back(lo);
  T.hi.push_back(hi);
  while (n > 1) {
    int m = n / 2;
    std::vector<V3> l2((size_t)m * m), h2((size_t)m * m);
    const auto& l1 = T.lo.back();
    const auto& h1 = T.hi.back();
    for (int y = 0; y < m; ++y)
      for (int x = 0; x < m; ++x) {
        V3 a = l1[(2 * y) * n + 2 * x], b = h1[(2 * y) * n + 2 * x];
        for (int k = 1; k < 4; ++k) {
          int yy = 2 * y + (k >> 1), xx = 2 * x + (k & 1);
          a = vmin(a, l1[yy * n + xx]);
          b = vmax(b, h1[yy * n + xx]);
        }
        l2[y * m + x] = a;
        h2[y * m + x] = b;
      }
    T.lo.push_back(l2);
    T.hi.push_back(h2);
    n = m;
  }
}

struct TriHit {
  double t, b0, b1, b2;
};

static bool watertight_tri(const Ray& r, V3 a, V3 b, V3 c, double cap, TriHit* h) {
  double dx = std::fabs(r.d.x), dy = std::fabs(r.d.y), dz = std::fabs(r.d.z);
  int kz = (dx >= dy && dx >= dz) ? 0 : (dy >= dz ? 1 : 2);
  int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
  if (at(r.d, kz) < 0) std::swap(kx, ky);
  double Sx = at(r.d, kx) / at(r.d, kz), Sy = at(r.d, ky) / at(r.d, kz), Sz = 1.0 / at(r.d, kz);
  V3 A = a - r.o, B = b - r.o, C = c - r.o;
  double Ax = at(A, kx) - Sx * at(A, kz), Ay = at(A, ky) - Sy * at(A, kz);
  double Bx = at(B, kx) - Sx * at(B, kz), By = at(B, ky) - Sy * at(B, kz);
  double Cx = at(C, kx) - Sx * at(C, kz), Cy = at(C, ky) - Sy * at(C, kz);
  double U = Cx * By - Cy * Bx, V = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
  if ((U < 0 || V < 0 || W < 0) && (U > 0 || V > 0 || W > 0)) return false;
  double det = U + V + W;
  if (det == 0.0) return false;
  double Az = Sz * at(A, kz), Bz = Sz * at(B, kz), Cz = Sz * at(C, kz);
  double T = U * Az + V * Bz + W * Cz;
  double t = T / det;
  if (!(t >= r.tmin && t <= cap)) return false;
  h->t = t;
  h->b0 = U / det;
  h->b1 = V / det;
  h->b2 = W / det;
  return true;
}

static bool brute_patch(const Tess& T, const Ray& r, double& best_t, double& bu, double& bv) {
  bool found = false;
  int top = (int)T.lo.size() - 1;
  struct Item { int lvl, x, y; };
  std::vector<Item> st;
  st.push_back({top, 0, 0});
  const int res = T.res;
  while (!st.empty()) {
    Item it = st.back();
    st.pop_back();
    int n = res >> it.lvl;
    double e;
    if (!slab(r, T.lo[it.lvl][it.y * n + it.x], T.hi[it.lvl][it.y * n + it.x], best_t, &e)) continue;
    if (it.lvl > 0) {
      for (int k = 0; k < 4; ++k) st.push_back({it.lvl - 1, 2 * it.x + (k & 1), 2 * it.y + (k >> 1)});
      continue;
    }
    int x = it.x, y = it.y;
    V3 p00 = T.pts[y * (res + 1) + x], p10 = T.pts[y * (res + 1) + x + 1];
    V3 p01 = T.pts[(y + 1) * (res + 1) + x], p11 = T.pts[(y + 1) * (res + 1) + x + 1];
    double u0 = (double)x / res, u1 = (double)(x + 1) / res, v0 = (double)y / res, v1 = (double)(y + 1) / res;
    TriHit h;
    if (watertight_tri(r, p00, p10, p11, best_t, &h)) {
      best_t = h.t;
      bu = h.b0 * u0 + h.b1 * u1 + h.b2 * u1;
      bv = h.b0 * v0 + h.b1 * v0 + h.b2 * v1;
      found = true;
    }
    if (watertight_tri(r, p00, p11, p01, best_t, &h)) {
      best_t = h.t;
      bu = h.b0 * u0 + h.b1 * u1 + h.b2 * u0;
      bv = h.b0 * v0 + h.b1 * v1 + h.b2 * v1;
      found = true;
    }
  }
  return found;
}

// ---------------------------------------------------------- secondary rays
// Orthonormal tangents for a unit normal (Duff et al. 2017).
static void onb(V3 n, V3* t, V3* b) {
  double sign = n.z >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sign + n.z);
  double bb = n.x * n.y * a;
  *t = {1.0 + sign * n.x * n.x * a, sign * bb, -sign * n.x};
  *b = {bb, sign + n.y * n.y * a, -n.y};
}

}  // namespace orc

using namespace orc;

extern "C" {

// ---- patch math (inputs: 20 x 3 doubles, slot order above) ----
void orc_patch_eval(const double* cp, int gregory, double u, double v, double* f, double* fu, double* fv) {
  Patch P;
  for (int s = 0; s < 20; ++s) P.cp[s] = {cp[3 * s], cp[3 * s + 1], cp[3 * s + 2]};
  P.gregory = gregory != 0;
  V3 a, b, c;
  patch_eval(P, u, v, &a, &b, &c);
  if (f) { f[0] = a.x; f[1] = a.y; f[2] = a.z; }
  if (fu) { fu[0] = b.x; fu[1] = b.y; fu[2] = b.z; }
  if (fv) { fv[0] = c.x; fv[1] = c.y; fv[2] = c.z; }
}

void orc_bezier_eval(const double* grid, double u, double v, double* out12) {
  Grid g;
  for (int s = 0; s < 16; ++s) g.p[s] = {grid[3 * s], grid[3 * s + 1], grid[3 * s + 2]};
  V3 r[4];
  bezier_eval(g, u, v, &r[0], &r[1], &r[2], &r[3]);
  for (int k = 0; k < 4; ++k) {
    out12[3 * k] = r[k].x;
    out12[3 * k + 1] = r[k].y;
    out12[3 * k + 2] = r[k].z;
  }
}

void orc_split(const double* grid, int axis, double* left, double* right) {
  Grid g, L, R;
  for (int s = 0; s < 16; ++s) g.p[s] = {grid[3 * s], grid[3 * s + 1], grid[3 * s + 2]};
  split_half(g, axis, &L, &R);
  for (int s = 0; s < 16; ++s) {
    left[3 * s] = L.p[s].x; left[3 * s + 1] = L.p[s].y; left[3 * s + 2] = L.p[s].z;
    right[3 * s] = R.p[s].x; right[3 * s + 1] = R.p[s].y; right[3 * s + 2] = R.p[s].z;
  }
}

void orc_crop(const double* grid, double u0, double u1, double v0, double v1, double* out) {
  Grid g;
  for (int s = 0; s < 16; ++s) g.p[s] = {grid[3 * s], grid[3 * s + 1], grid[3 * s + 2]};
  Grid q = crop(g, u0, u1, v0, v1);
  for (int s = 0; s < 16; ++s) {
    out[3 * s] = q.p[s].x; out[3 * s + 1] = q.p[s].y; out[3 * s + 2] = q.p[s].z;
  }
}

double orc_wbar(int k, double t0, double t1) { return wbar(k, t0, t1); }

void orc_inner_extremes(const double* cp, double u0, double u1, double v0, double v1, double* A12, double* B12) {
  Patch P;
  for (int s = 0; s < 20; ++s) P.cp[s] = {cp[3 * s], cp[3 * s + 1], cp[3 * s + 2]};
  P.gregory = true;
  for (int k = 0; k < 4; ++k) {
    V3 A, B;
    inner_extremes(P, k, u0, u1, v0, v1, &A, &B);
    A12[3 * k] = A.x; A12[3 * k + 1] = A.y; A12[3 * k + 2] = A.z;
    B12[3 * k] = B.x; B12[3 * k + 1] = B.y; B12[3 * k + 2] = B.z;
  }
}

void orc_calc_points_and_d(const double* cp, int gregory, double u0, double u1, double v0, double v1,
                           double* q, double* d) {
  Patch P;
  for (int s = 0; s < 20; ++s) P.cp[s] = {cp[3 * s], cp[3 * s + 1], cp[3 * s + 2]};
  P.gregory = gregory != 0;
  Bound b = calc_points_and_d(P, u0, u1, v0, v1);
  for (int s = 0; s < 16; ++s) {
    q[3 * s] = b.q.p[s].x; q[3 * s + 1] = b.q.p[s].y; q[3 * s + 2] = b.q.p[s].z;
  }
  d[0] = b.d.x; d[1] = b.d.y; d[2] = b.d.z;
}

// ---- scenes ----
// Rows of patch k's local frame (9 doubles; the identity when the scene is not local).
void orc_patch_frame(void* s, uint32_t k, double* rows9) {
  const Scene& S = *(Scene*)s;
  Frame3 F = S.local ? S.frames[k] : Frame3{{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const V3 r[3] = {F.r0, F.r1, F.r2};
  for (int a = 0; a < 3; ++a) {
    rows9[3 * a] = r[a].x;
    rows9[3 * a + 1] = r[a].y;
    rows9[3 * a + 2] = r[a].z;
  }
}

// flags bit 0: subdivide in patch-local frames.
void* orc_scene_create(const float* cp, const uint8_t* types, uint32_t n, int L, int use_bvh, int flags) {
  Scene* S = new Scene();
  S->L = L;
  S->use_bvh = use_bvh != 0;
  S->local = (flags & 1) != 0;
  S->patches.resize(n);
  for (uint32_t k = 0; k < n; ++k) load_patch(S->patches[k], cp + 60 * (size_t)k, types[k]);
  if (S->local) {
    S->frames.resize(n);
    S->local_patches.resize(n);
    for (uint32_t k = 0; k < n; ++k) {
      const Patch& P = S->patches[k];
      const Frame3 F = local_frame(P);
      Patch Q = P;
      for (int sl = 0; sl < 20; ++sl) Q.cp[sl] = to_frame(F, P.cp[sl]);
      const int m = Q.gregory ? 20 : 16;
      Q.lo = Q.hi = Q.cp[0];
      for (int sl = 1; sl < m; ++sl) {
        Q.lo = vmin(Q.lo, Q.cp[sl]);
        Q.hi = vmax(Q.hi, Q.cp[sl]);
      }
      // Sec. 3.4: in a patch's own frame, corners and straight edges lie on box faces
      // shared with neighbouring patches, where rounding can open gaps; every box is
      // grown by 2^-19 of the patch's largest extent in its frame to close them
      const V3 ext = Q.hi - Q.lo;
      Q.pad = std::ldexp(std::max(ext.x, std::max(ext.y, ext.z)), -19);
      S->frames[k] = F;
      S->local_patches[k] = Q;
    }
  }
  S->order.resize(n);
  for (uint32_t k = 0; k < n; ++k) S->order[k] = k;
  if (S->use_bvh && n > 0) build_node(*S, 0, n);
  return S;
}

void orc_scene_destroy(void* s) { delete (Scene*)s; }

uint32_t orc_scene_nodes(void* s) { return (uint32_t)((Scene*)s)->nodes.size(); }

// Closest hits of n rays (n x 8 floats: o, tmin, d, tmax).  Outputs per ray: t
// (tmax if no hit), patch id (0xFFFFFFFF if none), u, v and, if counters is
// non-null, eight counters: BVH nodes, candidate patches, split steps,
// backtracks, Gregory bound recomputations, leaf records, Bezier re-crops after
// backtracking, Gregory candidates.
void orc_intersect(void* s, const float* rays, uint32_t n, int nthreads, double* t, uint32_t* id,
                   double* u, double* v, uint32_t* counters) {
  const Scene& S = *(Scene*)s;
  parallel_for(n, nthreads, [&](uint32_t i) {
    Ray r = load_ray(rays + 8 * (size_t)i);
    Best b;
    Counters c = {0, 0, 0, 0, 0, 0, 0, 0};
    trace_ray(S, r, b, c);
    t[i] = b.t;
    id[i] = b.id;
    u[i] = b.u;
    v[i] = b.v;
    if (counters) {
      uint32_t* o = counters + 8 * (size_t)i;
      o[0] = c.node; o[1] = c.cand; o[2] = c.split; o[3] = c.backtrack;
      o[4] = c.greg; o[5] = c.leaf; o[6] = c.crop; o[7] = c.cand_greg;
    }
  });
}

// orc_intersect for rays given in double precision (n x 8 doubles), e.g. rays moved
// off the fp32 grid by the parity gate's graze check.
void orc_intersect_f64(void* s, const double* rays, uint32_t n, int nthreads, double* t, uint32_t* id, double* u,
                       double* v) {
  const Scene& S = *(Scene*)s;
  parallel_for(n, nthreads, [&](uint32_t i) {
    const double* r8 = rays + 8 * (size_t)i;
    Ray r;
    r.o = {r8[0], r8[1], r8[2]};
    r.tmin = r8[3];
    r.d = {r8[4], r8[5], r8[6]};
    r.tmax = r8[7];
    Best b;
    Counters c = {0, 0, 0, 0, 0, 0, 0, 0};
    trace_ray(S, r, b, c);
    t[i] = b.t;
    id[i] = b.id;
    u[i] = b.u;
    v[i] = b.v;
  });
}

// orc_intersect in another child order (OrderHint, measurement of what a learned
// order could save): mode kHindsight with hint_id, hint_u, hint_v a closest hit of
// each ray (0xFFFFFFFF: none), e.g. orc_intersect's own; mode kLookahead ignores the
// hints.
void orc_intersect_hinted(void* s, const float* rays, uint32_t n, int nthreads, int mode, const uint32_t* hint_id,
                          const double* hint_u, const double* hint_v, double* t, uint32_t* id, double* u, double* v,
                          uint32_t* counters) {
  const Scene& S = *(Scene*)s;
  const uint32_t leaf = kFull >> S.L;
  parallel_for(n, nthreads, [&](uint32_t i) {
    Ray r = load_ray(rays + 8 * (size_t)i);
    Best b;
    Counters c = {0, 0, 0, 0, 0, 0, 0, 0};
    OrderHint h;
    h.mode = mode;
    h.id = hint_id[i];
    h.pu = std::min((uint32_t)(hint_u[i] / kUnit) & ~(leaf - 1), kFull - leaf);
    h.pv = std::min((uint32_t)(hint_v[i] / kUnit) & ~(leaf - 1), kFull - leaf);
    trace_ray(S, r, b, c, (mode == kHindsight && h.id == kNoHit) ? nullptr : &h);  // other modes ignore the hint
    t[i] = b.t;
    id[i] = b.id;
    u[i] = b.u;
    v[i] = b.v;
    uint32_t* o = counters + 8 * (size_t)i;
    o[0] = c.node; o[1] = c.cand; o[2] = c.split; o[3] = c.backtrack;
    o[4] = c.greg; o[5] = c.leaf; o[6] = c.crop; o[7] = c.cand_greg;
  });
}

// One ray against one patch with a given initial cap; records the (pos, size)
// of every split step in seq (4 uint32 each, at most max_seq steps) and
// returns the number of steps.  hit4 = (t, id-as-double, u, v).
int orc_trace_patch(void* s, uint32_t patch, const float* ray8, double cap, uint32_t* seq, int max_seq,
                    double* hit4) {
  const Scene& S = *(Scene*)s;
  Ray r = load_ray(ray8);
  Best b = {cap, kNoHit, 0.0, 0.0};
  Counters c = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<Split> tr;
  if (ray_valid(r)) intersect_patch(work_patch(S, patch), patch, work_ray(S, patch, r), S.L, b, c, &tr);
  int n = (int)std::min<size_t>(tr.size(), (size_t)max_seq);
  for (int k = 0; k < n; ++k) {
    seq[4 * k] = tr[k].pu; seq[4 * k + 1] = tr[k].pv; seq[4 * k + 2] = tr[k].su; seq[4 * k + 3] = tr[k].sv;
  }
  hit4[0] = b.t;
  hit4[1] = (double)b.id;
  hit4[2] = b.u;
  hit4[3] = b.v;
  return (int)tr.size();
}

// Brute-force closest hits against res x res tessellations (see above).
void orc_bruteforce(void* s, const float* rays, uint32_t n, int res, int nthreads, double* t, uint32_t* id,
                    double* u, double* v) {
  const Scene& S = *(Scene*)s;
  const uint32_t np = (uint32_t)S.patches.size();
  std::vector<Ray> R(n);
  for (uint32_t i = 0; i < n; ++i) {
    R[i] = load_ray(rays + 8 * (size_t)i);
    t[i] = R[i].tmax;
    id[i] = kNoHit;
    u[i] = v[i] = 0.0;
  }
  // candidate lists per patch
  std::vector<std::vector<uint32_t>> cand(np);
  for (uint32_t i = 0; i < n; ++i) {
    if (!ray_valid(R[i])) continue;
    for (uint32_t k = 0; k < np; ++k) {
      double e;
      if (slab(R[i], S.patches[k].lo, S.patches[k].hi, R[i].tmax, &e)) cand[k].push_back(i);
    }
  }
  int nt = nthreads <= 0 ? (int)std::max(1u, std::thread::hardware_concurrency()) : nthreads;
  std::vector<std::vector<Best>> local(nt, std::vector<Best>());
  std::atomic<uint32_t> next(0);
  auto work = [&](int tid) {
    std::vector<Best>& L = local[tid];
    L.assign(n, Best{0, kNoHit, 0, 0});
    for (uint32_t i = 0; i < n; ++i) L[i].t = R[i].tmax;
    Tess T;
    for (;;) {
      uint32_t k = next.fetch_add(1);
      if (k >= np) break;
      if (cand[k].empty()) continue;
      tessellate(S.patches[k], res, T);
      for (uint32_t i : cand[k]) {
        double bt = R[i].tmax, bu = 0, bv = 0;
        if (brute_patch(T, R[i], bt, bu, bv) && better(bt, k, L[i])) L[i] = Best{bt, k, bu, bv};
      }
    }
  };
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k) th.emplace_back(work, k);
  for (auto& x : th) x.join();
  for (uint32_t i = 0; i < n; ++i) {
    Best b = {R[i].tmax, kNoHit, 0, 0};
    for (int k = 0; k < nt; ++k)
      if (local[k][i].id != kNoHit && better(local[k][i].t, local[k][i].id, b)) b = local[k][i];
    t[i] = b.t;
    id[i] = b.id;
    u[i] = b.u;
    v[i] = b.v;
  }
}

// Secondary rays from hits (the self-intersection offset of Sec. 3.3): origin
// at o + t d, pushed along the unit normal f_u x f_v (turned against d) by the
// L1 size of the box of the leaf domain containing (u, v) (calcPointsAndD on it);
// direction cosine-weighted from two uniforms per ray (Malley's method).  Rays
// without a hit yield an inactive ray (o = 0, d = (0, 0, 1), tmin = 0, tmax = -1).
void orc_bounce(void* s, const float* rays, const float* hits, const float* uniforms, uint32_t n, double* out) {
  const Scene& S = *(Scene*)s;
  const uint32_t leaf = kFull >> S.L;
  for (uint32_t i = 0; i < n; ++i) {
    double* o = out + 8 * (size_t)i;
    uint32_t pid;
    std::memcpy(&pid, hits + 4 * (size_t)i + 1, 4);
    double t = hits[4 * (size_t)i];
    if (pid == kNoHit || pid >= S.patches.size() || !std::isfinite(t)) {
      for (int k = 0; k < 8; ++k) o[k] = 0.0;
      o[6] = 1.0;
      o[7] = -1.0;
      continue;
    }
    Ray r = load_ray(rays + 8 * (size_t)i);
    double hu = hits[4 * (size_t)i + 2], hv = hits[4 * (size_t)i + 3];
    const Patch& P = S.patches[pid];
    V3 x = r.o + t * r.d;
    V3 fu, fv;
    patch_eval(P, hu, hv, nullptr, &fu, &fv);
    V3 nn = cross(fu, fv);
    double len = std::sqrt(dot(nn, nn));
    nn = (1.0 / len) * nn;
    if (dot(nn, r.d) > 0.0) nn = -1.0 * nn;
    // the leaf domain containing (u, v)
    uint32_t pu = std::min((uint32_t)std::floor(hu / kUnit) & ~(leaf - 1), kFull - leaf);
    uint32_t pv = std::min((uint32_t)std::floor(hv / kUnit) & ~(leaf - 1), kFull - leaf);
    Bound b = calc_points_and_d_int(work_patch(S, pid), pu, pv, leaf, leaf);  // box in the frame subdivision uses
    V3 lo, hi;
    grid_box(b.q, b.d, work_patch(S, pid).pad, &lo, &hi);
    double off = (hi.x - lo.x) + (hi.y - lo.y) + (hi.z - lo.z);
    V3 org = x + off * nn;
    double u1 = uniforms[2 * (size_t)i], u2 = uniforms[2 * (size_t)i + 1];
    double rr = std::sqrt(u1), phi = 2.0 * M_PI * u2, z = std::sqrt(std::max(0.0, 1.0 - u1));
    V3 tt, bb;
    onb(nn, &tt, &bb);
    V3 dir = (rr * std::cos(phi)) * tt + (rr * std::sin(phi)) * bb + z * nn;
    o[0] = org.x; o[1] = org.y; o[2] = org.z; o[3] = 0.0;
    o[4] = dir.x; o[5] = dir.y; o[6] = dir.z; o[7] = std::numeric_limits<double>::infinity();
  }
}

// ---------------------------------------------------------------------------
// Alg. 3 as a bit-trail loop, used only by the control-logic equivalence test:
// the same split sequence and hit must come out of the recursion above.
// State: pos, size, one trail per axis, axis; a set trail bit marks a pending
// sibling at that level.  Backtracking picks the deepest pending level: the
// lowest set bit of either trail, and on equal bit positions the v split,
// which lies one level deeper than the u split with the same size.
static int ctz32(uint32_t x) {
  if (x == 0) return 32;
  int n = 0;
  while (!(x & 1u)) {
    x >>= 1;
    ++n;
  }
  return n;
}

int orc_trace_patch_alg3(void* s, uint32_t patch, const float* ray8, double cap, uint32_t* seq, int max_seq,
                         double* hit4) {
  const Scene& S = *(Scene*)s;
  const Patch& P = work_patch(S, patch);
  Ray r = work_ray(S, patch, load_ray(ray8));
  hit4[0] = cap;
  hit4[1] = (double)kNoHit;
  hit4[2] = hit4[3] = 0.0;
  if (!ray_valid(r)) return 0;
  const uint32_t leaf = kFull >> S.L;
  uint32_t pos[2] = {0, 0}, size[2] = {kFull, kFull}, trail[2] = {0, 0};
  int axis = 0;
  Best best = {cap, kNoHit, 0.0, 0.0};
  Grid p;
  V3 d = {0, 0, 0};
  if (P.gregory) {
    Bound b = calc_points_and_d_int(P, 0, 0, kFull, kFull);
    p = b.q;
    d = b.d;
  } else {
    for (int k = 0; k < 16; ++k) p.p[k] = P.cp[k];
  }
  double tcur = 0.0;
  int steps = 0;
  for (;;) {
    bool subdividing = false;
    if (!(size[0] == leaf && size[1] == leaf)) {
      if (steps < max_seq) {
        seq[4 * steps] = pos[0]; seq[4 * steps + 1] = pos[1];
        seq[4 * steps + 2] = size[0]; seq[4 * steps + 3] = size[1];
      }
      ++steps;
      Grid gl, gr;
      split_half(p, axis, &gl, &gr);
      V3 lol, hil, lor, hir;
      grid_box(gl, d, P.pad, &lol, &hil);
      grid_box(gr, d, P.pad, &lor, &hir);
      double tl = 0, tr = 0;
      bool hl = slab(r, lol, hil, best.t, &tl), hr = slab(r, lor, hir, best.t, &tr);
      if (hl || hr) {
        subdividing = true;
        bool go_r = hr && (!hl || tr < tl);
        tcur = go_r ? tr : tl;
        size[axis] >>= 1;
        if (hl && hr) trail[axis] ^= size[axis];
        if (go_r) {
          p = gr;
          pos[axis] ^= size[axis];
        } else {
          p = gl;
        }
        axis = 1 - axis;
      }
    } else if (better(tcur, patch, best)) {
      best.t = tcur;
      best.id = patch;
      best.u = (pos[0] + size[0] / 2) * kUnit;
      best.v = (pos[1] + size[1] / 2) * kUnit;
    }
    if (!subdividing) {
      if (trail[0] == 0 && trail[1] == 0) break;
      int lu = ctz32(trail[0]), lv = ctz32(trail[1]);
      axis = lu < lv ? 0 : 1;
      if (axis == 0) {
        size[0] = 1u << lu;
        size[1] = 1u << (lu + 1);
      } else {
        size[0] = size[1] = 1u << lv;
      }
      pos[axis] ^= size[axis];
      trail[axis] ^= size[axis];
      pos[0] &= ~(size[0] - 1);
      pos[1] &= ~(size[1] - 1);
      axis = 1 - axis;
    }
    if (!subdividing || P.gregory) {
      Bound b = calc_points_and_d_int(P, pos[0], pos[1], size[0], size[1]);
      p = b.q;
      d = b.d;
    }
  }
  hit4[0] = best.t;
  hit4[1] = (double)best.id;
  hit4[2] = best.u;
  hit4[3] = best.v;
  return steps;
}

// Box of the leaf at (pu, pv) (units 2^-23) as the method forms it (Alg. 3): its
// parent's lower grid (crop, or calcPointsAndD for a Gregory patch) split at 1/2
// along v, the last axis, the leaf's half extended by the parent's d, in the frame
// subdivision uses.
static void alg3_leaf_box(const Scene& S, uint32_t patch, uint32_t pu, uint32_t pv, V3* lo, V3* hi) {
  const Patch& P = work_patch(S, patch);
  const uint32_t leaf = kFull >> S.L;
  uint32_t ppv = pv & ~(2 * leaf - 1);
  Bound b = calc_points_and_d_int(P, pu, ppv, leaf, 2 * leaf);
  Grid gl, gr;
  split_half(b.q, 1, &gl, &gr);
  grid_box((pv & leaf) ? gr : gl, b.d, P.pad, lo, hi);
}

// Entry distance of a ray into that box; ancestors are not tested.  Returns +inf
// when the box is missed.
double orc_leaf_entry(void* s, uint32_t patch, const float* ray8, uint32_t pu, uint32_t pv) {
  const Scene& S = *(Scene*)s;
  Ray r = work_ray(S, patch, load_ray(ray8));
  V3 lo, hi;
  alg3_leaf_box(S, patch, pu, pv, &lo, &hi);
  double e;
  if (!ray_valid(r) || !slab(r, lo, hi, std::numeric_limits<double>::infinity(), &e))
    return std::numeric_limits<double>::infinity();
  return e;
}

// The same box as [lo, hi] (6 doubles).
void orc_leaf_box_alg3(void* s, uint32_t patch, uint32_t pu, uint32_t pv, double* box6) {
  V3 lo, hi;
  alg3_leaf_box(*(const Scene*)s, patch, pu, pv, &lo, &hi);
  box6[0] = lo.x; box6[1] = lo.y; box6[2] = lo.z; box6[3] = hi.x; box6[4] = hi.y; box6[5] = hi.z;
}

// Box [lo, hi] (6 doubles) of a domain's lower grid plus displacement
// (calcPointsAndD), in the frame subdivision uses (the patch's, when local).
void orc_domain_box(void* s, uint32_t patch, uint32_t pu, uint32_t pv, uint32_t su, uint32_t sv, double* box6) {
  const Scene& S = *(Scene*)s;
  const Patch& P = work_patch(S, patch);
  Bound b = calc_points_and_d_int(P, pu, pv, su, sv);
  V3 lo, hi;
  grid_box(b.q, b.d, P.pad, &lo, &hi);
  box6[0] = lo.x; box6[1] = lo.y; box6[2] = lo.z; box6[3] = hi.x; box6[4] = hi.y; box6[5] = hi.z;
}

}  // extern "C"
