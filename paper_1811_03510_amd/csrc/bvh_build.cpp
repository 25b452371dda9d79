// Binned-SAH BVH build over patch boxes (host, C++17, threads at the top levels).
//
// With one patch per leaf a subtree over k patches has exactly k-1 internal
// nodes, so the depth-first layout is known before the subtree is built: the
// left child of node i is node i+1, the right child node i+k_left.  Subtrees are
// therefore built independently (and in parallel) into disjoint index ranges.

#include "bvh_build.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>

namespace ccs {
namespace {

constexpr int kBins = 32;
constexpr uint32_t kParallelMin = 1u << 15;

struct Bounds {
  float lo[3], hi[3];
  void reset() {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::numeric_limits<float>::infinity();
      hi[k] = -std::numeric_limits<float>::infinity();
    }
  }
  void grow(const float* l, const float* h) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], l[k]);
      hi[k] = std::max(hi[k], h[k]);
    }
  }
  void grow(const Bounds& b) { grow(b.lo, b.hi); }
  float area() const {
    float d[3];
    for (int k = 0; k < 3; ++k) d[k] = std::max(0.0f, hi[k] - lo[k]);
    return 2.0f * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
  }
};

struct Builder {
  const std::vector<BuildBox>& boxes;
  std::vector<uint32_t> idx;
  std::vector<float> cen;  // 3 per box
  BvhOutput& out;
  uint32_t sah_depth;
  int threads_left;

  Builder(const std::vector<BuildBox>& b, BvhOutput& o, uint32_t sd, int nt)
      : boxes(b), out(o), sah_depth(sd), threads_left(nt) {}

  Bounds range_bounds(uint32_t b, uint32_t e) const {
    Bounds r;
    r.reset();
    for (uint32_t k = b; k < e; ++k) r.grow(boxes[idx[k]].lo, boxes[idx[k]].hi);
    return r;
  }

  uint32_t split_range(uint32_t b, uint32_t e, uint32_t depth) {
    float clo[3], chi[3];
    for (int k = 0; k < 3; ++k) {
      clo[k] = std::numeric_limits<float>::infinity();
      chi[k] = -std::numeric_limits<float>::infinity();
    }
    for (uint32_t k = b; k < e; ++k)
      for (int a = 0; a < 3; ++a) {
        clo[a] = std::min(clo[a], cen[3 * idx[k] + a]);
        chi[a] = std::max(chi[a], cen[3 * idx[k] + a]);
      }
    int widest = 0;
    for (int a = 1; a < 3; ++a)
      if (chi[a] - clo[a] > chi[widest] - clo[widest]) widest = a;
    const uint32_t mid = b + (e - b) / 2;
    auto median = [&](int axis) {
      std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](uint32_t x, uint32_t y) {
        const float cx = cen[3 * x + axis], cy = cen[3 * y + axis];
        return cx < cy || (cx == cy && x < y);
      });
      return mid;
    };
    if (!(chi[widest] > clo[widest])) return mid;  // all centroids coincide: any split
    if (depth >= sah_depth) return median(widest);
    float best_cost = std::numeric_limits<float>::infinity();
    int best_axis = -1, best_bin = -1;
    for (int a = 0; a < 3; ++a) {
      const float ext = chi[a] - clo[a];
      if (!(ext > 0.0f)) continue;
      const float scale = kBins / ext;
      Bounds bb[kBins];
      uint32_t cnt[kBins];
      for (int q = 0; q < kBins; ++q) {
        bb[q].reset();
        cnt[q] = 0;
      }
      for (uint32_t k = b; k < e; ++k) {
        int q = (int)((cen[3 * idx[k] + a] - clo[a]) * scale);
        q = std::min(std::max(q, 0), kBins - 1);
        cnt[q]++;
        bb[q].grow(boxes[idx[k]].lo, boxes[idx[k]].hi);
      }
      float right_area[kBins];
      uint32_t right_cnt[kBins];
      Bounds acc;
      acc.reset();
      uint32_t c = 0;
      for (int q = kBins - 1; q > 0; --q) {
        acc.grow(bb[q]);
        c += cnt[q];
        right_area[q] = acc.area();
        right_cnt[q] = c;
      }
      acc.reset();
      c = 0;
      for (int q = 0; q < kBins - 1; ++q) {
        acc.grow(bb[q]);
        c += cnt[q];
        if (c == 0 || right_cnt[q + 1] == 0) continue;
        const float cost = acc.area() * (float)c + right_area[q + 1] * (float)right_cnt[q + 1];
        if (cost < best_cost) {
          best_cost = cost;
          best_axis = a;
          best_bin = q;
        }
      }
    }
    if (best_axis < 0) return median(widest);
    const float scale = kBins / (chi[best_axis] - clo[best_axis]);
    auto it = std::partition(idx.begin() + b, idx.begin() + e, [&](uint32_t x) {
      int q = (int)((cen[3 * x + best_axis] - clo[best_axis]) * scale);
      q = std::min(std::max(q, 0), kBins - 1);
      return q <= best_bin;
    });
    const uint32_t m = (uint32_t)(it - idx.begin());
    if (m == b || m == e) return median(widest);
    return m;
  }

  void set_child(uint32_t node, int side, const Bounds& bb, int32_t ref) {
    float* f = out.nodes.data() + 16 * (size_t)node;
    const int base = side ? 6 : 0;
    for (int k = 0; k < 3; ++k) {
      f[base + k] = bb.lo[k];
      f[base + 3 + k] = bb.hi[k];
    }
    std::memcpy(f + 12 + side, &ref, 4);
  }

  // Builds internal node `node` over idx[b, e) (e - b >= 2); returns its bounds
  // and the depth of its deepest leaf below it.
  Bounds build(uint32_t b, uint32_t e, uint32_t node, uint32_t depth, uint32_t* deepest) {
    const uint32_t m = split_range(b, e, depth);
    Bounds lb, rb;
    uint32_t dl = depth + 1, dr = depth + 1;
    const uint32_t left_node = node + 1, right_node = node + (m - b);
    auto do_left = [&]() {
      if (m - b == 1) {
        lb = range_bounds(b, m);
        out.leaf_parent[b] = (int32_t)((node << 1) | 0);
      } else {
        out.node_parent[left_node] = (int32_t)((node << 1) | 0);
        lb = build(b, m, left_node, depth + 1, &dl);
      }
    };
    auto do_right = [&]() {
      if (e - m == 1) {
        rb = range_bounds(m, e);
        out.leaf_parent[m] = (int32_t)((node << 1) | 1);
      } else {
        out.node_parent[right_node] = (int32_t)((node << 1) | 1);
        rb = build(m, e, right_node, depth + 1, &dr);
      }
    };
    bool spawned = false;
    std::thread th;
    if (e - b >= kParallelMin) {
      int left = __atomic_fetch_sub(&threads_left, 1, __ATOMIC_SEQ_CST);
      if (left > 1) {
        th = std::thread(do_left);
        spawned = true;
      } else {
        __atomic_fetch_add(&threads_left, 1, __ATOMIC_SEQ_CST);
      }
    }
    if (!spawned) do_left();
    do_right();
    if (spawned) {
      th.join();
      __atomic_fetch_add(&threads_left, 1, __ATOMIC_SEQ_CST);
    }
    set_child(node, 0, lb, m - b == 1 ? ~(int32_t)b : (int32_t)left_node);
    set_child(node, 1, rb, e - m == 1 ? ~(int32_t)m : (int32_t)right_node);
    *deepest = std::max(dl, dr);
    Bounds r = lb;
    r.grow(rb);
    return r;
  }
};

}  // namespace

BvhOutput build_bvh(const std::vector<BuildBox>& boxes, uint32_t sah_depth, int n_threads) {
  BvhOutput out;
  const uint32_t n = (uint32_t)boxes.size();
  if (n == 0) return out;
  const uint32_t n_nodes = n == 1 ? 1 : n - 1;
  out.nodes.assign(16 * (size_t)n_nodes, 0.0f);
  out.leaf_parent.assign(n, -1);
  out.node_parent.assign(n_nodes, -1);
  Builder B(boxes, out, sah_depth, std::max(1, n_threads));
  B.idx.resize(n);
  B.cen.resize(3 * (size_t)n);
  for (uint32_t k = 0; k < n; ++k) {
    B.idx[k] = k;
    for (int a = 0; a < 3; ++a) B.cen[3 * k + a] = 0.5f * (boxes[k].lo[a] + boxes[k].hi[a]);
  }
  if (n == 1) {
    // a lone patch fills both child slots (an inverted "empty" box would still pass
    // a min/max slab test); visiting it twice cannot change the closest hit
    Bounds b = B.range_bounds(0, 1);
    B.set_child(0, 0, b, ~(int32_t)0);
    B.set_child(0, 1, b, ~(int32_t)0);
    out.leaf_parent[0] = 0;
    out.max_depth = 1;
  } else {
    uint32_t deepest = 0;
    B.build(0, n, 0, 0, &deepest);
    out.max_depth = deepest;
  }
  out.perm = B.idx;
  return out;
}

}  // namespace ccs
