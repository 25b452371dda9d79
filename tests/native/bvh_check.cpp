// Structural check of the host BVH builder, built with the address and
// undefined-behaviour sanitizers by the CPU test suite.  For each synthetic box
// set it verifies that the hierarchy is a binary tree over exactly the input
// boxes (n - 1 nodes, each record reached once, perm a permutation), that the
// parent links agree with the child slots, that every child slot holds exactly
// the union of the boxes below it (min/max are exact in floating point), that
// max_depth is the deepest leaf, and that the result does not depend on the
// number of build threads.  Prints one line per case; exit status 1 on failure.

#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1811_03510_amd/csrc/bvh_build.h"

using ccs::BuildBox;
using ccs::BvhOutput;

namespace {

int g_failures = 0;

void check(bool ok, const std::string& what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what.c_str());
    ++g_failures;
  }
}

struct Box {
  float lo[3], hi[3];
};

Box slot(const BvhOutput& o, uint32_t node, int side) {
  const float* f = o.nodes.data() + 16 * (size_t)node + (side ? 6 : 0);
  Box b;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = f[a];
    b.hi[a] = f[3 + a];
  }
  return b;
}

int32_t child(const BvhOutput& o, uint32_t node, int side) {
  int32_t c;
  std::memcpy(&c, o.nodes.data() + 16 * (size_t)node + 12 + side, 4);
  return c;
}

bool same(const Box& x, const Box& y) {
  for (int a = 0; a < 3; ++a)
    if (x.lo[a] != y.lo[a] || x.hi[a] != y.hi[a]) return false;
  return true;
}

// Walks the subtree under slot (node, side); returns its union box and records depths.
Box walk(const BvhOutput& o, const std::vector<BuildBox>& in, uint32_t node, int side, uint32_t depth,
         std::vector<int>& seen_rec, std::vector<int>& seen_node, uint32_t& deepest, const char* name) {
  const int32_t c = child(o, node, side);
  Box u;
  if (c < 0) {
    const uint32_t r = (uint32_t)~c;
    check(r < seen_rec.size(), std::string(name) + ": record index in range");
    if (r >= seen_rec.size()) return slot(o, node, side);
    seen_rec[r]++;
    check(o.leaf_parent[r] == (int32_t)((node << 1) | (uint32_t)side), std::string(name) + ": leaf_parent link");
    const BuildBox& b = in[o.perm[r]];
    for (int a = 0; a < 3; ++a) {
      u.lo[a] = b.lo[a];
      u.hi[a] = b.hi[a];
    }
    deepest = std::max(deepest, depth);
  } else {
    const uint32_t k = (uint32_t)c;
    check(k < seen_node.size() && k != 0, std::string(name) + ": node index in range");
    if (k >= seen_node.size() || k == 0) return slot(o, node, side);
    seen_node[k]++;
    check(o.node_parent[k] == (int32_t)((node << 1) | (uint32_t)side), std::string(name) + ": node_parent link");
    const Box l = walk(o, in, k, 0, depth + 1, seen_rec, seen_node, deepest, name);
    const Box r = walk(o, in, k, 1, depth + 1, seen_rec, seen_node, deepest, name);
    for (int a = 0; a < 3; ++a) {
      u.lo[a] = std::min(l.lo[a], r.lo[a]);
      u.hi[a] = std::max(l.hi[a], r.hi[a]);
    }
  }
  check(same(u, slot(o, node, side)), std::string(name) + ": child slot is the union of its subtree");
  return u;
}

void verify(const char* name, const std::vector<BuildBox>& in, uint32_t sah_depth) {
  const int before = g_failures;
  const BvhOutput o = ccs::build_bvh(in, sah_depth, 1);
  const uint32_t n = (uint32_t)in.size();
  if (n == 0) {
    check(o.nodes.empty() && o.perm.empty() && o.max_depth == 0, std::string(name) + ": empty input, empty tree");
  } else {
    const uint32_t n_nodes = n == 1 ? 1 : n - 1;
    check(o.nodes.size() == 16 * (size_t)n_nodes, std::string(name) + ": n - 1 nodes");
    check(o.perm.size() == n && o.leaf_parent.size() == n && o.node_parent.size() == n_nodes,
          std::string(name) + ": output sizes");
    std::vector<int> hit(n, 0);
    for (uint32_t r = 0; r < n && r < o.perm.size(); ++r)
      if (o.perm[r] < n) hit[o.perm[r]]++;
    bool perm_ok = true;
    for (int h : hit) perm_ok = perm_ok && h == 1;
    check(perm_ok, std::string(name) + ": perm is a permutation");
    check(o.node_parent.empty() || o.node_parent[0] == -1, std::string(name) + ": root has no parent");
    std::vector<int> seen_rec(n, 0), seen_node(n_nodes, 0);
    uint32_t deepest = 0;
    if (n == 1) {
      const Box a = walk(o, in, 0, 0, 1, seen_rec, seen_node, deepest, name);
      const Box b = slot(o, 0, 1);
      check(child(o, 0, 1) == ~(int32_t)0 && same(a, b), std::string(name) + ": a lone patch fills both slots");
      check(seen_rec[0] == 1, std::string(name) + ": lone record reached");
    } else {
      walk(o, in, 0, 0, 1, seen_rec, seen_node, deepest, name);
      walk(o, in, 0, 1, 1, seen_rec, seen_node, deepest, name);
      bool once = true;
      for (int s : seen_rec) once = once && s == 1;
      check(once, std::string(name) + ": every record reached exactly once");
      once = true;
      for (uint32_t k = 1; k < n_nodes; ++k) once = once && seen_node[k] == 1;
      check(once, std::string(name) + ": every internal node reached exactly once");
    }
    check(deepest == o.max_depth, std::string(name) + ": max_depth is the deepest leaf");
    // below sah_depth every split is an object median, so no leaf lies deeper than
    // sah_depth + ceil(log2 n): the bound the traversal stack is sized by
    uint32_t log2n = 0;
    while ((1ull << log2n) < (uint64_t)n) ++log2n;
    check(o.max_depth <= sah_depth + log2n, std::string(name) + ": depth within sah_depth + ceil(log2 n)");
    const BvhOutput p = ccs::build_bvh(in, sah_depth, 8);
    check(p.nodes.size() == o.nodes.size() &&
              std::memcmp(p.nodes.data(), o.nodes.data(), o.nodes.size() * sizeof(float)) == 0 &&
              p.perm == o.perm && p.leaf_parent == o.leaf_parent && p.node_parent == o.node_parent &&
              p.max_depth == o.max_depth,
          std::string(name) + ": same tree with 1 and 8 build threads");
  }
  std::printf("%s %s: n=%u depth=%u\n", g_failures == before ? "ok" : "FAILED", name, n, o.max_depth);
}

std::vector<BuildBox> random_boxes(uint32_t n, uint32_t seed, float size) {
  std::mt19937 g(seed);
  std::uniform_real_distribution<float> U(-100.0f, 100.0f), S(0.0f, size);
  std::vector<BuildBox> v(n);
  for (auto& b : v)
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = U(g);
      b.hi[a] = b.lo[a] + S(g);
    }
  return v;
}

// The SAH depth the library uses for n patches with its 48-entry traversal stack.
uint32_t lib_sah_depth(uint32_t n) {
  uint32_t log2n = 0;
  while ((1ull << log2n) < (uint64_t)std::max<uint32_t>(n, 1)) ++log2n;
  return (uint32_t)std::max<int>(8, 48 - 1 - (int)log2n);
}

}  // namespace

int main() {
  verify("empty", {}, 40);
  verify("one", random_boxes(1, 1, 1.0f), 40);
  verify("two", random_boxes(2, 2, 1.0f), 40);
  verify("three", random_boxes(3, 3, 1.0f), 40);
  verify("random 1000", random_boxes(1000, 4, 5.0f), 40);
  verify("random 1000 median below depth 3", random_boxes(1000, 5, 5.0f), 3);
  {
    std::vector<BuildBox> v(257);
    for (auto& b : v)
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = -1.0f;
        b.hi[a] = 1.0f;
      }
    verify("identical 257", v, 40);
  }
  {
    std::vector<BuildBox> v = random_boxes(5000, 6, 0.5f);
    for (auto& b : v) {  // centroids on one line, flat in z
      b.lo[1] = b.hi[1] = 0.0f;
      b.lo[2] = b.hi[2] = 3.0f;
    }
    verify("collinear flat 5000, SAH to depth 40", v, 40);
    verify("collinear flat 5000", v, lib_sah_depth(5000));
  }
  {
    std::vector<BuildBox> v = random_boxes(70000, 7, 0.01f);  // above the parallel-build threshold
    for (size_t k = 0; k < v.size(); k += 2)
      for (int a = 0; a < 3; ++a) {
        v[k].lo[a] = v[k].lo[a] * 1e-3f + 1e4f;
        v[k].hi[a] = v[k].hi[a] * 1e-3f + 1e4f;
      }
    verify("two clusters 70000", v, lib_sah_depth(70000));
  }
  std::printf("%d failure(s)\n", g_failures);
  return g_failures ? 1 : 0;
}
