// C ABI of the intersector: validation, scene build and upload, launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ccs.h"
#include "bvh_build.h"
#include "ccs_internal.h"
#include "patch_math.h"

namespace {

thread_local std::string g_error;

ccs_status fail(ccs_status s, const std::string& msg) {
  g_error = msg;
  return s;
}

ccs_status hip_fail(hipError_t e, const char* what) {
  return fail(CCS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int kTraversalStack = (int)ccs::kMaxBvhDepth;  // the LDS node stack of the intersect kernel
constexpr uint32_t kQueueSlots = 256;  // ray-queue counters, one per launch in flight on a scene

// Device bytes held by the library (every scene and every call's temporaries).
std::atomic<uint64_t> g_live_bytes{0};

// The cap from CCS_MAX_DEVICE_BYTES, read on every allocation; 0 means none.
ccs_status device_cap(uint64_t& cap) {
  cap = 0;
  const char* v = std::getenv("CCS_MAX_DEVICE_BYTES");
  if (!v || !*v) return CCS_OK;
  char* end = nullptr;
  errno = 0;
  const unsigned long long c = std::strtoull(v, &end, 10);
  if (errno != 0 || *end != '\0' || v[0] == '-')
    return fail(CCS_ERR_INVALID_ARG, std::string("CCS_MAX_DEVICE_BYTES is not a byte count: ") + v);
  cap = (uint64_t)c;
  return CCS_OK;
}

// Every device allocation of the library goes through this pair.
ccs_status raw_alloc(void** q, size_t bytes) {
  *q = nullptr;
  uint64_t cap;
  ccs_status st = device_cap(cap);
  if (st != CCS_OK) return st;
  const uint64_t before = g_live_bytes.fetch_add(bytes);
  if (cap != 0 && before + bytes > cap) {
    g_live_bytes.fetch_sub(bytes);
    return fail(CCS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes would exceed " +
                                 "CCS_MAX_DEVICE_BYTES=" + std::to_string(cap) + " (" + std::to_string(before) +
                                 " bytes held)");
  }
  if (hipMalloc(q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    g_live_bytes.fetch_sub(bytes);
    *q = nullptr;
    return fail(CCS_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return CCS_OK;
}

void raw_free(void* q, size_t bytes) {
  if (!q) return;
  (void)hipFree(q);
  g_live_bytes.fetch_sub(bytes);
}

}  // namespace

struct ccs_scene {
  ccs::DeviceScene dev{};
  int device = 0;
  uint32_t bvh_depth = 0;
  uint64_t device_bytes = 0;
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  double build_seconds = 0.0;
  float* cp_stage = nullptr;  // device staging buffer for host refit input
  std::vector<uint32_t> level_offsets;  // nodes of depth d: level_nodes[level_offsets[d] .. level_offsets[d+1])
  uint32_t* queues = nullptr;  // kQueueSlots ray-queue counters
  std::atomic<uint32_t> next_queue{0};
  ccs_launch_params launch{0, 16, 1, 8, 3, 8};
  uint2* policy_w = nullptr;   // packed network fragments, allocated on first use
  float4* policy_b = nullptr;
  std::vector<std::pair<void*, size_t>> allocations;  // device buffers and their sizes
};

namespace {

template <class T>
ccs_status dev_alloc(ccs_scene* s, T** p, size_t count) {
  *p = nullptr;
  const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
  void* q = nullptr;
  ccs_status st = raw_alloc(&q, bytes);
  if (st != CCS_OK) return st;
  s->allocations.emplace_back(q, bytes);
  s->device_bytes += bytes;
  *p = static_cast<T*>(q);
  return CCS_OK;
}

void dev_free(ccs_scene* s, void* p) {
  for (size_t k = 0; k < s->allocations.size(); ++k)
    if (s->allocations[k].first == p) {
      raw_free(p, s->allocations[k].second);
      s->device_bytes -= s->allocations[k].second;
      s->allocations.erase(s->allocations.begin() + (long)k);
      return;
    }
}

// Also used on the error paths of scene creation, where an upload or the frame
// refit may still be queued: the device is drained before the memory goes.
void free_scene(ccs_scene* s) {
  if (!s) return;
  if (!s->allocations.empty()) {
    (void)hipDeviceSynchronize();
    (void)hipGetLastError();
  }
  for (const auto& a : s->allocations) raw_free(a.first, a.second);
  delete s;
}

bool is_gfx950(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

// Host copies of the caller's control points and tags (device input is fetched).
ccs_status fetch_inputs(const ccs_scene_desc* d, std::vector<float>& cp, std::vector<uint8_t>& types) {
  const size_t n = d->n_patches;
  cp.resize(n * 60);
  types.resize(n);
  if (n == 0) return CCS_OK;
  if (d->location == CCS_HOST) {
    std::memcpy(cp.data(), d->control_points, n * 60 * sizeof(float));
    std::memcpy(types.data(), d->patch_types, n);
    return CCS_OK;
  }
  hipError_t e = hipMemcpy(cp.data(), d->control_points, n * 60 * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(types.data(), d->patch_types, n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "copying scene input to the host");
  return CCS_OK;
}

ccs_status check_finite(const float* cp, size_t count) {
  for (size_t k = 0; k < count; ++k)
    if (!std::isfinite(cp[k])) return fail(CCS_ERR_INVALID_ARG, "control point value " + std::to_string(k) + " is not finite");
  return CCS_OK;
}

}  // namespace

namespace {

// Device scratch owned by one synchronous call, freed on every return path.  An
// error return can leave launches of the call queued that still read it, so the
// device is drained before the memory is released.
struct Scratch {
  std::vector<std::pair<void*, size_t>> p;
  ~Scratch() {
    if (p.empty()) return;
    (void)hipDeviceSynchronize();
    (void)hipGetLastError();
    for (const auto& q : p) raw_free(q.first, q.second);
  }
  template <class T>
  ccs_status alloc(T** out, size_t count) {
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    void* q = nullptr;
    *out = nullptr;
    ccs_status st = raw_alloc(&q, bytes);
    if (st != CCS_OK) return st;
    p.emplace_back(q, bytes);
    *out = static_cast<T*>(q);
    return CCS_OK;
  }
};

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Row order of epoch e: index = (a * position + c) mod n with gcd(a, n) = 1.
void epoch_permutation(uint64_t seed, uint64_t e, uint32_t n, uint64_t& a, uint64_t& c) {
  uint64_t x = seed ^ (e * 0xD1B54A32D192ED03ull);
  if (n <= 1) {
    a = 1;
    c = 0;
    return;
  }
  a = splitmix64(x) % n;
  if (a == 0) a = 1;
  while (gcd64(a, n) != 1) a = a + 1 < n ? a + 1 : 1;
  c = splitmix64(x) % n;
}

}  // namespace

extern "C" {

const char* ccs_last_error(void) { return g_error.c_str(); }

ccs_status ccs_scene_create(const ccs_scene_desc* desc, ccs_scene** out) {
  g_error.clear();
  if (!out) return fail(CCS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(CCS_ERR_INVALID_ARG, "desc is NULL");
  const uint32_t n = desc->n_patches;
  if (n > 0 && (!desc->control_points || !desc->patch_types))
    return fail(CCS_ERR_INVALID_ARG, "control_points or patch_types is NULL");
  if (n >= (1u << 31)) return fail(CCS_ERR_INVALID_ARG, "n_patches must be below 2^31");
  if (desc->leaf_depth < 1 || desc->leaf_depth > CCS_MAX_LEAF_DEPTH)
    return fail(CCS_ERR_INVALID_ARG, "leaf_depth must be in [1, " + std::to_string(CCS_MAX_LEAF_DEPTH) + "]");
  if (desc->location != CCS_HOST && desc->location != CCS_DEVICE)
    return fail(CCS_ERR_INVALID_ARG, "location must be CCS_HOST or CCS_DEVICE");
  if ((desc->flags & ~(CCS_FLAG_LOCAL_FRAMES | CCS_FLAG_SINGLE_BOX)) != 0)
    return fail(CCS_ERR_UNSUPPORTED, "unknown flags");
  if ((desc->flags & CCS_FLAG_SINGLE_BOX) && desc->leaf_depth > ccs::kMaxLeafDepth32)
    return fail(CCS_ERR_UNSUPPORTED, "the single-box ablation supports leaf depths up to " +
                                         std::to_string(ccs::kMaxLeafDepth32));

  // host-side validation needs no GPU; device input is fetched first
  std::vector<float> cp;
  std::vector<uint8_t> types;
  if (desc->location == CCS_HOST) {
    for (uint32_t k = 0; k < n; ++k)
      if (desc->patch_types[k] > 1) return fail(CCS_ERR_INVALID_ARG, "patch type " + std::to_string(k) + " is not 0 or 1");
    ccs_status st = check_finite(desc->control_points, (size_t)n * 60);
    if (st != CCS_OK) return st;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (!is_gfx950(dev)) return fail(CCS_ERR_UNSUPPORTED, "the current device is not gfx950");
  ccs_status st = fetch_inputs(desc, cp, types);
  if (st != CCS_OK) return st;
  if (desc->location == CCS_DEVICE) {
    for (uint32_t k = 0; k < n; ++k)
      if (types[k] > 1) return fail(CCS_ERR_INVALID_ARG, "patch type " + std::to_string(k) + " is not 0 or 1");
    st = check_finite(cp.data(), cp.size());
    if (st != CCS_OK) return st;
  }

  const auto t0 = std::chrono::steady_clock::now();
  // patch boxes (hull of 16 or 20 points) and fp32 anchors (box centres)
  std::vector<ccs::BuildBox> boxes(n);
  for (uint32_t k = 0; k < n; ++k) {
    const float* p = cp.data() + 60 * (size_t)k;
    const int np = types[k] == CCS_GREGORY ? 20 : 16;
    ccs::BuildBox& b = boxes[k];
    for (int a = 0; a < 3; ++a) b.lo[a] = b.hi[a] = p[a];
    for (int s = 1; s < np; ++s)
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::fmin(b.lo[a], p[3 * s + a]);
        b.hi[a] = std::fmax(b.hi[a], p[3 * s + a]);
      }
  }
  uint32_t log2n = 0;
  while ((1ull << log2n) < (uint64_t)std::max<uint32_t>(n, 1)) ++log2n;
  const uint32_t sah_depth = (uint32_t)std::max<int>(8, kTraversalStack - 1 - (int)log2n);
  const int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  ccs::BvhOutput bvh = ccs::build_bvh(boxes, sah_depth, threads);
  if (n > 0 && bvh.max_depth >= (uint32_t)kTraversalStack)
    return fail(CCS_ERR_UNSUPPORTED, "BVH deeper than the traversal stack");

  // records in leaf order
  std::vector<float> recs((size_t)n * ccs::kRecFloats, 0.0f);
  std::vector<uint32_t> inv_perm(n);
  ccs_scene* s = new ccs_scene();
  for (int a = 0; a < 3; ++a) {
    s->lo[a] = n ? INFINITY : 0.0f;
    s->hi[a] = n ? -INFINITY : 0.0f;
  }
  for (uint32_t r = 0; r < n; ++r) {
    const uint32_t k = bvh.perm[r];
    inv_perm[k] = r;
    const float* p = cp.data() + 60 * (size_t)k;
    float* q = recs.data() + (size_t)r * ccs::kRecFloats;
    const ccs::BuildBox& b = boxes[k];
    float anc[3];
    for (int a = 0; a < 3; ++a) {
      anc[a] = 0.5f * (b.lo[a] + b.hi[a]);
      s->lo[a] = std::fmin(s->lo[a], b.lo[a]);
      s->hi[a] = std::fmax(s->hi[a], b.hi[a]);
    }
    for (int sl = 0; sl < 16; ++sl)
      for (int a = 0; a < 3; ++a) q[16 * a + sl] = p[3 * sl + a] - anc[a];
    for (int sl = 16; sl < 20; ++sl)
      for (int a = 0; a < 3; ++a) q[48 + 4 * a + (sl - 16)] = p[3 * sl + a] - anc[a];
    q[60] = anc[0];
    q[61] = anc[1];
    q[62] = anc[2];
    uint32_t meta = k | (types[k] == CCS_GREGORY ? ccs::kGregoryBit : 0u);
    std::memcpy(q + 63, &meta, 4);
  }
  s->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  s->device = dev;
  s->bvh_depth = bvh.max_depth;
  const uint32_t n_nodes = n ? (uint32_t)(bvh.nodes.size() / 16) : 0;
  ccs::DeviceScene& D = s->dev;
  D.n_patches = n;
  D.n_nodes = n_nodes;
  D.leaf_depth = (int)desc->leaf_depth;
  D.single_box = (desc->flags & CCS_FLAG_SINGLE_BOX) != 0;
  float4* nodes = nullptr;
  uint32_t *perm = nullptr, *invp = nullptr, *lvl = nullptr;
  int32_t *lpar = nullptr, *npar = nullptr;
  float* drec = nullptr;
  if ((st = dev_alloc(s, &nodes, (size_t)n_nodes * 4)) != CCS_OK || (st = dev_alloc(s, &drec, recs.size())) != CCS_OK ||
      (st = dev_alloc(s, &perm, n)) != CCS_OK || (st = dev_alloc(s, &invp, n)) != CCS_OK ||
      (st = dev_alloc(s, &lpar, n)) != CCS_OK || (st = dev_alloc(s, &npar, n_nodes)) != CCS_OK ||
      (st = dev_alloc(s, &lvl, n_nodes)) != CCS_OK || (st = dev_alloc(s, &s->queues, kQueueSlots)) != CCS_OK) {
    free_scene(s);
    return st;
  }
  // nodes grouped by depth for the level-by-level refit (parents precede children
  // in the depth-first layout, so one pass gives every depth)
  std::vector<uint32_t> node_depth(n_nodes, 0), level_nodes(n_nodes);
  uint32_t max_d = 0;
  for (uint32_t k = 1; k < n_nodes; ++k) {
    const int32_t link = bvh.node_parent[k];
    node_depth[k] = link < 0 ? 0 : node_depth[(uint32_t)link >> 1] + 1;
    max_d = std::max(max_d, node_depth[k]);
  }
  s->level_offsets.assign(n_nodes ? max_d + 2 : 1, 0);
  for (uint32_t k = 0; k < n_nodes; ++k) s->level_offsets[node_depth[k] + 1]++;
  for (size_t d = 1; d < s->level_offsets.size(); ++d) s->level_offsets[d] += s->level_offsets[d - 1];
  {
    std::vector<uint32_t> fill(s->level_offsets.begin(), s->level_offsets.end() - 1);
    for (uint32_t k = 0; k < n_nodes; ++k) level_nodes[fill[node_depth[k]]++] = k;
  }
  hipStream_t stream = (hipStream_t)desc->stream;
  struct Up {
    void* dst;
    const void* src;
    size_t bytes;
  } ups[] = {{nodes, bvh.nodes.data(), bvh.nodes.size() * sizeof(float)},
             {drec, recs.data(), recs.size() * sizeof(float)},
             {perm, bvh.perm.data(), (size_t)n * 4},
             {invp, inv_perm.data(), (size_t)n * 4},
             {lpar, bvh.leaf_parent.data(), (size_t)n * 4},
             {npar, bvh.node_parent.data(), (size_t)n_nodes * 4},
             {lvl, level_nodes.data(), (size_t)n_nodes * 4}};
  for (const Up& u : ups) {
    if (u.bytes == 0) continue;
    e = hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
      free_scene(s);
      return hip_fail(e, "uploading the scene");
    }
  }
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    free_scene(s);
    return hip_fail(e, "synchronizing the scene upload");
  }
  D.nodes = nodes;
  D.recs = drec;
  D.perm = perm;
  D.inv_perm = invp;
  D.leaf_parent = lpar;
  D.node_parent = npar;
  D.level_nodes = lvl;
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    free_scene(s);
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  D.n_cus = (uint32_t)std::max(1, cus);
  D.n_frames = 1;
  D.frame_rec_floats = (size_t)n * ccs::kRecFloats;
  D.frame_node_f4 = (size_t)n_nodes * 4;
  if ((desc->flags & CCS_FLAG_LOCAL_FRAMES) && n > 0) {
    // frames, and records in them, come from the refit kernel, so that creation and
    // every later refit compute them with the same arithmetic
    D.frame_frames_f4 = (size_t)n * 3;
    if ((st = dev_alloc(s, &D.frames, D.frame_frames_f4)) != CCS_OK) {
      free_scene(s);
      return st;
    }
    st = ccs_refit_frame(s, 0, cp.data(), CCS_HOST, desc->stream);
    if (st == CCS_OK) {
      e = hipStreamSynchronize(stream);
      if (e != hipSuccess) st = hip_fail(e, "placing patches in their frames");
    }
    if (st != CCS_OK) {
      free_scene(s);
      return st;
    }
  }
  *out = s;
  return CCS_OK;
}

ccs_status ccs_scene_set_frames(ccs_scene* s, uint32_t n_frames) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (n_frames < 1 || n_frames > 4096) return fail(CCS_ERR_INVALID_ARG, "n_frames must be in [1, 4096]");
  ccs::DeviceScene& D = s->dev;
  if (n_frames == D.n_frames) return CCS_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronizing before re-allocating frames");
  float* recs = nullptr;
  float4* nodes = nullptr;
  float4* frames = nullptr;
  ccs_status st = dev_alloc(s, &recs, D.frame_rec_floats * n_frames);
  if (st == CCS_OK) st = dev_alloc(s, &nodes, D.frame_node_f4 * n_frames);
  if (st == CCS_OK && D.frames) st = dev_alloc(s, &frames, D.frame_frames_f4 * n_frames);
  auto drop_new = [&]() {
    if (recs) dev_free(s, recs);
    if (nodes) dev_free(s, nodes);
    if (frames) dev_free(s, frames);
  };
  if (st != CCS_OK) {
    drop_new();
    return st;
  }
  // every frame starts as a copy of frame 0
  for (uint32_t f = 0; f < n_frames && e == hipSuccess; ++f) {
    if (D.frame_rec_floats)
      e = hipMemcpy(recs + f * D.frame_rec_floats, D.recs, D.frame_rec_floats * sizeof(float), hipMemcpyDeviceToDevice);
    if (e == hipSuccess && D.frame_node_f4)
      e = hipMemcpy(nodes + f * D.frame_node_f4, D.nodes, D.frame_node_f4 * sizeof(float4), hipMemcpyDeviceToDevice);
    if (e == hipSuccess && frames)
      e = hipMemcpy(frames + f * D.frame_frames_f4, D.frames, D.frame_frames_f4 * sizeof(float4),
                    hipMemcpyDeviceToDevice);
  }
  if (e != hipSuccess) {
    drop_new();
    return hip_fail(e, "copying frame 0");
  }
  dev_free(s, D.recs);
  dev_free(s, const_cast<float4*>(D.nodes));
  if (D.frames) dev_free(s, D.frames);
  D.recs = recs;
  D.nodes = nodes;
  D.frames = frames;
  D.n_frames = n_frames;
  return CCS_OK;
}

ccs_status ccs_refit_frame(ccs_scene* s, uint32_t frame, const float* control_points, int32_t location,
                           void* stream) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (frame >= s->dev.n_frames) return fail(CCS_ERR_INVALID_ARG, "frame out of range");
  if (s->dev.n_patches == 0) return CCS_OK;
  if (!control_points) return fail(CCS_ERR_INVALID_ARG, "control_points is NULL");
  if (location != CCS_HOST && location != CCS_DEVICE)
    return fail(CCS_ERR_INVALID_ARG, "location must be CCS_HOST or CCS_DEVICE");
  if (location == CCS_DEVICE && (reinterpret_cast<uintptr_t>(control_points) & 15u) != 0)
    return fail(CCS_ERR_INVALID_ARG, "device control_points must be 16-byte aligned");
  const size_t count = (size_t)s->dev.n_patches * 60;
  hipStream_t st = (hipStream_t)stream;
  const float* src = control_points;
  if (location == CCS_HOST) {
    ccs_status c = check_finite(control_points, count);
    if (c != CCS_OK) return c;
    if (!s->cp_stage) {
      c = dev_alloc(s, &s->cp_stage, count);
      if (c != CCS_OK) return c;
    }
    hipError_t e = hipMemcpyAsync(s->cp_stage, control_points, count * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "copying refit input");
    src = s->cp_stage;
  }
  ccs::DeviceScene f = s->dev;
  f.recs = s->dev.recs + frame * s->dev.frame_rec_floats;
  f.nodes = s->dev.nodes + frame * s->dev.frame_node_f4;
  if (f.frames) f.frames = s->dev.frames + frame * s->dev.frame_frames_f4;
  hipError_t e = ccs::launch_refit(f, src, s->level_offsets.data(), (uint32_t)s->level_offsets.size() - 1, st);
  if (e != hipSuccess) return hip_fail(e, "refit launch");
  // host input goes through the scene's one staging buffer: wait until the refit has
  // read it, so that a refit on another stream cannot overwrite it meanwhile
  if (location == CCS_HOST && (e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "host refit");
  return CCS_OK;
}

ccs_status ccs_refit(ccs_scene* s, const float* control_points, int32_t location, void* stream) {
  return ccs_refit_frame(s, 0, control_points, location, stream);
}

static ccs_status launch_batches(const ccs_scene* s, const ccs::BatchTable& bt, uint32_t* counters, void* stream) {
  ccs_scene* m = const_cast<ccs_scene*>(s);
  const uint32_t slot = m->next_queue.fetch_add(1) % kQueueSlots;
  const uint32_t steps = s->launch.traverse_steps ? s->launch.traverse_steps : 0xFFFFFFFFu;
  ccs::LaunchParams lp{s->launch.fetch_min, s->launch.traverse_min, s->launch.grid_min, steps, s->launch.decide_min,
                       s->queues + slot};
  hipError_t e = ccs::launch_intersect(s->dev, bt, counters, lp, s->launch.waves_per_cu, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "intersect launch");
  return CCS_OK;
}

static ccs::BatchTable one_batch(const ccs_ray* rays, uint32_t n, ccs_hit* hits) {
  ccs::BatchTable bt{};
  bt.n_batches = 1;
  bt.prefix[0] = 0;
  bt.prefix[1] = n;
  bt.frame[0] = 0;
  bt.rays[0] = rays;
  bt.hits[0] = hits;
  return bt;
}

// The persistent kernel hands out rays from a 32-bit counter that overshoots n by
// at most 64 per resident wave: below 2^31 rays it cannot wrap.
constexpr uint32_t kMaxRaysPerCall = (1u << 31) - 1u;

ccs_status ccs_intersect(const ccs_scene* s, const ccs_ray* rays, uint32_t n, ccs_hit* hits, void* stream) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (n == 0) return CCS_OK;
  if (!rays || !hits) return fail(CCS_ERR_INVALID_ARG, "rays or hits is NULL");
  if (n > kMaxRaysPerCall) return fail(CCS_ERR_INVALID_ARG, "more than 2^31 - 1 rays in one call");
  return launch_batches(s, one_batch(rays, n, hits), nullptr, stream);
}

ccs_status ccs_intersect_counted(const ccs_scene* s, const ccs_ray* rays, uint32_t n, ccs_hit* hits,
                                 uint32_t* counters, void* stream) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (n == 0) return CCS_OK;
  if (!rays || !hits || !counters) return fail(CCS_ERR_INVALID_ARG, "rays, hits or counters is NULL");
  if (n > kMaxRaysPerCall) return fail(CCS_ERR_INVALID_ARG, "more than 2^31 - 1 rays in one call");
  return launch_batches(s, one_batch(rays, n, hits), counters, stream);
}

static ccs_status batched(const ccs_scene* s, const ccs_batch* batches, uint32_t n_batches, uint32_t* counters,
                          void* stream) {
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (n_batches == 0) return CCS_OK;
  if (!batches) return fail(CCS_ERR_INVALID_ARG, "batches is NULL");
  if (n_batches > (uint32_t)ccs::kMaxBatches)
    return fail(CCS_ERR_INVALID_ARG, "at most " + std::to_string(ccs::kMaxBatches) + " batches per call");
  ccs::BatchTable bt{};
  uint64_t total = 0;
  bt.n_batches = n_batches;
  for (uint32_t b = 0; b < n_batches; ++b) {
    const ccs_batch& x = batches[b];
    if (x.frame >= s->dev.n_frames) return fail(CCS_ERR_INVALID_ARG, "batch frame out of range");
    if (x.n > 0 && (!x.rays || !x.hits)) return fail(CCS_ERR_INVALID_ARG, "batch rays or hits is NULL");
    bt.prefix[b] = (uint32_t)total;
    bt.frame[b] = x.frame;
    bt.rays[b] = x.rays;
    bt.hits[b] = x.hits;
    total += x.n;
  }
  if (total > kMaxRaysPerCall) return fail(CCS_ERR_INVALID_ARG, "more than 2^31 - 1 rays in one call");
  bt.prefix[n_batches] = (uint32_t)total;
  if (total == 0) return CCS_OK;
  return launch_batches(s, bt, counters, stream);
}

ccs_status ccs_intersect_batched(const ccs_scene* s, const ccs_batch* batches, uint32_t n_batches, void* stream) {
  g_error.clear();
  return batched(s, batches, n_batches, nullptr, stream);
}

ccs_status ccs_intersect_batched_counted(const ccs_scene* s, const ccs_batch* batches, uint32_t n_batches,
                                         uint32_t* counters, void* stream) {
  g_error.clear();
  if (!counters) return fail(CCS_ERR_INVALID_ARG, "counters is NULL");
  return batched(s, batches, n_batches, counters, stream);
}

ccs_status ccs_scene_set_launch(ccs_scene* s, const ccs_launch_params* p) {
  g_error.clear();
  if (!s || !p) return fail(CCS_ERR_INVALID_ARG, "scene or params is NULL");
  if (p->fetch_min < 1 || p->fetch_min > 64 || p->traverse_min < 1 || p->traverse_min > 64 || p->grid_min < 1 ||
      p->grid_min > 64 || p->decide_min < 1 || p->decide_min > 64)
    return fail(CCS_ERR_INVALID_ARG, "phase thresholds must be in [1, 64]");
  s->launch = *p;
  return CCS_OK;
}

ccs_status ccs_scene_get_launch(const ccs_scene* s, ccs_launch_params* p) {
  g_error.clear();
  if (!s || !p) return fail(CCS_ERR_INVALID_ARG, "scene or params is NULL");
  *p = s->launch;
  if (p->waves_per_cu == 0)
    p->waves_per_cu = (uint32_t)ccs::max_waves_per_cu(false, s->dev.policy.w != nullptr, s->dev.single_box,
                                                      s->dev.leaf_depth > (int)ccs::kMaxLeafDepth32);
  return CCS_OK;
}

ccs_status ccs_bounce_frame(const ccs_scene* s, uint32_t frame, const ccs_ray* rays, const ccs_hit* hits,
                            const float* uniforms, uint32_t n, ccs_ray* out_rays, void* stream) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (frame >= s->dev.n_frames) return fail(CCS_ERR_INVALID_ARG, "frame out of range");
  if (n == 0) return CCS_OK;
  if (!rays || !hits || !uniforms || !out_rays) return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  if ((const void*)out_rays == (const void*)rays) return fail(CCS_ERR_INVALID_ARG, "out_rays aliases rays");
  ccs::DeviceScene f = s->dev;
  f.recs = s->dev.recs + frame * s->dev.frame_rec_floats;
  f.nodes = s->dev.nodes + frame * s->dev.frame_node_f4;
  if (f.frames) f.frames = s->dev.frames + frame * s->dev.frame_frames_f4;
  hipError_t e = ccs::launch_bounce(f, rays, hits, uniforms, n, out_rays, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bounce launch");
  return CCS_OK;
}

ccs_status ccs_bounce(const ccs_scene* s, const ccs_ray* rays, const ccs_hit* hits, const float* uniforms, uint32_t n,
                      ccs_ray* out_rays, void* stream) {
  return ccs_bounce_frame(s, 0, rays, hits, uniforms, n, out_rays, stream);
}

ccs_status ccs_compact_rays(const ccs_ray* rays, uint32_t n, ccs_ray* out_rays, uint32_t* out_index, uint32_t* work,
                            void* stream) {
  g_error.clear();
  if (!work) return fail(CCS_ERR_INVALID_ARG, "work is NULL");
  if (n > 0 && (!rays || !out_rays || !out_index)) return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  if (n > 0 && (const void*)out_rays == (const void*)rays) return fail(CCS_ERR_INVALID_ARG, "out_rays aliases rays");
  if (((uintptr_t)rays | (uintptr_t)out_rays) % 16 != 0 || ((uintptr_t)out_index | (uintptr_t)work) % 4 != 0)
    return fail(CCS_ERR_INVALID_ARG, "rays and out_rays must be 16-byte aligned, out_index and work 4-byte aligned");
  hipError_t e = ccs::launch_compact_rays(rays, n, out_rays, out_index, work, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "compaction launch");
  return CCS_OK;
}

ccs_status ccs_debug_grids(const ccs_scene* s, uint32_t frame, const uint32_t* patch_ids, const uint32_t* codes,
                           const uint32_t* depths, uint32_t n, float* out, void* stream) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (frame >= s->dev.n_frames) return fail(CCS_ERR_INVALID_ARG, "frame out of range");
  if (n == 0) return CCS_OK;
  if (!patch_ids || !codes || !depths || !out) return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  if (s->dev.leaf_depth > (int)ccs::kMaxLeafDepth32)
    return fail(CCS_ERR_UNSUPPORTED, "32-bit path codes: leaf depths up to " + std::to_string(ccs::kMaxLeafDepth32));
  ccs::DeviceScene f = s->dev;
  f.recs = s->dev.recs + frame * s->dev.frame_rec_floats;
  hipError_t e = ccs::launch_debug_grids(f, patch_ids, codes, depths, n, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "debug grid launch");
  return CCS_OK;
}

// ------------------------------------------------------- learned child ordering
ccs_status ccs_scene_set_policy(ccs_scene* s, const float* params, void* stream) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (!params) {
    s->dev.policy = ccs::PolicyDev{nullptr, nullptr};
    return CCS_OK;
  }
  if (s->dev.single_box) return fail(CCS_ERR_UNSUPPORTED, "the single-box ablation has no learned order");
  if (s->dev.leaf_depth > (int)ccs::kMaxLeafDepth32)
    return fail(CCS_ERR_UNSUPPORTED, "the learned order supports leaf depths up to " +
                                         std::to_string(ccs::kMaxLeafDepth32));
  if (s->bvh_depth >= ccs::kMaxBvhDepthLearned)
    return fail(CCS_ERR_UNSUPPORTED, "BVH depth " + std::to_string(s->bvh_depth) +
                                         " exceeds the learned-order kernel's node stack");
  if (!s->policy_w) {
    ccs_status st = dev_alloc(s, &s->policy_w, (size_t)ccs::kPolicyWTiles * 64);
    if (st == CCS_OK) st = dev_alloc(s, &s->policy_b, (size_t)ccs::kPolicyBTiles * 64);
    if (st != CCS_OK) return st;
  }
  hipError_t e = ccs::launch_policy_pack(params, s->policy_w, s->policy_b, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "policy pack launch");
  s->dev.policy = ccs::PolicyDev{s->policy_w, s->policy_b};
  return CCS_OK;
}

ccs_status ccs_policy_record(const ccs_scene* s, const ccs_ray* rays, const ccs_hit* hits, uint32_t n,
                             float* features, uint8_t* labels, void* stream) {
  g_error.clear();
  if (!s) return fail(CCS_ERR_INVALID_ARG, "scene is NULL");
  if (n == 0) return CCS_OK;
  if (!rays || !hits || !features || !labels) return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  if ((uint64_t)n * (uint64_t)s->dev.leaf_depth >= (1ull << 36))
    return fail(CCS_ERR_INVALID_ARG, "too many records for one call");
  hipError_t e = ccs::launch_record(s->dev, rays, hits, n, features, labels, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "record launch");
  return CCS_OK;
}

ccs_status ccs_policy_infer(const float* params, const float* features, uint32_t n, float* logits, void* stream) {
  g_error.clear();
  if (n == 0) return CCS_OK;
  if (!params || !features || !logits) return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  Scratch sc;
  uint2* w = nullptr;
  float4* b = nullptr;
  ccs_status st = sc.alloc(&w, (size_t)ccs::kPolicyWTiles * 64);
  if (st == CCS_OK) st = sc.alloc(&b, (size_t)ccs::kPolicyBTiles * 64);
  if (st != CCS_OK) return st;
  hipStream_t str = (hipStream_t)stream;
  hipError_t e = ccs::launch_policy_pack(params, w, b, str);
  if (e == hipSuccess) e = ccs::launch_policy_infer(ccs::PolicyDev{w, b}, features, n, logits, str);
  if (e == hipSuccess) e = hipStreamSynchronize(str);
  if (e != hipSuccess) return hip_fail(e, "policy inference");
  return CCS_OK;
}

ccs_status ccs_policy_grad(const float* params, const float* features, const uint8_t* labels, uint32_t n,
                           uint32_t bf16, float* grad, float* loss, void* stream) {
  g_error.clear();
  if (!params || !grad || !loss || (n > 0 && (!features || !labels)))
    return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  hipStream_t str = (hipStream_t)stream;
  const uint32_t nblk = std::max<uint32_t>(1, (n + 63) / 64);
  Scratch sc;
  float *partial = nullptr, *lossp = nullptr;
  ccs_status st = sc.alloc(&partial, (size_t)nblk * ccs::kPolicyParams);
  if (st == CCS_OK) st = sc.alloc(&lossp, (size_t)2 * nblk);
  if (st != CCS_OK) return st;
  hipError_t e = hipSuccess;
  if (n == 0) {
    e = ccs::launch_fill(partial, ccs::kPolicyParams, 0.0f, str);
    if (e == hipSuccess) e = ccs::launch_fill(lossp, 2, 0.0f, str);
  } else {
    e = ccs::launch_mlp_grad(params, features, labels, n, n, 0, 1, 0, bf16 != 0, partial, lossp, str);
  }
  if (e == hipSuccess) e = ccs::launch_mlp_reduce(partial, lossp, nblk, grad, loss, str);
  if (e == hipSuccess) e = hipStreamSynchronize(str);
  if (e != hipSuccess) return hip_fail(e, "policy gradient");
  return CCS_OK;
}

ccs_status ccs_policy_grad_noalloc(const float* params, const float* features, const uint8_t* labels, uint32_t n,
                                   uint32_t bf16, float* grad, float* loss, void* stream) {
  g_error.clear();
  if (!params || !grad || !loss || (n > 0 && (!features || !labels)))
    return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  if (n > ccs::kGradScratchBlocks * 64u)
    return fail(CCS_ERR_INVALID_ARG, "n = " + std::to_string(n) + " rows exceeds the " +
                                         std::to_string(ccs::kGradScratchBlocks * 64u) +
                                         " rows of the preallocated gradient scratch");
  float *partial = nullptr, *lossp = nullptr;
  hipError_t e = ccs::grad_scratch(&partial, &lossp);
  if (e != hipSuccess) return hip_fail(e, "gradient scratch address");
  hipStream_t str = (hipStream_t)stream;
  const uint32_t nblk = std::max<uint32_t>(1, (n + 63) / 64);
  if (n == 0) {  // one block of zeros (a fill kernel, no memset node under graph capture)
    e = ccs::launch_fill(partial, ccs::kPolicyParams, 0.0f, str);
    if (e == hipSuccess) e = ccs::launch_fill(lossp, 2, 0.0f, str);
  } else {  // every block writes its whole partial row and its loss pair
    e = ccs::launch_mlp_grad(params, features, labels, n, n, 0, 1, 0, bf16 != 0, partial, lossp, str);
  }
  if (e == hipSuccess) e = ccs::launch_mlp_reduce(partial, lossp, nblk, grad, loss, str);
  if (e != hipSuccess) return hip_fail(e, "policy gradient");
  return CCS_OK;
}

ccs_status ccs_policy_train(float* params, const float* features, const uint8_t* labels, uint32_t n,
                            const ccs_train_params* tp, ccs_adam_state* state, float* loss_history, void* stream) {
  g_error.clear();
  if (!params || !tp || (n > 0 && (!features || !labels))) return fail(CCS_ERR_INVALID_ARG, "a pointer is NULL");
  if (state && (!state->m || !state->v)) return fail(CCS_ERR_INVALID_ARG, "Adam state moments are NULL");
  if (n == 0 || tp->steps == 0) return CCS_OK;
  if (tp->batch == 0) return fail(CCS_ERR_INVALID_ARG, "batch is 0");
  if (!(tp->lr > 0.0f) || !(tp->beta1 >= 0.0f && tp->beta1 < 1.0f) || !(tp->beta2 >= 0.0f && tp->beta2 < 1.0f) ||
      !(tp->eps > 0.0f))
    return fail(CCS_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
  const uint64_t t0 = state ? state->t : 0;
  if (t0 > (1ull << 32)) return fail(CCS_ERR_INVALID_ARG, "Adam step count above 2^32");
  const uint32_t batch = std::min(tp->batch, n);
  const uint32_t nblk = (batch + 63) / 64;
  const uint32_t per_epoch = std::max<uint32_t>(1, n / batch);
  hipStream_t str = (hipStream_t)stream;
  Scratch sc;
  float *partial = nullptr, *lossp = nullptr, *m = state ? state->m : nullptr, *v = state ? state->v : nullptr;
  ccs_status st = sc.alloc(&partial, (size_t)nblk * ccs::kPolicyParams);
  if (st == CCS_OK) st = sc.alloc(&lossp, (size_t)2 * nblk);
  if (st == CCS_OK && !state) st = sc.alloc(&m, (size_t)ccs::kPolicyParams);
  if (st == CCS_OK && !state) st = sc.alloc(&v, (size_t)ccs::kPolicyParams);
  if (st != CCS_OK) return st;
  hipError_t e = hipSuccess;
  if (!state) {
    e = ccs::launch_fill(m, ccs::kPolicyParams, 0.0f, str);
    if (e == hipSuccess) e = ccs::launch_fill(v, ccs::kPolicyParams, 0.0f, str);
  }
  // beta^t by the same sequence of double products an uninterrupted run forms
  double b1t = 1.0, b2t = 1.0;
  for (uint64_t k = 0; k < t0 && (b1t != 0.0 || b2t != 0.0); ++k) {  // both stay 0 once they reach it
    b1t *= tp->beta1;
    b2t *= tp->beta2;
  }
  uint64_t pa = 1, pc = 0, cur_epoch = ~0ull;
  for (uint32_t s = 0; s < tp->steps && e == hipSuccess; ++s) {
    const uint64_t step = t0 + s;
    const uint64_t epoch = step / per_epoch;
    if (epoch != cur_epoch) {
      epoch_permutation(tp->seed, epoch, n, pa, pc);
      cur_epoch = epoch;
    }
    const uint64_t pos0 = (step % per_epoch) * batch;
    e = ccs::launch_mlp_grad(params, features, labels, n, batch, pos0, pa, pc, tp->bf16 != 0, partial, lossp, str);
    b1t *= tp->beta1;
    b2t *= tp->beta2;
    if (e == hipSuccess)
      e = ccs::launch_mlp_adam(params, m, v, partial, lossp, nblk, tp->lr, tp->beta1, tp->beta2, tp->eps,
                               (float)(1.0 / (1.0 - b1t)), (float)(1.0 / (1.0 - b2t)),
                               loss_history ? loss_history + s : nullptr, str);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(str);
  if (e != hipSuccess) return hip_fail(e, "policy training");
  if (state) state->t = t0 + tp->steps;
  return CCS_OK;
}

uint64_t ccs_device_bytes_in_use(void) { return g_live_bytes.load(); }

ccs_status ccs_scene_info_get(const ccs_scene* s, ccs_scene_info* info) {
  g_error.clear();
  if (!s || !info) return fail(CCS_ERR_INVALID_ARG, "scene or info is NULL");
  info->n_patches = s->dev.n_patches;
  info->n_nodes = s->dev.n_nodes;
  info->leaf_depth = (uint32_t)s->dev.leaf_depth;
  info->bvh_depth = s->bvh_depth;
  info->device_bytes = s->device_bytes;
  for (int a = 0; a < 3; ++a) {
    info->lo[a] = s->lo[a];
    info->hi[a] = s->hi[a];
  }
  info->build_seconds = s->build_seconds;
  info->n_frames = s->dev.n_frames;
  return CCS_OK;
}

void ccs_scene_destroy(ccs_scene* s) { free_scene(s); }  // drains the device first

}  // extern "C"
