// Closest-hit kernel: BVH traversal over patch boxes and, per candidate patch,
// the stackless hierarchical subdivision of Alg. 3 (Sec. 3.3) in fp32.
//
// Persistent waves (wave64, one wave per block).  Every lane carries one ray
// through a small state machine:
//   FETCH    waiting for a ray from the launch's global queue
//   TRAVERSE walking the BVH (node stack in LDS, interleaved by lane) to the
//            next candidate patch, nearest child first, pruned by the best hit
//   STEP     one subdivision step of Alg. 3 on the current grid
//   GRID     waiting for its grid (and Gregory displacement) to be recomputed
//            for the current domain: after a backtrack, and after every step
//            on a Gregory patch (Alg. 3 recomputes Gregory bounds at each node)
//   DEAD     the queue is empty
// Each iteration of the wave's loop runs the split step for the STEP lanes and
// runs a fetch, a traversal or a recompute phase only when at least a given
// number of lanes waits for it (or no lane could step otherwise), so that the
// expensive, divergent phases run on well-filled waves.  Which lane holds which
// ray, and when, never changes a ray's result.
//
// Alg. 3 state per lane (registers only, no stack):
//   code  interleaved path bits of the current domain; split k (u at even k)
//         owns bit 2L-1-k and is set when the upper half was taken;
//   trail same bit layout; a set bit marks a pending sibling (both halves hit);
//   depth number of splits on the path (next axis: u iff depth is even);
//   G     the current grid (lower bounding grid for a Gregory patch), held so
//         that the split runs along its first index; mirror bits per axis;
//   d     the Gregory displacement of the current domain (0 for Bezier).
// Backtracking takes the lowest set trail bit (the deepest pending level, one
// count-trailing-zeros for both axes at once), flips that path bit and clears
// the bits below it.  A pair of leaf children is resolved at its parent: the
// closer one hit is recorded, its sibling cannot be closer (Sec. 3.3).

#include <algorithm>

#include "ccs_internal.h"
#include "patch_math.h"
#include "policy.h"
#include "ray_valid.h"

namespace ccs {

constexpr int kBlock = 64;
constexpr uint32_t kGridOwners = kBlock / 3;  // lanes whose grids one recompute phase serves

enum Mode : int { kFetch = 0, kTraverse = 1, kStep = 2, kGrid = 3, kDead = 4, kDecide = 5 };

struct Counts {
  uint32_t node, cand, split, backtrack, greg, leaf, crop, cand_greg;
};


// Batch of launch ray k (a wave-uniform scan: the table is never indexed per lane).
__device__ __forceinline__ uint32_t batch_of(const BatchTable& bt, uint32_t k) {
  uint32_t b = 0;
  for (uint32_t q = 1; q < bt.n_batches; ++q) b = k >= bt.prefix[q] ? q : b;
  return b;
}

template <bool kStats>
__device__ __forceinline__ void write_hit(const BatchTable& bt, uint32_t* __restrict__ counters, uint32_t rid,
                                          float best_t, uint32_t best_id, float u, float v, const Counts& cnt) {
  const bool hit = best_id != kNoHit;
  float4 h;
  h.x = hit ? best_t : __builtin_inff();
  h.y = __uint_as_float(best_id);
  h.z = hit ? u : 0.0f;
  h.w = hit ? v : 0.0f;
  ccs_hit* hits = bt.hits[0];
  uint32_t local = rid;
  for (uint32_t q = 1; q < bt.n_batches; ++q)
    if (rid >= bt.prefix[q]) {
      hits = bt.hits[q];
      local = rid - bt.prefix[q];
    }
  reinterpret_cast<float4*>(hits)[local] = h;
  if (kStats) {
    uint4* c = reinterpret_cast<uint4*>(counters + 8 * (size_t)rid);
    c[0] = make_uint4(cnt.node, cnt.cand, cnt.split, cnt.backtrack);
    c[1] = make_uint4(cnt.greg, cnt.leaf, cnt.crop, cnt.cand_greg);
  }
}

// kLearned: the child-ordering network picks the u-half at decision nodes
// (policy.h).  The lane first descends the closest-first way, stores the
// node's policy inputs and waits in DECIDE; the wave then runs the network for
// all waiting lanes on the matrix cores.  A lane whose network prefers the other
// u-half flips that level's path bit (its trail bit stays set, so the
// closest-first half becomes the pending sibling) and has its grid recomputed;
// one split later it takes the v-half of the network's top grandchild when both
// v-halves are hit.
// Three waves per SIMD (at most 168 VGPRs): the closest-first variant fits by
// itself; the learned variant is held to it (a few loop-invariant values of the
// ray-fetch and leaf-record paths then live in scratch instead of registers).
//
// kSingle (the ablation of Sec. 3.3's two-box test, closest-first kernels only):
// a step tests only the box of the current domain (the hull of its grid, grown by
// its own displacement) and, when it is hit above the leaf depth, splits and
// enters the lower half with the upper one pending; a missed box backtracks, and
// a hit leaf box is recorded at its own entry distance.  No distance orders the
// halves, and every pending half costs a grid recompute.
template <bool kStats, bool kLearned, bool kSingle, typename CodeT>
__device__ __forceinline__ void trace_body(DeviceScene s, BatchTable bt, uint32_t* __restrict__ counters,
                                           LaunchParams lp) {
  constexpr int kStack = kLearned ? (int)kMaxBvhDepthLearned : (int)kMaxBvhDepth;
  __shared__ int stack[kStack * kBlock];
  // learned order, 16 words per lane: the node's corners and slab results from the
  // split until the decision, then the network's inputs, then its logits; and the
  // node's mirror bits
  __shared__ __align__(16) uint32_t s_feat[kLearned ? 64 * 16 : 4];
  __shared__ uint8_t s_mirror[kLearned ? 64 : 4];
  __shared__ float s_dir[3][kBlock];  // world direction: read only when a candidate is set up
  __shared__ float s_uv[2][kBlock];   // (u, v) of the best hit: written only by leaf records
  const int lane = threadIdx.x;
  const int L2 = 2 * s.leaf_depth;
  const float leaf_scale = __uint_as_float((uint32_t)(127 - s.leaf_depth) << 23);  // 2^-L

  const uint32_t n = bt.prefix[bt.n_batches];
  int mode = kFetch;
  uint32_t rid = 0;
  const float4* nodes = s.nodes;  // the current ray's frame
  const float* recs = s.recs;
  RayP wr = {0, 0, 0, 0, 0, 0, 0};  // world frame
  float pox = 0.0f, poy = 0.0f, poz = 0.0f, ptmin = 0.0f;  // origin and tmin in the current patch frame
  float pt0 = 0.0f;                                         // ray parameter of the patch frame's origin
  float best_t = 0.0f;
  uint32_t best_id = kNoHit;
  Counts cnt = {0, 0, 0, 0, 0, 0, 0, 0};
  int cur = 0, sp = 0;
  uint32_t rec_idx = 0, pmeta = 0;  // current patch record and its meta bits (index | Gregory bit)
  Grid G;
  float dx = 0.0f, dy = 0.0f, dz = 0.0f;
  CodeT code = 0, trail = 0;  // 32 bits for L <= 16, 64 bits beyond
  uint32_t mirror = 0;
  int depth = 0;
  uint32_t vpref = 0;  // learned order: bit 0 set = take the v-half in bit 1 at the next split
  float pad2 = 0.0f;   // patch-local frames: twice the current patch's box pad (added to d)
  float pix = 0.0f, piy = 0.0f, piz = 0.0f;  // reciprocal direction in the current patch's frame

  for (;;) {
    if (__ballot(mode != kDead) == 0) break;
    uint64_t mf = __ballot(mode == kFetch);
    uint64_t mt = __ballot(mode == kTraverse);
    uint64_t ms = __ballot(mode == kStep);
    uint64_t mg = __ballot(mode == kGrid);
    if (kLearned) ms |= __ballot(mode == kDecide);  // lanes that will step once decided

    // Wave priority: a wave in the fetch or traversal phase is about to wait on a
    // chain of dependent loads (queue atomic and ray, or node after node), so it
    // issues ahead of waves in the arithmetic phases of the same SIMD and its loads
    // leave earlier; results do not depend on it.
    __builtin_amdgcn_s_setprio(1);
    // ------------------------------------------------------------ fetch rays
    if (mf != 0 && ((uint32_t)__popcll(mf) >= lp.fetch_min || (mt | ms | mg) == 0)) {
      const int leader = __ffsll((unsigned long long)mf) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(lp.queue, (uint32_t)__popcll(mf));
      base = __shfl(base, leader);
      if (mode == kFetch) {
        rid = base + (uint32_t)__popcll(mf & ((1ull << lane) - 1ull));
        if (rid >= n) {
          mode = kDead;
        } else {
          const ccs_ray* rays = bt.rays[0];
          uint32_t local = rid, frame = bt.frame[0];
          for (uint32_t q = 1; q < bt.n_batches; ++q)
            if (rid >= bt.prefix[q]) {
              rays = bt.rays[q];
              local = rid - bt.prefix[q];
              frame = bt.frame[q];
            }
          nodes = s.nodes + (size_t)frame * s.frame_node_f4;
          recs = s.recs + (size_t)frame * s.frame_rec_floats;
          const float4* r4 = reinterpret_cast<const float4*>(rays + local);
          const float4 ro = r4[0], rd = r4[1];
          const bool valid = ray_traced(ro, rd) && s.n_nodes > 0;
          best_t = rd.w;
          best_id = kNoHit;
          if (kStats) cnt = Counts{0, 0, 0, 0, 0, 0, 0, 0};
          if (!valid) {
            write_hit<kStats>(bt, counters, rid, best_t, best_id, 0.0f, 0.0f, cnt);
          } else {
            wr.ox = ro.x;
            wr.oy = ro.y;
            wr.oz = ro.z;
            wr.ix = safe_inv(rd.x);
            wr.iy = safe_inv(rd.y);
            wr.iz = safe_inv(rd.z);
            wr.tmin = ro.w;
            s_dir[0][lane] = rd.x;
            s_dir[1][lane] = rd.y;
            s_dir[2][lane] = rd.z;
            cur = 0;
            sp = 0;
            mode = kTraverse;
          }
        }
      }
      mt = __ballot(mode == kTraverse);
    }

    __builtin_amdgcn_s_setprio(2);
    // ------------------------------------------- traverse to the next candidate
    if (mt != 0 && ((uint32_t)__popcll(mt) >= lp.traverse_min || (ms | mg) == 0)) {
      // at most traverse_steps node visits per phase: lanes still walking keep their
      // place and continue next time, so one lane's long walk does not hold the wave
      for (uint32_t it = 0; mode == kTraverse && it < lp.traverse_steps; ++it) {
        if (cur < 0) {  // candidate patch: set up Alg. 3 at the root
          if (kStats) cnt.cand++;
          rec_idx = (uint32_t)(~cur);
          const float* rec = recs + (size_t)rec_idx * kRecFloats;
          const float4 meta = reinterpret_cast<const float4*>(rec)[15];
          pmeta = __float_as_uint(meta.w);
          if (s.frames) {
            // patch-local frame: origin and direction mapped by the patch's rows
            const float4* fr = s.frames + (size_t)bt.frame[batch_of(bt, rid)] * s.frame_frames_f4 + 3 * (size_t)rec_idx;
            const float4 r0 = fr[0], r1 = fr[1], r2 = fr[2];
            float pdx, pdy, pdz;
            patch_frame_rows(meta, r0, r1, r2, wr.ox, wr.oy, wr.oz, s_dir[0][lane], s_dir[1][lane], s_dir[2][lane],
                             wr.tmin, pox, poy, poz, pdx, pdy, pdz, ptmin, pt0);
            pix = safe_inv(pdx);
            piy = safe_inv(pdy);
            piz = safe_inv(pdz);
            // boxes grown by the pad on all sides: the low planes move by -pad through the
            // origin (o + pad), the high planes by +pad through d + 2 pad
            pox += r0.w;
            poy += r0.w;
            poz += r0.w;
            pad2 = 2.0f * r0.w;
          } else {
            patch_frame(meta, wr.ox, wr.oy, wr.oz, s_dir[0][lane], s_dir[1][lane], s_dir[2][lane], wr.tmin, pox,
                        poy, poz, ptmin, pt0);
            pix = wr.ix;
            piy = wr.iy;
            piz = wr.iz;
          }
          code = trail = 0;
          mirror = 0;
          depth = 0;
          if (pmeta & kGregoryBit) {
            if (kStats) cnt.cand_greg++;
            mode = kGrid;
          } else {
            PatchPts P;
            load_grid(rec, P, false);
            orient(P.x, false, G.x);
            orient(P.y, false, G.y);
            orient(P.z, false, G.z);
            dx = dy = dz = pad2;
            mode = kStep;
          }
          break;
        }
        if (kStats) cnt.node++;
        const float4* nd = nodes + 4 * (size_t)cur;
        const float4 a = nd[0], b = nd[1], c = nd[2], e = nd[3];
        const int c0 = __float_as_int(e.x), c1 = __float_as_int(e.y);
        // the cap is widened by a few ulps so that a box entered at the best distance
        // itself is never lost to rounding (equal distances go to the lower patch id)
        const float capw = best_t + fabsf(best_t) * 0x1p-21f;
        const float t0 = slab(wr, a.x, a.y, a.z, a.w, b.x, b.y, capw);
        const float t1 = slab(wr, b.z, b.w, c.x, c.y, c.z, c.w, capw);
        const bool h0 = t0 != __builtin_inff(), h1 = t1 != __builtin_inff();
        if (h0 && h1) {
          const bool first1 = t1 < t0;
          // the host rejects BVHs deeper than kStack, so sp < kStack always holds here
          if (sp < kStack) {
            stack[sp * kBlock + lane] = first1 ? c0 : c1;
            ++sp;
          }
          cur = first1 ? c1 : c0;
        } else if (h0 || h1) {
          cur = h0 ? c0 : c1;
        } else if (sp > 0) {
          --sp;
          cur = stack[sp * kBlock + lane];
        } else {
          write_hit<kStats>(bt, counters, rid, best_t, best_id, s_uv[0][lane], s_uv[1][lane], cnt);
          mode = kFetch;
        }
      }
      ms = __ballot(mode == kStep);
      if (kLearned) ms |= __ballot(mode == kDecide);
      mg = __ballot(mode == kGrid);
    }

    __builtin_amdgcn_s_setprio(0);
    // ---------------------------------------------- recompute grids in a batch
    // Three lanes per waiting lane: the lane of rank r among those waiting (the
    // owner) has the x, y and z components of its grid computed by lanes 3r, 3r+1
    // and 3r+2 (helpers, whatever their own mode), each with the arithmetic of
    // calc_points_and_d for its component, and pulls them back.  At most
    // kGridOwners lanes are served per phase; the others wait for the next one.
    if (mg != 0 && ((uint32_t)__popcll(mg) >= lp.grid_min || ms == 0)) {
      const uint32_t n_wait = (uint32_t)__popcll(mg);
      const uint32_t n_own = n_wait < kGridOwners ? n_wait : kGridOwners;
      const uint32_t rank = (uint32_t)__popcll(mg & ((1ull << lane) - 1ull));
      const bool owner = mode == kGrid && rank < n_own;
      // lanes past the helpers compute owner 0's grid again (the instructions run for the
      // whole wave anyway; their results are never pulled)
      const uint32_t hr0 = (uint32_t)lane / 3u, hc = (uint32_t)lane - 3u * hr0;
      const uint32_t hr = hr0 < n_own ? hr0 : 0u;
      // the owner's record, path code, depth and type, read by its helpers
      const int from = (int)nth_set_bit(mg, hr) * 4;
      const uint64_t rp = reinterpret_cast<uint64_t>(recs + (size_t)rec_idx * kRecFloats);
      const uint32_t dg = (uint32_t)depth | ((pmeta & kGregoryBit) ? 0x100u : 0u);
      const uint32_t h_lo = (uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)(uint32_t)rp);
      const uint32_t h_hi = (uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)(uint32_t)(rp >> 32));
      CodeT h_code = (uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)(uint32_t)code);
      if constexpr (sizeof(CodeT) == 8)
        h_code |= (CodeT)(uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)(uint32_t)(code >> 32)) << 32;
      const uint32_t h_dg = (uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)dg);
      float qo[4][4], dc;
      {
        const float* hrec = reinterpret_cast<const float*>(((uint64_t)h_hi << 32) | h_lo);
        const int hd = (int)(h_dg & 0xFFu);
        // domain of the node at depth hd: position from the path code, sizes from the depth
        const float u0 = (float)compact_even(h_code >> 1) * leaf_scale;
        const float v0 = (float)compact_even(h_code) * leaf_scale;
        const float su = __uint_as_float((uint32_t)(127 - ((hd + 1) >> 1)) << 23);
        const float sv = __uint_as_float((uint32_t)(127 - (hd >> 1)) << 23);
        float q[4][4];
        calc_component(hrec + 16 * hc, hrec + 48 + 4 * hc, (h_dg & 0x100u) != 0, u0, u0 + su, v0, v0 + sv, q, dc);
        orient(q, (hd & 1) != 0, qo);
      }
      const int to = owner ? (int)(12u * rank) : 0;  // byte index of the owner's x helper
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int v = __float_as_int(qo[a][b]);
          const float gx = __int_as_float(__builtin_amdgcn_ds_bpermute(to, v));
          const float gy = __int_as_float(__builtin_amdgcn_ds_bpermute(to + 4, v));
          const float gz = __int_as_float(__builtin_amdgcn_ds_bpermute(to + 8, v));
          G.x[a][b] = owner ? gx : G.x[a][b];
          G.y[a][b] = owner ? gy : G.y[a][b];
          G.z[a][b] = owner ? gz : G.z[a][b];
        }
      const float ddx = __int_as_float(__builtin_amdgcn_ds_bpermute(to, __float_as_int(dc)));
      const float ddy = __int_as_float(__builtin_amdgcn_ds_bpermute(to + 4, __float_as_int(dc)));
      const float ddz = __int_as_float(__builtin_amdgcn_ds_bpermute(to + 8, __float_as_int(dc)));
      if (owner) {
        dx = ddx + pad2;  // pad2 is 0 outside patch-local frames
        dy = ddy + pad2;
        dz = ddz + pad2;
        mirror = 0;
        mode = kStep;
        if (kStats) {
          if (pmeta & kGregoryBit)
            cnt.greg++;
          else
            cnt.crop++;
        }
      }
    }

    // ----------------------------- learned order: the network for waiting lanes
    if (kLearned) {
      const uint64_t md = __ballot(mode == kDecide);
      const uint32_t n_dec = (uint32_t)__popcll(md);
      if (md != 0 && (n_dec >= lp.decide_min || __ballot(mode == kStep) == 0)) {
        // deciding lanes take consecutive slots, so the network runs on ceil(n / 16)
        // column tiles instead of every tile holding one of them (all slot reads of
        // the node values precede the first input store in the wave's program order)
        const uint32_t slot = (uint32_t)__popcll(md & ((1ull << lane) - 1ull));
        if (mode == kDecide) {
          // inputs of the node one level up (the u-split just taken), with the direction in
          // the frame the patch is subdivided in
          const float fdx = s.frames ? __builtin_amdgcn_rcpf(pix) : s_dir[0][lane];
          const float fdy = s.frames ? __builtin_amdgcn_rcpf(piy) : s_dir[1][lane];
          const float fdz = s.frames ? __builtin_amdgcn_rcpf(piz) : s_dir[2][lane];
          float f[16];
          policy_features(policy_load_node(s_feat, lane, s_mirror[lane]), pox, poy, poz, fdx, fdy, fdz, depth - 1,
                          s.leaf_depth, (pmeta & kGregoryBit) != 0, f);
          policy_store_inputs<16>(s_feat, (int)slot, f);
        }
        const uint64_t need = n_dec >= 64 ? ~0ull : (1ull << n_dec) - 1ull;
        policy_wave<16>(s.policy, s_feat, need, lane);  // the whole wave: matrix-core operands span all lanes
        if (mode == kDecide) {
          const float4 lg = reinterpret_cast<const float4*>(s_feat)[4 * slot];
          const uint32_t top = policy_top(lg.x, lg.y, lg.z, lg.w);
          const CodeT bit = (CodeT)1 << (L2 - depth);  // path bit of the u-split just taken
          vpref = 1u | ((top & 1u) << 1);
          if (((top >> 1) != 0) != ((code & bit) != 0)) {
            code ^= bit;  // the other u-half first; the trail bit keeps the closest-first one pending
            mode = kGrid;
          } else {
            mode = (pmeta & kGregoryBit) ? kGrid : kStep;
          }
        }
      }
    }

    // -------------------------------------------------- one subdivision step
    if (mode == kStep) {
      if (kStats) cnt.split++;
      bool backtrack;
      if constexpr (kSingle) {
        // the box of the current domain only: its grid's hull, the maximum side grown
        // by the domain's own displacement
        SlabPair one = {ptmin, __builtin_inff(), ptmin, __builtin_inff()};
        grid_fold(G.x, pox, pix, dx, one);
        grid_fold(G.y, poy, piy, dy, one);
        grid_fold(G.z, poz, piz, dz, one);
        const float cap = (best_t - pt0) + (fabsf(best_t) + fabsf(pt0)) * 0x1p-22f;
        const bool hit = one.na <= fminf(widen_far(one.fa), cap);
        backtrack = true;
        if (hit && depth == L2) {
          const float tf = pt0 + one.na;
          const uint32_t pid = pmeta & kIdMask;
          if (tf < best_t || (tf == best_t && pid < best_id)) {
            best_t = tf;
            best_id = pid;
            s_uv[0][lane] = (float)(2u * compact_even(code >> 1) + 1u) * (0.5f * leaf_scale);
            s_uv[1][lane] = (float)(2u * compact_even(code) + 1u) * (0.5f * leaf_scale);
            if (kStats) cnt.leaf++;
          }
        } else if (hit) {
          // split and enter the lower half, the upper one pending
          const int axis = depth & 1;
          const bool second = ((mirror >> axis) & 1u) != 0;  // the lower half is register-second when mirrored
          Row7 ex[4], ey[4], ez[4];
          SlabPair unused = {0.0f, 0.0f, 0.0f, 0.0f};
          split_fold(G.x, 0.0f, 1.0f, 0.0f, ex, unused);
          split_fold(G.y, 0.0f, 1.0f, 0.0f, ey, unused);
          split_fold(G.z, 0.0f, 1.0f, 0.0f, ez, unused);
          take_half(ex, second, G.x);
          take_half(ey, second, G.y);
          take_half(ez, second, G.z);
          trail |= (CodeT)1 << (L2 - 1 - depth);
          if (second) mirror ^= (1u << axis);
          depth++;
          backtrack = false;
          if (pmeta & kGregoryBit) mode = kGrid;  // the child's own bound (Alg. 2 on its domain)
        }
      } else {
        // split each component and fold its two child boxes into the slab test at once
        Row7 ex[4], ey[4], ez[4];
        SlabPair sp2 = {ptmin, __builtin_inff(), ptmin, __builtin_inff()};
        split_fold(G.x, pox, pix, dx, ex, sp2);
        split_fold(G.y, poy, piy, dy, ey, sp2);
        split_fold(G.z, poz, piz, dz, ez, sp2);
        // the best distance in the patch frame: best_t - pt0 carries the rounding of
        // best_t = pt0 + t and of the difference (each at most 2^-24 relative), so it
        // is widened by twice their bound and a leaf at the best distance is never pruned
        const float cap = (best_t - pt0) + (fabsf(best_t) + fabsf(pt0)) * 0x1p-22f;
        const float fa = fminf(widen_far(sp2.fa), cap), fb = fminf(widen_far(sp2.fb), cap);
        const bool ha = sp2.na <= fa, hb = sp2.nb <= fb;
        const float ta = sp2.na, tb = sp2.nb;
        const int axis = depth & 1;
        const bool mir = ((mirror >> axis) & 1u) != 0;
        const bool h_lo = mir ? hb : ha, h_up = mir ? ha : hb;
        const float t_lo = mir ? tb : ta, t_up = mir ? ta : tb;
        bool go_up = h_up && (!h_lo || t_up < t_lo);
        const CodeT bit = (CodeT)1 << (L2 - 1 - depth);
        const uint32_t mirror0 = mirror;
        bool decide = false;
        if (kLearned) {
          // v-split after a decision: the network's v-half when both are hit (not at the
          // leaf pair, which is resolved by distance)
          if ((vpref & 1u) && axis == 1 && ha && hb && depth != L2 - 1) go_up = (vpref & 2u) != 0;
          vpref = 0;
          decide = axis == 0 && ha && hb;
        }
        // the chosen half replaces the grid on every path: when the lane backtracks or
        // leaves the patch instead, the grid is rebuilt before it is read again
        const bool second = go_up != mir;
        if (kLearned && decide) {
          // the node's corners in storage order (0,0), (3,0), (0,3), (3,3) and its slab
          // results, kept for the decision (formed there, off this phase's registers)
          const float sx[4] = {ex[0].v[0], ex[0].v[6], ex[3].v[0], ex[3].v[6]};
          const float sy[4] = {ey[0].v[0], ey[0].v[6], ey[3].v[0], ey[3].v[6]};
          const float sz[4] = {ez[0].v[0], ez[0].v[6], ez[3].v[0], ez[3].v[6]};
          policy_store_node(s_feat, lane, sx, sy, sz, sp2);
          s_mirror[lane] = (uint8_t)mirror0;
        }
        take_half(ex, second, G.x);
        take_half(ey, second, G.y);
        take_half(ez, second, G.z);
        backtrack = !(ha || hb);
        if (!backtrack) {
          if (depth == L2 - 1) {
            const float tf = pt0 + (go_up ? t_up : t_lo);
            const uint32_t pid = pmeta & kIdMask;
            if (tf < best_t || (tf == best_t && pid < best_id)) {
              const CodeT lc = code | (go_up ? bit : (CodeT)0);
              best_t = tf;
              best_id = pid;
              s_uv[0][lane] = (float)(2u * compact_even(lc >> 1) + 1u) * (0.5f * leaf_scale);
              s_uv[1][lane] = (float)(2u * compact_even(lc) + 1u) * (0.5f * leaf_scale);
              if (kStats) cnt.leaf++;
            }
            backtrack = true;
          } else {
            if (ha && hb) trail |= bit;
            if (go_up) code |= bit;
            if (second) mirror ^= (1u << axis);
            depth++;
            if (pmeta & kGregoryBit) mode = kGrid;  // Alg. 3 recomputes a Gregory grid at every node
            if (kLearned && decide) mode = kDecide;
          }
        }
      }
      if (backtrack) {
        if (trail != 0) {
          const int b = sizeof(CodeT) == 8 ? __builtin_ctzll((uint64_t)trail) : __builtin_ctz((uint32_t)trail);
          const CodeT tb_bit = (CodeT)1 << b;
          trail ^= tb_bit;
          code = (code ^ tb_bit) & ~(tb_bit - 1);
          depth = L2 - b;
          mode = kGrid;
          if (kStats) cnt.backtrack++;
        } else {
          if (sp > 0) {  // next candidate from the stack
            --sp;
            cur = stack[sp * kBlock + lane];
            mode = kTraverse;
          } else {  // ray done
            write_hit<kStats>(bt, counters, rid, best_t, best_id, s_uv[0][lane], s_uv[1][lane], cnt);
            mode = kFetch;
          }
        }
      }
    }
  }
}

template <bool kStats, bool kLearned>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_trace(DeviceScene s, BatchTable bt, uint32_t* __restrict__ counters,
                                                  LaunchParams lp) {
  trace_body<kStats, kLearned, false, uint32_t>(s, bt, counters, lp);
}

// Leaf depths above 16: the path and trail words in 64 bits (closest-first order only).
template <bool kStats>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_trace_deep(
    DeviceScene s, BatchTable bt, uint32_t* __restrict__ counters, LaunchParams lp) {
  trace_body<kStats, false, false, uint64_t>(s, bt, counters, lp);
}

template <bool kStats>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_trace_single_box(
    DeviceScene s, BatchTable bt, uint32_t* __restrict__ counters, LaunchParams lp) {
  trace_body<kStats, false, true, uint32_t>(s, bt, counters, lp);
}

// Grid of a subdomain by both of the kernel's routes, for measuring their fp32
// deviation (Sec. 3.4 compares recomputed control points with subdivided ones).
// One thread per query q = (patch record, path code, depth), with the path code
// laid out as in k_trace.  Output row of kDebugGridFloats floats:
//   [0, 60)    the record's stored points: x, y, z of slots 0..15, then x, y, z of P^v
//   [60, 108)  calcPointsAndD on the domain, as the grid phase computes it (one
//              component at a time): x, y, z of q[i][j] at 16 c + 4 j + i
//   [108, 111) its displacement d
//   [111, 159) Bezier patches: the root grid split depth times along the path by
//              the split step's arithmetic (de Casteljau halves, transposed and
//              mirrored write-back), un-oriented to the same layout; NaN for Gregory
//   [159]      0 for a valid query, NaN when the query is out of range
template <int kF>
__device__ __forceinline__ void store_canonical(float* out, const float g[4][4], bool odd, uint32_t mirror, int c) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      // register (a, b): a runs along the next split's axis (u at even depth)
      const int ra = odd ? b : a, rb = odd ? a : b;  // register indices along u, along v
      const int i = (mirror & 1u) ? 3 - ra : ra, j = (mirror & 2u) ? 3 - rb : rb;
      out[kF + 16 * c + 4 * j + i] = g[a][b];
    }
}

__global__ __launch_bounds__(64) void k_debug_grids(DeviceScene s, const uint32_t* __restrict__ patch,
                                                    const uint32_t* __restrict__ code_in,
                                                    const uint32_t* __restrict__ depth_in, uint32_t n,
                                                    float* __restrict__ out) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float* o = out + (size_t)q * kDebugGridFloats;
  const uint32_t pid = patch[q], code = code_in[q], depth = depth_in[q];
  const int L2 = 2 * s.leaf_depth;
  // the path code holds bits for the depth splits taken and none below or above them
  const bool valid = pid < s.n_patches && depth <= (uint32_t)L2 &&
                     ((uint64_t)code & ((1ull << (L2 - (int)depth)) - 1ull)) == 0 && ((uint64_t)code >> L2) == 0;
  if (!valid) {
    for (int k = 0; k < kDebugGridFloats; ++k) o[k] = __uint_as_float(0x7FC00000u);
    return;
  }
  const float* rec = s.recs + (size_t)s.inv_perm[pid] * kRecFloats;
  for (int k = 0; k < 60; ++k) o[k] = rec[k];
  const bool greg = (__float_as_uint(rec[63]) & kGregoryBit) != 0;
  const float leaf_scale = __uint_as_float((uint32_t)(127 - s.leaf_depth) << 23);
  const float u0 = (float)compact_even(code >> 1) * leaf_scale, v0 = (float)compact_even(code) * leaf_scale;
  const float su = __uint_as_float((uint32_t)(127 - (((int)depth + 1) >> 1)) << 23);
  const float sv = __uint_as_float((uint32_t)(127 - ((int)depth >> 1)) << 23);
  for (int c = 0; c < 3; ++c) {
    float qc[4][4], dc;
    calc_component(rec + 16 * c, rec + 48 + 4 * c, greg, u0, u0 + su, v0, v0 + sv, qc, dc);
    store_canonical<60>(o, qc, false, 0u, c);
    o[108 + c] = dc;
  }
  if (greg) {
    for (int k = 111; k < 159; ++k) o[k] = __uint_as_float(0x7FC00000u);
  } else {
    PatchPts P;
    load_grid(rec, P, false);
    Grid G;
    orient(P.x, false, G.x);
    orient(P.y, false, G.y);
    orient(P.z, false, G.z);
    uint32_t mirror = 0;
    for (uint32_t k = 0; k < depth; ++k) {
      const int axis = (int)(k & 1u);
      const bool up = (code >> (L2 - 1 - (int)k)) & 1u;
      const bool mir = ((mirror >> axis) & 1u) != 0;
      Row7 ex[4], ey[4], ez[4];
      SlabPair sp2 = {0.0f, 0.0f, 0.0f, 0.0f};  // the slab results are not used here
      split_fold(G.x, 0.0f, 1.0f, 0.0f, ex, sp2);
      split_fold(G.y, 0.0f, 1.0f, 0.0f, ey, sp2);
      split_fold(G.z, 0.0f, 1.0f, 0.0f, ez, sp2);
      const bool second = up != mir;
      take_half(ex, second, G.x);
      take_half(ey, second, G.y);
      take_half(ez, second, G.z);
      if (second) mirror ^= 1u << axis;
    }
    const bool odd = (depth & 1u) != 0;
    store_canonical<111>(o, G.x, odd, mirror, 0);
    store_canonical<111>(o, G.y, odd, mirror, 1);
    store_canonical<111>(o, G.z, odd, mirror, 2);
  }
  o[159] = 0.0f;
}

hipError_t launch_debug_grids(const DeviceScene& s, const uint32_t* patch, const uint32_t* code,
                              const uint32_t* depth, uint32_t n, float* out, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_grids, dim3((n + 63) / 64), dim3(64), 0, stream, s, patch, code, depth, n, out);
  return hipGetLastError();
}

__global__ void k_queue_reset(uint32_t* q) { *q = 0u; }

template <bool kStats, bool kLearned, bool kSingle, bool kDeep>
static int resident_waves_per_cu() {
  static int per_cu = -1;
  if (per_cu < 0) {
    int v = 0;
    if (kSingle)
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_trace_single_box<kStats>, kBlock, 0);
    else if (kDeep)
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_trace_deep<kStats>, kBlock, 0);
    else
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_trace<kStats, kLearned>, kBlock, 0);
    per_cu = std::max(1, v);
  }
  return per_cu;
}

int max_waves_per_cu(bool counted, bool learned, bool single_box, bool deep) {
  if (single_box)
    return counted ? resident_waves_per_cu<true, false, true, false>() : resident_waves_per_cu<false, false, true, false>();
  if (learned)
    return counted ? resident_waves_per_cu<true, true, false, false>() : resident_waves_per_cu<false, true, false, false>();
  if (deep)
    return counted ? resident_waves_per_cu<true, false, false, true>() : resident_waves_per_cu<false, false, false, true>();
  return counted ? resident_waves_per_cu<true, false, false, false>() : resident_waves_per_cu<false, false, false, false>();
}

hipError_t launch_intersect(const DeviceScene& s, const BatchTable& bt, uint32_t* counters, const LaunchParams& lp,
                            uint32_t waves_per_cu, hipStream_t stream) {
  const uint32_t n = bt.prefix[bt.n_batches];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, stream, lp.queue);
  // the host refuses the learned order and the single-box ablation above kMaxLeafDepth32
  const bool deep = s.leaf_depth > (int)kMaxLeafDepth32;
  const bool learned = s.policy.w != nullptr && !s.single_box && !deep;
  int per_cu = max_waves_per_cu(counters != nullptr, learned, s.single_box && !deep, deep);
  if (waves_per_cu > 0) per_cu = std::min(per_cu, (int)waves_per_cu);
  const uint32_t waves = (uint32_t)(per_cu * s.n_cus);
  const uint32_t needed = (n + kBlock - 1) / kBlock;
  const dim3 grid(std::min(waves, needed)), block(kBlock);
  if (deep) {
    if (counters)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace_deep<true>), grid, block, 0, stream, s, bt, counters, lp);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace_deep<false>), grid, block, 0, stream, s, bt, nullptr, lp);
  } else if (s.single_box) {
    if (counters)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace_single_box<true>), grid, block, 0, stream, s, bt, counters, lp);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace_single_box<false>), grid, block, 0, stream, s, bt, nullptr, lp);
  } else if (learned) {
    if (counters)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace<true, true>), grid, block, 0, stream, s, bt, counters, lp);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace<false, true>), grid, block, 0, stream, s, bt, nullptr, lp);
  } else {
    if (counters)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace<true, false>), grid, block, 0, stream, s, bt, counters, lp);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_trace<false, false>), grid, block, 0, stream, s, bt, nullptr, lp);
  }
  return hipGetLastError();
}

}  // namespace ccs
