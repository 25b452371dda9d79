/*
 * ccs.h -- closest-hit ray intersection with Catmull-Clark subdivision surfaces
 * in patch form (bicubic Bezier and Gregory patches) on AMD Instinct MI355X.
 *
 * The method is the stackless hierarchical subdivision of Binder & Keller,
 * "Massively Parallel Stackless Ray Tracing of Catmull-Clark Subdivision
 * Surfaces" (arXiv:1811.03510): a BVH over patch bounds (Sec. 4, results
 * discussion), then per candidate patch the bit-trail subdivision of Alg. 3 with
 * Bezier bounds on subdomains (Sec. 3.1, Alg. 1) and Gregory bounds from Alg. 2
 * (Sec. 3.2).  The reported hit is the entry distance into the closest leaf box
 * together with the centre of the leaf's parameter domain: Sec. 3 states that
 * intersecting the nested boxes alone yields the intersection up to almost
 * floating-point precision.
 *
 * Conventions shared by every entry point
 *   - Patch input: n x 20 x 3 floats (fp32), patch-major.  Slot s of a patch
 *     holds point s as (x, y, z).  Slots 0..15 are the 4x4 grid,
 *     slot(i, j) = 4*j + i with i along u and j along v (Sec. 3.1).  For a
 *     Gregory patch (Sec. 3.2) slots 5, 6, 9, 10 hold P^u of the inner points
 *     (1,1), (2,1), (1,2), (2,2) and slots 16..19 hold P^v in the same order; the
 *     inner point is (du P^u + dv P^v) / (du + dv) with du = u or 1-u and
 *     dv = v or 1-v for i = 1 or 2 and j = 1 or 2 (the weighting of Alg. 2).
 *     A Bezier patch ignores slots 16..19.
 *   - Patch types: n bytes, CCS_BEZIER (0) or CCS_GREGORY (1).
 *   - Leaf depth L: each patch is subdivided L times along u and L times along v
 *     (alternating, u first, Sec. 3.3); domains are integers in units of 2^-23
 *     (Alg. 3).  1 <= L <= 16.
 *   - Rays: ccs_ray, 32 bytes.  A hit t is in units of the given (not
 *     necessarily unit) direction and lies in [tmin, tmax] (closed).  Rays with a
 *     non-finite origin or direction, a zero direction or tmin > tmax miss.
 *   - Hits: ccs_hit, 16 bytes.  A miss is {t = +inf, patch_id = CCS_NO_HIT,
 *     u = 0, v = 0}.  Among equal distances the smaller patch id wins.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Functions marked asynchronous only enqueue work on that stream.
 *   - Errors: every entry point returns a ccs_status; no exception crosses the
 *     boundary.  ccs_last_error() gives a message for the calling thread.
 */
#ifndef CCS_H
#define CCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CCS_NO_HIT 0xFFFFFFFFu
/* Per-axis leaf depth L.  Alg. 3's domains (units of 2^-23) would allow 22, but the
 * fp32 subdivision's rounding, a few ulps of the patch's extent after 40 splits,
 * then exceeds a leaf box (2^-22 of the extent): at L = 22 rays were measured to
 * pass through surfaces.  Up to 16 the intersection kernels keep a domain's path and
 * trail in 32-bit words; from 17 to 20 in 64-bit words, closest-first order only:
 * the learned order (ccs_scene_set_policy), the single-box ablation
 * (CCS_FLAG_SINGLE_BOX) and ccs_debug_grids return CCS_ERR_UNSUPPORTED there. */
#define CCS_MAX_LEAF_DEPTH 20
/* Scene flag: subdivide every patch in its own frame (Sec. 3.4: boxes in patch-local
 * frames overlap less, so fewer subdomains survive the slab tests).  The frame of a
 * patch has rows r0 = unit(p30 - p00), r1 = unit of (p03 - p00) with its r0 part
 * removed, r2 = r0 x r1 (the identity when the u or v edge is degenerate), computed
 * in double and stored in fp32; patch points and each candidate ray are mapped by
 * it, so ray parameters are unchanged and the subdivision boxes, including the leaf
 * box whose entry distance is reported, are boxes in the patch's frame, each grown
 * on all sides by 2^-19 of the patch's largest extent in that frame (corners and
 * straight edges lie on box faces there, where rounding would open gaps between
 * neighbours; Sec. 3.4 closes them by growing boxes).  The BVH stays in world
 * space.  Frames follow the geometry on refit. */
#define CCS_FLAG_LOCAL_FRAMES 1u
/* Scene flag, for measurement only: each step of Alg. 3 tests only the box of the
 * current domain (its grid's hull, grown by the domain's own displacement for a
 * Gregory patch) instead of the two child boxes of Sec. 3.3; a hit box above the
 * leaf depth is split and its lower half entered with the upper half pending, a
 * missed one backtracks, and a hit leaf box is recorded at its own entry distance.
 * Sec. 3.3 reports that the two-box test nearly halves the traversal time against
 * this.  Results obey the same contract (closest leaf box hit; a Gregory leaf box
 * is then the leaf's own bound).  Closest-first only: ccs_scene_set_policy
 * returns CCS_ERR_UNSUPPORTED on such a scene; leaf depths up to 16. */
#define CCS_FLAG_SINGLE_BOX 2u

typedef enum ccs_status {
  CCS_OK = 0,
  CCS_ERR_INVALID_ARG = 1, /* null pointer, bad tag, L out of range, non-finite input, size mismatch */
  CCS_ERR_OOM = 2,         /* device or host allocation failed, or refused by CCS_MAX_DEVICE_BYTES */
  CCS_ERR_HIP = 3,         /* a HIP runtime call failed; see ccs_last_error() */
  CCS_ERR_UNSUPPORTED = 4  /* no gfx950 device, an unknown flag, or a BVH too deep for a kernel's stack */
} ccs_status;

typedef enum ccs_patch_type { CCS_BEZIER = 0, CCS_GREGORY = 1 } ccs_patch_type;

typedef enum ccs_location { CCS_HOST = 0, CCS_DEVICE = 1 } ccs_location;

/* Ray {o, tmin, d, tmax}: float4-aligned so that one ray is two 16-byte loads. */
typedef struct ccs_ray {
  float ox, oy, oz, tmin;
  float dx, dy, dz, tmax;
} ccs_ray;

/* Closest hit: entry distance into the leaf box, patch index into the input
 * arrays, and the centre (u, v) of the leaf domain (Alg. 3's intersection
 * record (pos, size) expressed as a point). */
typedef struct ccs_hit {
  float t;
  uint32_t patch_id;
  float u, v;
} ccs_hit;

typedef struct ccs_scene ccs_scene;

typedef struct ccs_scene_desc {
  const float* control_points;  /* n x 20 x 3 fp32, layout above; host or device (see location) */
  const uint8_t* patch_types;   /* n tags; same location as control_points */
  uint32_t n_patches;           /* 0 <= n < 2^31; an empty scene makes every ray miss */
  int32_t location;             /* CCS_HOST or CCS_DEVICE */
  uint32_t leaf_depth;          /* L, 1..CCS_MAX_LEAF_DEPTH (20) */
  uint32_t flags;               /* 0, or CCS_FLAG_LOCAL_FRAMES and/or CCS_FLAG_SINGLE_BOX */
  void* stream;                 /* hipStream_t used for the uploads */
} ccs_scene_desc;

typedef struct ccs_scene_info {
  uint32_t n_patches;
  uint32_t n_nodes;       /* BVH nodes (binary, one patch per leaf) */
  uint32_t leaf_depth;
  uint32_t bvh_depth;     /* deepest leaf */
  uint64_t device_bytes;  /* device memory owned by the scene */
  float lo[3], hi[3];     /* scene bounds (union of patch boxes) */
  double build_seconds;   /* host BVH build time */
  uint32_t n_frames;      /* geometry frames held (animation playback) */
} ccs_scene_info;

/* Builds a scene (Sec. 3: patch bounds, then a hierarchy over them).
 * Validates on the host: non-null pointers, tags in {0, 1}, 1 <= L <= 16,
 * finite control points (device inputs are copied to the host to be scanned).
 * Computes per patch an anchor (the fp32 centre of its box; Sec. 3.4 anchors
 * patches at the origin for precision), the anchored control points and the
 * hull box of its 16 or 20 points (Sec. 3.1, 3.2), builds a binary BVH with
 * binned SAH splits on the host (Sec. 4), and uploads everything.
 * Synchronous: on return the caller may free its buffers; the scene owns every
 * device buffer it uses.  Errors: CCS_ERR_INVALID_ARG, CCS_ERR_OOM, CCS_ERR_HIP,
 * CCS_ERR_UNSUPPORTED (no gfx950 device).  *out is NULL on error. */
ccs_status ccs_scene_create(const ccs_scene_desc* desc, ccs_scene** out);

/* Moves the control points of an existing scene (animation playback, the use
 * case named in the abstract).  Same n, same tags, same layout as at creation.
 * Anchors stay at their creation values.  On the GPU: anchored points and patch
 * boxes are recomputed, then the BVH node boxes level by level from the deepest
 * (one launch per level); the topology is unchanged.  Asynchronous on `stream`;
 * device input must be 16-byte aligned and stay valid until the stream passes
 * this call.  Host input is staged in a per-scene device buffer and the call
 * returns when the refit is done (synchronous).
 * Host input is scanned for non-finite values (CCS_ERR_INVALID_ARG); device input
 * is not scanned (non-finite points then give unspecified hits, never a fault). */
ccs_status ccs_refit(ccs_scene* scene, const float* control_points, int32_t location, void* stream);

/* Frames (animation playback, the use case named in the abstract): a scene can
 * hold n_frames copies of its patch geometry that share one BVH topology.
 * Frame 0 is the creation geometry; ccs_scene_set_frames copies it into every
 * frame, after which ccs_refit_frame moves one frame's control points.
 * Synchronizes the device; frees and re-allocates the frame storage
 * (n_frames x (256 B per patch + 64 B per node)).  1 <= n_frames <= 4096. */
ccs_status ccs_scene_set_frames(ccs_scene* scene, uint32_t n_frames);

/* ccs_refit applied to one frame (ccs_refit is frame 0). */
ccs_status ccs_refit_frame(ccs_scene* scene, uint32_t frame, const float* control_points, int32_t location,
                           void* stream);

/* One batch of a batched launch: n rays traced against `frame`. */
typedef struct ccs_batch {
  uint32_t frame;
  uint32_t n;
  const ccs_ray* rays;  /* device, n rays */
  ccs_hit* hits;        /* device, n hits */
} ccs_batch;

/* Closest hits of several batches of uneven size, possibly of different
 * frames, in one persistent launch with one ray queue over all of them (no
 * per-batch tail).  batches is a host array of at most 32 entries, copied into
 * the launch's arguments: it may be freed on return, and the launch can be
 * captured in a HIP graph.  Each hit equals what ccs_intersect gives for that
 * ray on that frame.  Asynchronous on `stream`; at most 2^31 - 1 rays. */
ccs_status ccs_intersect_batched(const ccs_scene* scene, const ccs_batch* batches, uint32_t n_batches,
                                 void* stream);

/* As ccs_intersect_batched, with the per-ray work counters of
 * ccs_intersect_counted: counters (device, 8 uint32 per ray) row k belongs to ray
 * k of the launch, the batches' rays taken in order (batch 0's first).  The same
 * separately compiled counting kernel; used for measurement. */
ccs_status ccs_intersect_batched_counted(const ccs_scene* scene, const ccs_batch* batches, uint32_t n_batches,
                                         uint32_t* counters, void* stream);

/* Closest hits of n rays (Alg. 3 per candidate patch, candidates from the BVH
 * nearest first, the best distance so far pruning both).  rays and hits are
 * device pointers owned by the caller; n == 0 is a no-op.  Asynchronous on
 * `stream`.  Deterministic: the result of each ray does not depend on launch
 * geometry or on the other rays.  Each call takes one of 256 per-scene
 * ray-queue counters in turn: at most 256 calls on one scene may be in flight
 * at once (across all streams).  At most 2^31 - 1 rays (CCS_ERR_INVALID_ARG). */
ccs_status ccs_intersect(const ccs_scene* scene, const ccs_ray* rays, uint32_t n, ccs_hit* hits,
                         void* stream);

/* As ccs_intersect, and also writes per-ray work counters (device, n x 8
 * uint32): BVH nodes visited, candidate patches, subdivision steps (Alg. 3
 * splits), backtracks, Gregory bound recomputations (Alg. 2, including each
 * Gregory candidate's root), leaf records, Bezier grid re-crops after
 * backtracking (Alg. 1), Gregory candidates.  A separately compiled copy of the
 * same kernel; used for measurement. */
ccs_status ccs_intersect_counted(const ccs_scene* scene, const ccs_ray* rays, uint32_t n, ccs_hit* hits,
                                 uint32_t* counters, void* stream);

/* Launch configuration of the intersection kernel.  Results never depend on
 * it (each ray's computation is independent of which lane runs it and when);
 * only the speed does.  The kernel keeps persistent waves whose lanes each
 * carry a ray through fetch, traversal, subdivision steps and grid
 * recomputations; a wave runs the fetch, traversal or recompute phase only when
 * at least the given number of its 64 lanes waits for it (or nothing else can
 * run), so that these divergent phases run on filled waves. */
typedef struct ccs_launch_params {
  uint32_t waves_per_cu;   /* resident waves per compute unit; 0 = as many as fit */
  uint32_t fetch_min;      /* 1..64 lanes waiting for a new ray */
  uint32_t traverse_min;   /* 1..64 lanes waiting to traverse to their next candidate */
  uint32_t grid_min;       /* 1..64 lanes waiting for a grid recomputation */
  uint32_t traverse_steps; /* BVH nodes a lane visits per traversal phase; 0 = until it reaches a candidate */
  uint32_t decide_min;     /* 1..64 lanes waiting for the child-ordering network (learned order only) */
} ccs_launch_params;

/* Sets the launch configuration used by later ccs_intersect* calls on the
 * scene.  Defaults: {0, 16, 1, 8, 3, 8}.  CCS_ERR_INVALID_ARG for thresholds
 * outside [1, 64].  Not synchronized with calls in flight on other threads. */
ccs_status ccs_scene_set_launch(ccs_scene* scene, const ccs_launch_params* params);

/* The current launch configuration, waves_per_cu resolved to the number used. */
ccs_status ccs_scene_get_launch(const ccs_scene* scene, ccs_launch_params* params);

/* Secondary rays from hits (Sec. 3.3, self-intersection): for hit i the origin is
 * o + t d moved along the unit normal f_u x f_v at (u, v) (turned against d) by
 * the L1 size of the box of the leaf domain containing (u, v) (Alg. 2 bounds on
 * that domain); the direction is cosine-weighted about the normal from the two
 * uniforms uniforms[2i], uniforms[2i+1] in [0, 1) (Malley's method; polar disk
 * map; tangent frame of Duff et al. 2017).  A miss gives an inactive ray
 * {o = 0, tmin = 0, d = (0, 0, 1), tmax = -1}.  All pointers are device pointers
 * of n elements; out_rays may not alias rays.  Asynchronous on `stream`. */
ccs_status ccs_bounce(const ccs_scene* scene, const ccs_ray* rays, const ccs_hit* hits, const float* uniforms,
                      uint32_t n, ccs_ray* out_rays, void* stream);

/* As ccs_bounce, with the geometry of animation frame `frame` (hits from a
 * ccs_intersect_batched batch on that frame).  CCS_ERR_INVALID_ARG for a frame
 * outside the scene's frames. */
ccs_status ccs_bounce_frame(const ccs_scene* scene, uint32_t frame, const ccs_ray* rays, const ccs_hit* hits,
                            const float* uniforms, uint32_t n, ccs_ray* out_rays, void* stream);

/* Stream compaction of a ray array for path tracing (Sec. 4: each bounce level
 * traces the reflection rays of the previous level's hits; a bounce of a missed
 * ray is inactive, so later levels hold few active rays among many).  Copies the
 * rays of rays[0, n) that the intersection entry points trace -- finite origin
 * and direction, tmin and tmax not NaN, a nonzero direction and tmin <= tmax,
 * decided with fp32 denormals flushed to zero as the intersection kernel does --
 * to out_rays[0, m) in their input order, writes the input index of out_rays[k]
 * to out_index[k], and m to work[0].  Every other ray would be returned as a miss
 * by an intersection entry point.  `work` is caller-owned device memory of
 * CCS_COMPACT_WORK_WORDS(n) uint32 (word 0 the count, the rest the scan's
 * per-block counts); the library allocates nothing, so calls with different
 * `work` buffers may run concurrently.  All pointers are device pointers; out_rays
 * and out_index hold up to n elements and may not alias rays.  Asynchronous on
 * `stream`: read m after the stream has reached the call.  n = 0 sets work[0] = 0. */
#define CCS_COMPACT_WORK_WORDS(n) (1u + (uint32_t)(((uint64_t)(n) + 255u) / 256u))
ccs_status ccs_compact_rays(const ccs_ray* rays, uint32_t n, ccs_ray* out_rays, uint32_t* out_index, uint32_t* work,
                            void* stream);

/* Measurement of the fp32 grid arithmetic (Sec. 3.4 compares control points
 * recomputed for a subdomain with those reached by repeated subdivision).  For
 * query k: patch patch_ids[k] (index into the creation arrays), the subdomain
 * reached by depths[k] splits (u first, alternating) whose halves are the bits of
 * codes[k] (split s owns bit 2L-1-s, set for the upper half; no other bits set;
 * scenes with L <= 16, CCS_ERR_UNSUPPORTED above).
 * out (n x CCS_DEBUG_GRID_FLOATS fp32) row k holds, as stored on `frame`
 * (anchored, and mapped into the patch frame with CCS_FLAG_LOCAL_FRAMES):
 *   [0, 60)    the patch's stored points: x, y, z of slots 0..15, then of the P^v;
 *   [60, 108)  Alg. 2 (calcPointsAndD) on the subdomain as the intersection kernel
 *              recomputes it: component c of grid point (i, j) at 60 + 16c + 4j + i;
 *   [108, 111) its displacement d (0 for a Bezier patch);
 *   [111, 159) Bezier patches: the stored grid split along the path by the
 *              intersection kernel's split step (de Casteljau halves), same
 *              layout; NaN for a Gregory patch (its grid is recomputed at every node);
 *   [159]      0, or NaN for a query out of range (every value of its row is NaN).
 * All pointers are device pointers; asynchronous on `stream`. */
#define CCS_DEBUG_GRID_FLOATS 160
ccs_status ccs_debug_grids(const ccs_scene* scene, uint32_t frame, const uint32_t* patch_ids, const uint32_t* codes,
                           const uint32_t* depths, uint32_t n, float* out, void* stream);

/* ---------------------------------------------------- learned child ordering
 * Alg. 3 visits the two halves of a split closest box first (Sec. 3.3).  A
 * small network can choose instead at the splits along u where both halves are
 * hit: it ranks the node's four grandchildren (u-half, v-half) from 16 inputs
 * and the traversal enters the u-half, then one split later the v-half, of the
 * top-ranked one (the v-choice only where both v-halves are hit and the children
 * are not leaves).  Only hit halves are entered and every pending half is still
 * visited, so hits are those of Alg. 3 up to the order in which equal or
 * non-nested Gregory boxes are met.
 *
 * Inputs of a decision node (all scaled by s, the largest magnitude among the
 * first 12): 0..11 its grid's corner points (u0,v0), (u1,v0), (u0,v1), (u1,v1)
 * minus the ray's entry point into the node box, in the frame (e1, e2, d/|d|)
 * of Duff et al. 2017; 12, 13 entry and exit distance of the lower minus the
 * upper u-half times |d| / s, clamped to [-4, 4], / 4; 14 depth / 2L; 15 1 for a
 * Gregory patch.  Network: 16 -> 32 -> 32 -> 4 with ReLU, parameters
 * CCS_POLICY_PARAMS fp32 values in the order W1 (32 x 16, row = output unit),
 * b1 (32), W2 (32 x 32), b2 (32), W3 (4 x 32), b3 (4); logit k ranks grandchild
 * 2 * u_upper + v_upper.  Inference rounds inputs, weights and hidden
 * activations to bfloat16 (nearest, ties to even) and accumulates in fp32 on the
 * matrix cores. */
#define CCS_POLICY_PARAMS 1732
#define CCS_NO_LABEL 255

/* Attaches the network (params: device pointer, CCS_POLICY_PARAMS fp32) to the
 * scene: later ccs_intersect* calls use the learned order.  NULL detaches it
 * (closest-first order).  The weights are packed on `stream`; params may be
 * freed once the stream has passed the call.  CCS_ERR_UNSUPPORTED when the
 * scene's BVH is deeper than 31 levels (the learned kernel's node stack) or its
 * leaf depth above 16. */
ccs_status ccs_scene_set_policy(ccs_scene* scene, const float* params, void* stream);

/* Training records for n rays and their hits on frame 0 (device pointers).
 * Record r*L + k (L = leaf depth, k < L) describes the node of depth 2k on the
 * path to ray r's reported leaf: features[16 (r L + k) ..] its 16 inputs and
 * labels[r L + k] the grandchild holding the leaf; CCS_NO_LABEL (inputs zero)
 * where the ray missed or does not meet both u-halves' boxes (slab test without
 * the cap: the reported hit lies on the boxes' boundary as often as not).  features: n L 16 floats, labels:
 * n L bytes, caller-owned.  Asynchronous on `stream`. */
ccs_status ccs_policy_record(const ccs_scene* scene, const ccs_ray* rays, const ccs_hit* hits, uint32_t n,
                             float* features, uint8_t* labels, void* stream);

/* Logits (n x 4 fp32) of the network for n input rows (n x 16 fp32), computed
 * as during traversal.  Device pointers.  Synchronous (returns when done). */
ccs_status ccs_policy_infer(const float* params, const float* features, uint32_t n, float* logits, void* stream);

/* Mean softmax cross-entropy over the rows whose label is not CCS_NO_LABEL and
 * its gradient (CCS_POLICY_PARAMS fp32) with respect to params.  bf16 != 0:
 * inputs, weights and hidden activations rounded to bfloat16 as in inference,
 * the gradient passing straight through the roundings.  Device pointers; loss is
 * one float.  Synchronous. */
ccs_status ccs_policy_grad(const float* params, const float* features, const uint8_t* labels, uint32_t n,
                           uint32_t bf16, float* grad, float* loss, void* stream);

/* ccs_policy_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * allocation): the same kernels and results, with the per-block partial
 * gradients in a preallocated device array of the library (1.7 MiB per device,
 * held until the process ends) instead of temporaries.  Asynchronous on `stream`
 * (no synchronization).  At most 16384 rows (CCS_ERR_INVALID_ARG beyond).
 * Every call on one device shares that array: calls that overlap on a device
 * (other streams, other threads) race and must be serialized by the caller; a
 * call's grad and loss are final once its stream has passed it. */
#define CCS_GRAD_NOALLOC_MAX_ROWS 16384
ccs_status ccs_policy_grad_noalloc(const float* params, const float* features, const uint8_t* labels, uint32_t n,
                                   uint32_t bf16, float* grad, float* loss, void* stream);

typedef struct ccs_train_params {
  uint32_t steps;  /* optimizer steps */
  uint32_t batch;  /* rows per step (at most n); an epoch is floor(n / batch) steps */
  float lr, beta1, beta2, eps; /* Adam (Kingma & Ba 2015) */
  uint64_t seed;   /* row order: a seeded affine permutation of the rows per epoch */
  uint32_t bf16;   /* as in ccs_policy_grad */
  uint32_t reserved;
} ccs_train_params;

/* Adam's moments and step count, for training in several calls: m and v are
 * caller-owned device arrays of CCS_POLICY_PARAMS floats, t the number of steps
 * already taken with them (all zero for a fresh start; at most 2^32). */
typedef struct ccs_adam_state {
  float* m;
  float* v;
  uint64_t t;
} ccs_adam_state;

/* Trains params (device, CCS_POLICY_PARAMS fp32, updated in place) with Adam
 * on the rows (features n x 16, labels n) for tp->steps minibatches.
 * state: NULL to start from zero moments at step 0 (moments then live in
 * temporaries), else read and updated in place, t advanced by tp->steps; step
 * t + s of a resumed call draws the minibatch and bias corrections that global
 * step t + s draws in one uninterrupted call, so k steps followed by j resumed
 * steps give the bits of k + j steps at once (same n, tp except steps).
 * loss_history: NULL or device array of tp->steps floats receiving each step's
 * minibatch loss before its update.  Deterministic for a given seed.
 * Synchronous. */
ccs_status ccs_policy_train(float* params, const float* features, const uint8_t* labels, uint32_t n,
                            const ccs_train_params* tp, ccs_adam_state* state, float* loss_history, void* stream);

ccs_status ccs_scene_info_get(const ccs_scene* scene, ccs_scene_info* info);

/* Device memory cap.  Every device allocation of the library (scene buffers,
 * animation frames, packed network operands, the temporaries of the synchronous
 * policy calls) is refused with CCS_ERR_OOM when it would bring the bytes the
 * library holds in this process above the value of the environment variable
 * CCS_MAX_DEVICE_BYTES (a decimal byte count, read at each allocation; unset,
 * empty or 0: no cap; anything else: CCS_ERR_INVALID_ARG).  A call that fails
 * this way frees whatever it had allocated.  ccs_device_bytes_in_use() returns
 * the bytes held right now: the sum of ccs_scene_info.device_bytes over live
 * scenes plus the temporaries of calls in progress.  Thread-safe. */
uint64_t ccs_device_bytes_in_use(void);

/* Frees every device buffer of the scene (synchronizes the device first).  NULL is a no-op. */
void ccs_scene_destroy(ccs_scene* scene);

/* Message of the last failing call on this thread ("" if none).  Valid until the
 * next ccs_* call on the same thread. */
const char* ccs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CCS_H */
