"""FP64 reference of the child-ordering policy's inputs and labels (TEST
INFRASTRUCTURE ONLY: used by ``tests/`` alone).

The paper orders children closest-first (Sec. 3.3); the learned policy replaces
that choice at the nodes of even depth (the next split runs along u) where both
u-halves are hit, and ranks the node's four grandchildren (u-half, v-half).
Its 16 inputs describe the ray against the node, all in a ray-centred frame and
scaled by the node's size so that they are free of position, orientation and
scale:

  0..11  the four corner control points of the node's grid, in the order
         (u0,v0), (u1,v0), (u0,v1), (u1,v1) (the surface points there for a
         Bezier patch; for a Gregory patch the corners of its lower bounding
         grid of Alg. 2), relative to the point where the ray enters the
         node's box, in the
         orthonormal frame (e1, e2, d/|d|) of Duff et al. 2017 ("Building an
         Orthonormal Basis, Revisited"), divided by s = the largest magnitude
         among these 12 values
  12     (entry(lower u-half) - entry(upper u-half)) |d| / s, clamped to [-4, 4], / 4
  13     (exit(lower u-half) - exit(upper u-half)) |d| / s, clamped to [-4, 4], / 4
  14     depth / (2 L)
  15     1 for a Gregory patch, else 0

where the node box is the union of the two u-half boxes of Alg. 3's split (box
of the half's control points, grown by the parent's Gregory displacement on the
max side) and entries and exits are those of the slab test without the cap.
During traversal the node is a decision when both halves pass the capped slab
test.  A training record is the node of even depth on the path to a ray's
reported leaf where the ray meets both halves' boxes (no cap: the reported hit
lies on the boxes' boundary as often as not, where a capped test would turn on
rounding); its label is the grandchild holding that leaf, 2 * (u-half) +
(v-half).
"""
from __future__ import annotations

import numpy as np

from . import calc_points_and_d, split

NO_LABEL = 255


def onb(n):
    """Duff et al. 2017: (e1, e2) completing the unit vector n to a right-handed frame."""
    sign = np.copysign(1.0, n[2])
    a = -1.0 / (sign + n[2])
    b = n[0] * n[1] * a
    e1 = np.array([1.0 + sign * n[0] * n[0] * a, sign * b, -sign * n[0]])
    e2 = np.array([b, sign + n[1] * n[1] * a, -n[1]])
    return e1, e2


def _slab(lo, hi, o, d, tmin):
    """Entry and exit of the ray o + t d, t >= tmin, through the box [lo, hi] (C8
    without the cap); an axis with d = 0 is unbounded inside the planes, empty outside."""
    near, far = tmin, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if not (lo[a] <= o[a] <= hi[a]):
                return np.inf, -np.inf
            continue
        t0, t1 = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        near, far = max(near, min(t0, t1)), min(far, max(t0, t1))
    return near, far


def node_features(cp20, gregory: bool, ray8, u0, v0, size, depth: int, leaf_depth: int, cap: float):
    """(features (16,), valid) at the node [u0, u0+size] x [v0, v0+size] of even depth."""
    o = np.asarray(ray8[:3], dtype=np.float64)
    d = np.asarray(ray8[4:7], dtype=np.float64)
    tmin = float(ray8[3])
    q, disp = calc_points_and_d(cp20, gregory, u0, u0 + size, v0, v0 + size)
    A, B = split(q, 0)
    lo_a, hi_a = A.min(axis=0), A.max(axis=0) + disp
    lo_b, hi_b = B.min(axis=0), B.max(axis=0) + disp
    na, fa = _slab(lo_a, hi_a, o, d, tmin)
    nb, fb = _slab(lo_b, hi_b, o, d, tmin)
    valid = (na <= min(fa, cap)) and (nb <= min(fb, cap))
    f = np.zeros(16)
    if not valid:
        return f, False
    dl = np.linalg.norm(d)
    dn = d / dl
    e1, e2 = onb(dn)
    p = o + min(na, nb) * d
    corners = q[[0, 3, 12, 15]] - p  # slots (i, j) = (0,0), (3,0), (0,3), (3,3)
    loc = np.stack([corners @ e1, corners @ e2, corners @ dn], axis=1)
    s = max(np.abs(loc).max(), 1e-30)
    f[:12] = (loc / s).reshape(-1)
    f[12] = np.clip((na - nb) * dl / s, -4.0, 4.0) / 4.0
    f[13] = np.clip((fa - fb) * dl / s, -4.0, 4.0) / 4.0
    f[14] = depth / (2.0 * leaf_depth)
    f[15] = 1.0 if gregory else 0.0
    return f, True


def path_records(cp20, gregory: bool, ray8, u: float, v: float, leaf_depth: int, cap: float = np.inf):
    """Records (features (L, 16), labels (L,)) along the path to the leaf holding
    (u, v): one per even depth 0, 2, ..., 2L-2; label 255 where the ray does not
    meet both u-halves' boxes under `cap` (records use no cap)."""
    L = leaf_depth
    iu, iv = int(np.floor(u * 2 ** L)), int(np.floor(v * 2 ** L))
    feats, labels = np.zeros((L, 16)), np.full(L, NO_LABEL, dtype=np.uint8)
    for k in range(L):
        size = 2.0 ** -k
        u0, v0 = (iu >> (L - k)) * size, (iv >> (L - k)) * size
        f, ok = node_features(cp20, gregory, ray8, u0, v0, size, 2 * k, L, cap)
        if ok:
            feats[k] = f
            labels[k] = 2 * ((iu >> (L - 1 - k)) & 1) + ((iv >> (L - 1 - k)) & 1)
    return feats, labels
