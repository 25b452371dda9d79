"""Pins of the oracle's patch-local frames (Sec. 3.4): the frame itself, exact
hits on flat patches (boxes in the patch's frame have no thickness), agreement
with the world-frame method and the work it saves."""
import numpy as np

import oracle as O
from paper_1811_03510_amd import scenes as S


def test_frames_are_orthonormal_and_follow_the_patch_edges(c1):
    sc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=True)
    for k in range(0, len(c1.cp), 7):
        R = sc.patch_frame(k)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert np.allclose(np.cross(R[0], R[1]), R[2], atol=1e-14)
        p = c1.cp[k].astype(np.float64)
        eu, ev = p[3] - p[0], p[12] - p[0]
        assert np.allclose(R[0], eu / np.linalg.norm(eu), atol=1e-14)
        assert abs(np.dot(R[2], eu)) < 1e-12 and abs(np.dot(R[2], ev)) < 1e-12 * np.linalg.norm(ev)
        assert np.dot(R[1], ev) > 0
    world = O.Scene(c1.cp, c1.types, c1.leaf_depth)
    assert np.array_equal(world.patch_frame(0), np.eye(3))


def test_degenerate_edges_fall_back_to_the_identity():
    g = np.zeros((20, 3), np.float32)
    for j in range(4):
        for i in range(4):
            g[4 * j + i] = (0.0, j / 3.0, (i * j) / 9.0)  # u edge p00 -> p30 collapsed to a point
    sc = O.Scene(g[None], np.zeros(1, np.uint8), 4, local_frames=True)
    assert np.array_equal(sc.patch_frame(0), np.eye(3))


def test_flat_patch_hits_are_exact_in_its_frame():
    """A tilted flat patch lies in its frame's r0-r1 plane, so every box is flat
    there and the entry distance is the plane's: t exact to the input's rounding
    and the gap-closing pad, and the reported leaf's box holds the closed-form hit
    (the world-frame method is only within a leaf's thickness)."""
    rng = np.random.default_rng(3)
    L = 8
    a = rng.normal(size=3)
    e1, e2 = rng.normal(size=3), rng.normal(size=3)
    g = np.zeros((20, 3))
    for j in range(4):
        for i in range(4):
            g[4 * j + i] = a + (i / 3.0) * e1 + (j / 3.0) * e2
    cp = g.astype(np.float32)[None]
    loc = O.Scene(cp, np.zeros(1, np.uint8), L, local_frames=True)
    wor = O.Scene(cp, np.zeros(1, np.uint8), L)
    P = cp[0].astype(np.float64)
    a32, e1_32, e2_32 = P[0], P[3] - P[0], P[12] - P[0]
    nrm = np.cross(e1_32, e2_32)
    n_ok, worse = 0, 0
    for _ in range(300):
        u, v = rng.uniform(0.05, 0.95, 2)
        x = a32 + u * e1_32 + v * e2_32
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if abs(np.dot(d, nrm)) < 0.3 * np.linalg.norm(nrm):
            continue
        o = x - rng.uniform(0.5, 3.0) * d
        ray = np.array([[*o, 0.0, *d, np.inf]], np.float32)
        r64 = ray[0].astype(np.float64)
        t_star = np.dot(a32 - r64[:3], nrm) / np.dot(r64[4:7], nrm)
        h = loc.intersect(ray)
        assert h["id"][0] == 0
        # the fp32 control points are flat only to their rounding: the boxes are as
        # thick as the points' spread along the frame normal r2, and no thicker
        # and every box is grown by the gap-closing pad, 2^-19 of the patch's extent
        Rf = loc.patch_frame(0)
        r2 = Rf[2]
        thick = np.ptp(P[:16] @ r2)
        pad = np.ldexp(np.ptp(P[:16] @ Rf.T, axis=0).max(), -19)
        cosv = abs(np.dot(r64[4:7], r2)) / np.linalg.norm(r64[4:7])
        assert thick < 1e-6
        assert abs(h["t"][0] - t_star) <= (thick + pad) / cosv + 1e-12 * max(1.0, abs(t_star)), (h["t"][0], t_star)
        xs = r64[:3] + t_star * r64[4:7]
        # the reported leaf's box (in the patch frame) holds the closed-form hit point
        lo, hi = loc.leaf_box(0, h["u"][0], h["v"][0])
        xf = loc.patch_frame(0) @ xs
        tol = thick + pad + 1e-9  # the leaf box is exact to the points' rounding and the pad
        assert np.all(xf >= lo - tol) and np.all(xf <= hi + tol)
        hw = wor.intersect(ray)
        worse += abs(hw["t"][0] - t_star) > 1e-6
        n_ok += 1
    assert n_ok > 150
    assert worse > 0.5 * n_ok  # the world-frame boxes of the tilted patch are thick


def test_local_frames_agree_with_world_and_save_work(c1, c1_oracle):
    loc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=True)
    rays = np.concatenate([c1.primary, c1.diffuse])
    a = c1_oracle.intersect(rays, counters=True)
    b = loc.intersect(rays, counters=True)
    same = a["id"] == b["id"]
    assert same.mean() >= 0.999
    both = same & (a["id"] != O.NO_HIT)
    # both report an entry into a leaf box around the same surface point
    assert np.abs(a["t"][both] - b["t"][both]).max() <= 1e-3 * c1.diameter
    k = O.COUNTER_NAMES.index("split")
    assert b["counters"][:, k].mean() < 0.8 * a["counters"][:, k].mean()
