"""How much any child order can save (the ceiling of the learned child order).

Alg. 3 visits the closer of two hit halves first (Sec. 3.3).  Two other orders,
wherever both halves are hit, bound what a learned order can save with either label:
the hindsight order knows each ray's final leaf and enters the half holding it first
(a perfect predictor of the final leaf), and the lookahead order tries both halves
first over the node's subtree and keeps the one with fewer split steps (a perfect
predictor of that work label).  On the 512-patch torus both stay within a fraction
of a per cent of closest-first's split steps, for primary and secondary rays alike:
once the closest leaf is known, what remains to visit lies in front of it (its boxes
are entered before the best distance, so the cap prunes none of it), and
closest-first already leaves the boxes behind the hit for last.  The hits are the
same rays' closest hits."""
import numpy as np

import oracle as O


def test_other_orders_save_almost_nothing(c1):
    for local in (False, True):
        osc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=local)
        for cls, rays in (("primary", c1.primary), ("diffuse", c1.diffuse)):
            o = osc.intersect(rays, counters=True)
            hit = o["id"] != O.NO_HIT
            s0 = o["counters"][:, 2].astype(np.float64).mean()
            for label, h in (("hindsight", osc.intersect_hinted(rays, o)),
                             ("lookahead", osc.intersect_hinted(rays, lookahead=True))):
                # the same closest hits (Gregory boxes need not nest, so an order may pick
                # the other of two leaves that tie within the leaf box; none does here)
                assert np.array_equal(o["id"], h["id"]), label
                assert np.allclose(o["t"][hit], h["t"][hit], rtol=1e-12, atol=0), label
                s1 = h["counters"][:, 2].astype(np.float64).mean()
                print(f"torus512 {cls} ({'local' if local else 'world'}): splits per ray closest-first {s0:.3f}, "
                      f"{label} {s1:.3f} ({100 * (1 - s1 / s0):.2f} % fewer)")
                assert s1 <= s0, label
                assert s1 >= 0.98 * s0, label  # the ceiling of a learned order: under 2 % of the split steps


def test_hindsight_hint_steers_the_order(c1, c1_oracle):
    """A hint toward a leaf that is not the closest one changes the visiting order
    (more split steps) but never the result: the order does not decide hits."""
    rays = c1.diffuse[::16]
    o = c1_oracle.intersect(rays, counters=True)
    hit = o["id"] != O.NO_HIT
    wrong = dict(id=o["id"].copy(), u=1.0 - o["u"], v=1.0 - o["v"])  # the mirrored leaf
    h = c1_oracle.intersect_hinted(rays, wrong)
    assert np.array_equal(h["id"], o["id"]) and np.allclose(h["t"][hit], o["t"][hit], rtol=1e-12, atol=0)
    assert h["counters"][:, 2].sum() > o["counters"][:, 2].sum()


def test_single_box_mode_equals_alg3_on_bezier_patches(c1):
    """The oracle's single-box mode (Sec. 3.3's alternative: each node tests only its
    own box, the crop of the grid to its domain) against Alg. 3's two-box recursion
    (child boxes from de Casteljau halves): on Bezier patches a child's box is the
    same box either way and the closest leaf is reached by both, so every hit is
    the same leaf at the same distance (up to the crop's rounding); and the mode
    takes more box tests per ray, as Sec. 3.3 reports.  With Gregory patches the
    leaf boxes differ (own bound vs the parent's half), so hits may move to a
    neighbouring leaf within the distance tolerance."""
    types0 = np.zeros_like(c1.types)
    for local in (False, True):
        osc = O.Scene(c1.cp, types0, c1.leaf_depth, local_frames=local)
        for rays in (c1.primary, c1.diffuse):
            a = osc.intersect(rays, counters=True)
            b = osc.intersect_single_box(rays)
            hit = a["id"] != O.NO_HIT
            assert np.array_equal(a["id"], b["id"])
            assert np.allclose(a["t"][hit], b["t"][hit], rtol=1e-12, atol=1e-13)
            assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["v"], b["v"])
            assert b["counters"][:, 2].mean() > 1.5 * a["counters"][:, 2].mean()
    osc = O.Scene(c1.cp, c1.types, c1.leaf_depth)
    a, b = osc.intersect(c1.diffuse), osc.intersect_single_box(c1.diffuse)
    hit = a["id"] != O.NO_HIT
    assert np.array_equal(a["id"], b["id"])
    assert np.abs(a["t"][hit] - b["t"][hit]).max() <= 1e-4 * c1.diameter


def test_retesting_resumed_siblings_saves_little(c1):
    """Alg. 3 resumes a pending sibling without re-testing its box against the best
    distance found since (reading R11).  Skipping siblings whose box was entered beyond
    it leaves every hit unchanged and saves a few per cent of the split steps (and more
    of the grid recomputes, which every resumed sibling costs): what is left to visit
    after the closest leaf lies mostly in front of it."""
    for local in (False, True):
        osc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=local)
        for cls, rays in (("primary", c1.primary), ("diffuse", c1.diffuse)):
            a = osc.intersect(rays, counters=True)
            b = osc.intersect_retest(rays)
            hit = a["id"] != O.NO_HIT
            assert np.array_equal(a["id"], b["id"]) and np.array_equal(a["u"], b["u"]) and np.array_equal(a["v"], b["v"])
            assert np.allclose(a["t"][hit], b["t"][hit], rtol=1e-12, atol=0)
            s0, s1 = a["counters"][:, 2].mean(), b["counters"][:, 2].mean()
            r0 = (a["counters"][:, 4] + a["counters"][:, 6]).mean()
            r1 = (b["counters"][:, 4] + b["counters"][:, 6]).mean()
            print(f"torus512 {cls} ({'local' if local else 'world'}): splits {s0:.2f} -> {s1:.2f}, "
                  f"recomputes {r0:.2f} -> {r1:.2f}")
            assert s1 <= s0 and r1 <= r0
            assert s1 >= 0.9 * s0
