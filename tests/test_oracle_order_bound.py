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
