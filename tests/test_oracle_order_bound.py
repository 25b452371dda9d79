"""How much any child order can save (the ceiling of the learned child order).

Alg. 3 visits the closer of two hit halves first (Sec. 3.3).  The hindsight order
knows each ray's final leaf and, wherever both halves are hit, enters the half
holding it first: no predictor of the final leaf can do better than it.  On the
512-patch torus its split steps per ray stay within a fraction of a per cent of
closest-first ones, for primary and secondary rays alike: once the closest leaf is
known, what remains to visit lies in front of it (its boxes are entered before the
best distance, so the cap prunes none of it), and closest-first already leaves the
boxes behind the hit for last.  The hits are the same rays' closest hits."""
import numpy as np

import oracle as O


def _bound(osc, rays):
    o = osc.intersect(rays, counters=True)
    h = osc.intersect_hinted(rays, o)
    return o, h


def test_hindsight_order_saves_almost_nothing(c1):
    for local in (False, True):
        osc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=local)
        for cls, rays in (("primary", c1.primary), ("diffuse", c1.diffuse)):
            o, h = _bound(osc, rays)
            hit = o["id"] != O.NO_HIT
            # the same closest hits (Gregory boxes need not nest, so an order may pick the
            # other of two leaves that tie within the leaf box; none does here)
            assert np.array_equal(o["id"], h["id"])
            assert np.allclose(o["t"][hit], h["t"][hit], rtol=1e-12, atol=0)
            s0 = o["counters"][:, 2].astype(np.float64).mean()
            s1 = h["counters"][:, 2].astype(np.float64).mean()
            print(f"torus512 {cls} ({'local' if local else 'world'}): splits per ray closest-first {s0:.3f}, "
                  f"hindsight {s1:.3f} ({100 * (1 - s1 / s0):.2f} % fewer)")
            assert s1 <= s0
            assert s1 >= 0.98 * s0  # the ceiling of any learned order: under 2 % of the split steps


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
