"""The one-box-per-step ablation (CCS_FLAG_SINGLE_BOX; Sec. 3.3 reports that testing
the two child boxes instead nearly halves traversal time).  It must give the hits of
the oracle's single-box mode under the same gate (a Gregory leaf is then tested by
its own bound, not by the half of its parent's grid that Alg. 3 tests, so a ray
grazing the difference may name a neighbouring leaf), and it must do more
subdivision work per ray: without the child boxes' distances no half can be pruned
before its grid exists, and every pending half costs a recompute."""
import numpy as np
import pytest

import oracle as O
from oracle.parity import assert_gate, gate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("local", [False, True], ids=["world", "local"])
def test_single_box_matches_oracle_and_does_more_work(c1, local):
    from paper_1811_03510_amd import ccs
    L = c1.leaf_depth
    cp, ty = torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda()
    two = ccs.Scene(cp, ty, L, local_frames=local)
    one = ccs.Scene(cp, ty, L, local_frames=local, single_box=True)
    osc = O.Scene(c1.cp, c1.types, L, local_frames=local)
    for cls, rays in (("primary", c1.primary), ("diffuse", c1.diffuse)):
        r = torch.from_numpy(rays).cuda()
        _say(f"single-box ablation, torus512 {cls} ({len(rays)} rays, local frames: {local})")
        h1, c_one = one.intersect_counted(r)
        h2, c_two = two.intersect_counted(r)
        torch.cuda.synchronize()
        g = h1.cpu().numpy()
        assert_gate(gate(g, osc.intersect_single_box(rays), rays, osc, c1.diameter, L, label=f"single-box-{cls}"))
        # the plain launch gives the counted launch's hits
        assert np.array_equal(one.intersect(r).cpu().numpy().view(np.uint32), g.view(np.uint32))
        c_one, c_two = c_one.cpu().numpy().astype(np.float64), c_two.cpu().numpy().astype(np.float64)
        k = {n: i for i, n in enumerate(ccs.COUNTER_NAMES)}
        s1, s2 = c_one[:, k["split"]].mean(), c_two[:, k["split"]].mean()
        r1 = (c_one[:, k["crop"]] + c_one[:, k["greg"]]).mean()
        r2 = (c_two[:, k["crop"]] + c_two[:, k["greg"]]).mean()
        _say(f"  steps per ray: one box {s1:.2f}, two boxes {s2:.2f}; grid recomputes {r1:.2f} vs {r2:.2f}; "
             f"backtracks {c_one[:, k['backtrack']].mean():.2f} vs {c_two[:, k['backtrack']].mean():.2f}")
        # same candidates from the BVH (the traversal is shared), more work per candidate
        assert r1 > r2 and c_one[:, k["backtrack"]].mean() > c_two[:, k["backtrack"]].mean()


def test_single_box_refuses_a_learned_order(c1):
    from paper_1811_03510_amd import ccs
    one = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth,
                    single_box=True)
    with pytest.raises(ccs.CcsError) as e:
        one.set_policy(torch.zeros(ccs.POLICY_PARAMS, dtype=torch.float32, device="cuda"))
    assert e.value.status == ccs.CCS_ERR_UNSUPPORTED
