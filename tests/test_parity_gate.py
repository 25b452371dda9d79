"""The parity gate itself, on the CPU: identical results match, and each kind of
planted error is caught (or excused only by the rule written for it)."""
import numpy as np

import oracle as O
from oracle.parity import gate
from paper_1811_03510_amd import scenes as S


def _as_gpu(o):
    g = np.zeros((len(o["t"]), 4), np.float32)
    g[:, 0] = o["t"]
    g[:, 1] = o["id"].astype(np.uint32).view(np.float32)
    g[:, 2], g[:, 3] = o["u"], o["v"]
    return g


def test_identical_results_match(c1, c1_oracle):
    rays = c1.primary[::8]
    o = c1_oracle.intersect(rays)
    rep = gate(_as_gpu(o), o, rays, c1_oracle, c1.diameter, c1.leaf_depth)
    assert rep["ok"] and rep["match"] == len(rays)


def test_planted_errors_are_hard(c1, c1_oracle):
    rays = c1.primary[::8]
    o = c1_oracle.intersect(rays)
    hit = np.flatnonzero(o["id"] != O.NO_HIT)[:200]
    L = c1.leaf_depth
    leaf = 2.0 ** -L
    for kind in ("shift5", "late_t", "miss"):
        g = _as_gpu(o)
        if kind == "shift5":    # five leaves away along u (away from the patch edge)
            g[hit, 2] = np.where(g[hit, 2] > 0.5, g[hit, 2] - 5 * leaf, g[hit, 2] + 5 * leaf)
        elif kind == "late_t":  # beyond the distance tolerance
            g[hit, 0] += 2e-4 * c1.diameter
        else:                   # a hit dropped
            g[hit, 0] = np.inf
            g[hit, 1] = np.array([O.NO_HIT], np.uint32).view(np.float32)[0]
        rep = gate(g, o, rays, c1_oracle, c1.diameter, L)
        assert not rep["ok"] and rep["excused"]["hard"] == len(hit), (kind, rep["excused"])


def test_tangent_excuse_is_limited_to_grazing_rays(c1, c1_oracle):
    """A leaf a few leaves away is excused only for rays within 1.2 degrees of
    tangent that pass within the leaf box of the surface there."""
    rng = np.random.default_rng(4)
    L = c1.leaf_depth
    leaf = 2.0 ** -L
    k = 100
    u0, v0 = 0.43, 0.57
    x = S.surface_points(c1.cp, c1.types, np.array([k]), np.array([u0]), np.array([v0]))[0]
    _, fu, fv = O.patch_eval(c1.cp[k], bool(c1.types[k]), u0, v0)
    n = np.cross(fu, fv)
    n /= np.linalg.norm(n)
    tdir = fu / np.linalg.norm(fu)
    rays, want = [], []
    for cosv, kind in ((0.5, "hard"), (0.2, "hard"), (0.005, "tangent")):
        d = np.sqrt(1 - cosv ** 2) * tdir - cosv * n
        rays.append([*(x - 0.05 * d), 0.0, *d, np.inf])
        want.append(kind)
    rays = np.array(rays, np.float32)
    o = c1_oracle.intersect(rays)
    checked = 0
    for i, kind in enumerate(want):
        if o["id"][i] != k:
            continue
        checked += 1
        g = _as_gpu({key: o[key][i:i + 1] for key in ("t", "id", "u", "v")})
        # the next leaf along the ray's tangent direction (u grows along fu)
        g[0, 2] += 3 * leaf
        rep = gate(g, {key: o[key][i:i + 1] for key in ("t", "id", "u", "v")}, rays[i:i + 1], c1_oracle,
                   c1.diameter, L)
        got = [kk for kk, v in rep["excused"].items() if v]
        assert got == [kind], (i, rep["excused"])
    assert checked == 3


def test_graze_excuse_covers_the_box_alg3_records_a_leaf_by(c1):
    """A hit on a leaf whose Alg. 3 box (the parent's grid half with the parent's
    displacement, larger than the leaf's own bound for a Gregory patch) the ray only
    clips by rounding is a graze; one that misses that box by more is hard."""
    from oracle.parity import _lateral_margin, _path_in_box
    L = 4  # coarse leaves, where the two boxes differ by several times the slack
    osc = O.Scene(c1.cp, c1.types, L)
    n = 2 ** L
    uc, vc = (n // 3 + 0.5) / n, (n // 2 + 0.5) / n
    t_hit = 0.01
    checked = 0
    for pid in np.where(c1.types == 1)[0][:20]:
        lo, hi = osc.leaf_box_alg3(pid, uc, vc)
        olo, ohi = osc.leaf_box(pid, uc, vc)
        slack = 1e-3 * np.linalg.norm(hi - lo) + 1e-7 * (t_hit + 1.0)
        # the box corner (axes a, b; sides sa, sb) where the Alg. 3 box reaches
        # furthest beyond the leaf's own bound
        excess = lambda ax, sd: (hi - ohi)[ax] if sd > 0 else (olo - lo)[ax]
        score, a, b, sa, sb = max((min(excess(a, sa), excess(b, sb)), a, b, sa, sb)
                                  for a in range(3) for b in range(a + 1, 3) for sa in (1, -1) for sb in (1, -1))
        if score < 2 * slack:
            continue
        corner = np.where([sa > 0, sb > 0], [hi[a], hi[b]], [lo[a], lo[b]])
        kinds = []
        for miss in (0.25 * slack, 4.0 * slack):
            # in the plane of axes a and b, across the corner's diagonal at distance
            # miss / 2 from the corner: the path in the box is -miss
            delta = miss / (2.0 * np.sqrt(2.0))
            p = 0.5 * (lo + hi)
            p[a], p[b] = corner[0] + sa * delta, corner[1] + sb * delta
            d = np.zeros(3)
            d[a], d[b] = sa / np.sqrt(2.0), -sb / np.sqrt(2.0)
            ray = np.array([*(p - t_hit * d), 0.0, *d, np.inf])
            assert abs(_path_in_box(ray, lo, hi) + miss) <= 1e-3 * miss
            # across the ray the line passes the box corner at half the miss
            assert abs(_lateral_margin(ray, lo, hi)[0] + 0.5 * miss) <= 1e-3 * miss
            assert _path_in_box(ray, olo, ohi) < -slack  # the leaf's own bound alone excuses nothing
            r32 = ray.astype(np.float32)[None]
            o = osc.intersect(r32)
            if o["id"][0] != O.NO_HIT and o["t"][0] < t_hit - 1e-4 * c1.diameter:
                kinds = None  # the ray meets a nearer leaf: the planted hit is wrong whatever the box
                break
            g = _as_gpu(o)
            g[0, 0] = t_hit
            g[0, 1] = np.array([pid], np.uint32).view(np.float32)[0]
            g[0, 2], g[0, 3] = uc, vc
            rep = gate(g, o, r32, osc, c1.diameter, L)
            kinds.append([k for k, v in rep["excused"].items() if v])
        if kinds is None or ["seam"] in kinds or [] in kinds:
            continue  # the oracle hit another patch next to this one, or this leaf
        assert kinds == [["graze"], ["hard"]], (pid, kinds)
        checked += 1
    assert checked >= 3


def _edge_rays(c1, osc, n_rays=40, seed=11):
    """Rays from the torus camera aimed at points on patch edges (v = 0 of a patch,
    u uniform in (0.1, 0.9)) that the oracle hits within a leaf of an edge, with the
    patch across that edge: [(ray, oracle hit, neighbour patch, its (u, v) there)]."""
    rng = np.random.default_rng(seed)
    eye = np.array([0.0, -3.2, 2.0])
    L = c1.leaf_depth
    m = 2.0 ** -L
    # every patch's v = 1 boundary, sampled, to find the neighbour across a v = 0 edge
    us = np.linspace(0.1, 0.9, 5)
    top = np.stack([S.surface_points(c1.cp, c1.types, np.full(5, k), us, np.ones(5)) for k in range(len(c1.cp))])
    out = []
    for k in rng.permutation(len(c1.cp)):
        u = float(rng.uniform(0.1, 0.9))
        x = S.surface_points(c1.cp, c1.types, np.array([k]), np.array([u]), np.array([0.0]))[0]
        d = x - eye
        d /= np.linalg.norm(d)
        ray = np.array([*eye, 0.0, *d, np.inf], np.float32)
        o = osc.intersect(ray[None])
        if o["id"][0] == O.NO_HIT or min(o["u"][0], o["v"][0], 1 - o["u"][0], 1 - o["v"][0]) > m * (1 + 1e-6):
            continue
        xs = S.surface_points(c1.cp, c1.types, np.full(5, k), us, np.zeros(5))
        nb = int(np.argmin(np.abs(top - xs[None]).max(axis=(1, 2))))
        if nb == k or np.abs(top[nb] - xs).max() > 1e-6:
            continue
        out.append((ray, {key: o[key][:1] for key in ("t", "id", "u", "v")}, nb, (u, 1.0 - 0.5 * m)))
        if len(out) == n_rays:
            break
    return out


def test_far_wrong_patch_at_an_edge_is_hard(c1):
    """A ray through a patch edge that slips through a crack and names a patch
    farther along (itself hit near its own edge) is hard at any distance, also when
    the planted hit is nearer than the distance tolerance; the patch across the edge
    at the same point is excused (tie or seam)."""
    for local in (False, True):
        osc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=local)
        cases = _edge_rays(c1, osc)
        assert len(cases) >= 20, len(cases)
        L = c1.leaf_depth
        leaf = 2.0 ** -L
        for ray, o, nb, (unb, vnb) in cases:
            g = _as_gpu(o)
            far_id = (int(o["id"][0]) + 101) % len(c1.cp)
            for dist in (0.5 * c1.diameter, 0.01 * c1.diameter, 4 * leaf):
                gp = g.copy()
                gp[0, 0] = o["t"][0] + dist
                gp[0, 1] = np.array([far_id], np.uint32).view(np.float32)[0]
                gp[0, 2], gp[0, 3] = 0.5 * leaf, 0.5  # on the far patch's u = 0 edge
                rep = gate(gp, o, ray[None], osc, c1.diameter, L)
                assert rep["excused"]["hard"] == 1, (local, dist, rep["excused"])
            if int(o["id"][0]) != nb:
                gs = g.copy()
                gs[0, 1] = np.array([nb], np.uint32).view(np.float32)[0]
                gs[0, 2], gs[0, 3] = unb, vnb
                rep = gate(gs, o, ray[None], osc, c1.diameter, L)
                assert rep["excused"]["hard"] == 0, (local, rep["excused"], rep["hard"])


def test_far_hit_behind_a_thin_leaf_box_is_hard(c1):
    """The oracle's leaf boxes are thin wherever the surface is flat at leaf scale,
    so the ray's path through them is short even where it crosses them squarely; a
    GPU that names a patch behind such a hit is not excused as a graze."""
    for local in (False, True):
        osc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=local)
        rays = c1.primary[::4]
        o = osc.intersect(rays)
        hit = np.flatnonzero(o["id"] != O.NO_HIT)[:300]
        g = _as_gpu(o)
        g[hit, 0] = o["t"][hit] + 2e-3 * c1.diameter
        g[hit, 1] = ((o["id"][hit] + 7) % len(c1.cp)).astype(np.uint32).view(np.float32)
        g[hit, 2], g[hit, 3] = 0.5 * 2.0 ** -c1.leaf_depth, 0.5
        rep = gate(g, o, rays, osc, c1.diameter, c1.leaf_depth)
        assert rep["excused"]["hard"] == len(hit), (local, rep["excused"])


def test_ray_starting_within_rounding_of_a_leaf_box(c1):
    """A GPU hit at tmin on a leaf box the ray starts just outside of (by a quarter of
    the slack, so only rounding put the start inside) is a graze; the same report
    with the start four slacks outside, or with a later distance, is hard."""
    L = c1.leaf_depth
    checked = 0
    for local in (False, True):
        osc = O.Scene(c1.cp, c1.types, L, local_frames=local)
        rng = np.random.default_rng(17)
        for pid in rng.choice(len(c1.cp), 12, replace=False):
            uc, vc = (rng.integers(0, 2 ** L) + 0.5) * 2.0 ** -L, (rng.integers(0, 2 ** L) + 0.5) * 2.0 ** -L
            lo, hi = osc.leaf_box(pid, uc, vc)
            slack = 1e-3 * np.linalg.norm(hi - lo) + 1e-7
            R = osc.patch_frame(int(pid))
            kinds = []
            for gap, t_rep in ((0.25 * slack, 0.0), (4.0 * slack, 0.0), (0.25 * slack, 1e-3 * c1.diameter)):
                # start beyond the box's largest face along frame axis 2, moving away from it
                pf = 0.5 * (lo + hi)
                pf[2] = hi[2] + gap
                df = np.array([0.3, -0.2, 1.0])
                df /= np.linalg.norm(df)
                ray = np.array([*(R.T @ pf), 0.0, *(R.T @ df), np.inf])
                o = osc.intersect_f64(ray[None])  # the ray in double: the planted gap is exact
                g = np.zeros((1, 4), np.float32)
                g[0, 0] = t_rep
                g[0, 1] = np.array([pid], np.uint32).view(np.float32)[0]
                g[0, 2], g[0, 3] = uc, vc
                rep = gate(g, o, ray[None], osc, c1.diameter, L)
                kinds.append([k for k, v in rep["excused"].items() if v])
            if kinds[0] == []:
                continue  # the oracle reports this leaf itself (the float ray starts inside it)
            assert kinds == [["graze"], ["hard"], ["hard"]], (local, pid, kinds)
            checked += 1
    assert checked >= 10
