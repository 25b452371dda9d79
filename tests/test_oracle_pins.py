"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test compares the oracle with something other than itself: a different
algorithm for the same quantity (de Casteljau evaluation vs the Bernstein sum,
Alg. 1's Hermite-form crop vs successive cropping), closed forms (affine
patches, Bernstein maxima), special cases (a Gregory patch with coincident
pairs is its Bezier patch, Sec. 2.2), invariants (convex-hull containment,
nesting, the sign table of the Gregory weights) and brute force.
"""
import numpy as np
import pytest

import oracle as O
from paper_1811_03510_amd import scenes as S

RNG = np.random.default_rng(1811)


def rand_grid(rng=RNG, scale=1.0):
    return rng.normal(size=(16, 3)) * scale


def rand_gregory(rng=RNG):
    cp = np.zeros((20, 3))
    cp[:16] = rand_grid(rng)
    cp[16:] = cp[[5, 6, 9, 10]] + rng.normal(size=(4, 3)) * 0.3
    return cp


def lerp(a, b, t):
    return (1.0 - t) * a + t * b


def casteljau_point(pts, t):
    """Point of a cubic by repeated linear interpolation (de Casteljau's algorithm)."""
    p = list(pts)
    while len(p) > 1:
        p = [lerp(p[k], p[k + 1], t) for k in range(len(p) - 1)]
    return p[0]


def casteljau_surface(grid16, u, v):
    g = np.asarray(grid16).reshape(4, 4, 3)  # [j, i]
    rows = [casteljau_point(g[j], u) for j in range(4)]
    return casteljau_point(rows, v)


# ----------------------------------------------------------------- evaluation
def test_bernstein_sum_equals_de_casteljau_and_interpolates_corners():
    for _ in range(50):
        g = rand_grid()
        u, v = RNG.uniform(size=2)
        f = O.bezier_eval(g, u, v)[0]
        np.testing.assert_allclose(f, casteljau_surface(g, u, v), rtol=0, atol=1e-13)
    g = rand_grid()
    for (u, v), s in {(0, 0): 0, (1, 0): 3, (0, 1): 12, (1, 1): 15}.items():
        assert np.array_equal(O.bezier_eval(g, u, v)[0], g[s])


def test_derivatives_match_finite_differences():
    h = 1e-5
    for _ in range(20):
        g = rand_grid()
        u, v = RNG.uniform(0.1, 0.9, size=2)
        f, fu, fv, fuv = O.bezier_eval(g, u, v)
        cfu = (casteljau_surface(g, u + h, v) - casteljau_surface(g, u - h, v)) / (2 * h)
        cfv = (casteljau_surface(g, u, v + h) - casteljau_surface(g, u, v - h)) / (2 * h)
        cfuv = (casteljau_surface(g, u + h, v + h) - casteljau_surface(g, u + h, v - h)
                - casteljau_surface(g, u - h, v + h) + casteljau_surface(g, u - h, v - h)) / (4 * h * h)
        np.testing.assert_allclose(fu, cfu, atol=1e-8)
        np.testing.assert_allclose(fv, cfv, atol=1e-8)
        np.testing.assert_allclose(fuv, cfuv, atol=1e-4)


def gregory_blend_point(cp, k, u, v):
    """Inner point k of a Gregory patch at (u, v) in the Alg. 2 weighting (test-side)."""
    i, j = (1 if k % 2 == 0 else 2), (1 if k < 2 else 2)
    du = u if i == 1 else 1 - u
    dv = v if j == 1 else 1 - v
    return (du * cp[[5, 6, 9, 10][k]] + dv * cp[16 + k]) / (du + dv)


def test_gregory_eval_is_blended_bezier_and_fd_derivatives():
    h = 1e-6
    for _ in range(20):
        cp = rand_gregory()
        u, v = RNG.uniform(0.05, 0.95, size=2)
        g = cp[:16].copy()
        for k, s in enumerate([5, 6, 9, 10]):
            g[s] = gregory_blend_point(cp, k, u, v)
        f, fu, fv = O.patch_eval(cp, True, u, v)
        np.testing.assert_allclose(f, casteljau_surface(g, u, v), atol=1e-13)
        fp = lambda uu, vv: O.patch_eval(cp, True, uu, vv)[0]
        np.testing.assert_allclose(fu, (fp(u + h, v) - fp(u - h, v)) / (2 * h), atol=2e-7)
        np.testing.assert_allclose(fv, (fp(u, v + h) - fp(u, v - h)) / (2 * h), atol=2e-7)


# ------------------------------------------------------------------- cropping
def alg1_crop(g, u0, u1, v0, v1):
    """Alg. 1 (Hermite form from corner values, first derivatives and twists), test-side."""
    du, dv = (u1 - u0) / 3.0, (v1 - v0) / 3.0
    E = {(a, b): O.bezier_eval(g, a, b) for a in (u0, u1) for b in (v0, v1)}
    f = lambda a, b: E[(a, b)][0]
    fu = lambda a, b: E[(a, b)][1]
    fv = lambda a, b: E[(a, b)][2]
    fuv = lambda a, b: E[(a, b)][3]
    q = np.zeros((4, 4, 3))  # [i, j]
    q[0, 0], q[3, 0], q[0, 3], q[3, 3] = f(u0, v0), f(u1, v0), f(u0, v1), f(u1, v1)
    q[1, 0] = q[0, 0] + du * fu(u0, v0)
    q[2, 0] = q[3, 0] - du * fu(u1, v0)
    q[0, 1] = q[0, 0] + dv * fv(u0, v0)
    q[3, 1] = q[3, 0] + dv * fv(u1, v0)
    q[0, 2] = q[0, 3] - dv * fv(u0, v1)
    q[3, 2] = q[3, 3] - dv * fv(u1, v1)
    q[1, 3] = q[0, 3] + du * fu(u0, v1)
    q[2, 3] = q[3, 3] - du * fu(u1, v1)
    q[1, 1] = q[1, 0] + dv * fv(u0, v0) + du * dv * fuv(u0, v0)
    q[2, 1] = q[3, 1] - du * fu(u1, v0) - du * dv * fuv(u1, v0)
    q[1, 2] = q[1, 3] - dv * fv(u0, v1) - du * dv * fuv(u0, v1)
    q[2, 2] = q[2, 3] - dv * fv(u1, v1) + du * dv * fuv(u1, v1)
    return q.transpose(1, 0, 2).reshape(16, 3)  # slot 4j + i


def test_crop_equals_alg1_and_reparametrised_evaluation():
    for _ in range(30):
        g = rand_grid()
        u0, u1 = np.sort(RNG.uniform(size=2))
        v0, v1 = np.sort(RNG.uniform(size=2))
        q = O.crop(g, u0, u1, v0, v1)
        np.testing.assert_allclose(q, alg1_crop(g, u0, u1, v0, v1), atol=1e-12)
        for s in np.linspace(0, 1, 9):
            for t in np.linspace(0, 1, 9):
                a = casteljau_surface(q, s, t)
                b = casteljau_surface(g, u0 + s * (u1 - u0), v0 + t * (v1 - v0))
                np.testing.assert_allclose(a, b, atol=1e-12)


def test_split_halves_equal_crop_to_halves():
    for _ in range(20):
        g = rand_grid()
        L, R = O.split(g, 0)
        np.testing.assert_allclose(L, O.crop(g, 0, 0.5, 0, 1), atol=1e-15)
        np.testing.assert_allclose(R, O.crop(g, 0.5, 1, 0, 1), atol=1e-15)
        L, R = O.split(g, 1)
        np.testing.assert_allclose(L, O.crop(g, 0, 1, 0, 0.5), atol=1e-15)
        np.testing.assert_allclose(R, O.crop(g, 0, 1, 0.5, 1), atol=1e-15)


# -------------------------------------------------------------------- Gregory
def test_gregory_with_coincident_pairs_is_its_bezier_patch():
    for _ in range(20):
        g = rand_grid()
        cp = np.concatenate([g, g[[5, 6, 9, 10]]])
        u, v = RNG.uniform(size=2)
        np.testing.assert_allclose(O.patch_eval(cp, True, u, v)[0], O.patch_eval(cp, False, u, v)[0],
                                   atol=1e-15)
        u0, u1 = np.sort(RNG.uniform(size=2))
        v0, v1 = np.sort(RNG.uniform(size=2))
        q, d = O.calc_points_and_d(cp, True, u0, u1, v0, v1)
        assert np.all(d == 0.0)
        np.testing.assert_array_equal(q, O.crop(g, u0, u1, v0, v1))


def test_gregory_convention_boundary_dependence():
    """P^u is the point used across the boundaries running along u (v = 0, v = 1), P^v
    across those running along v (u = 0, u = 1): checked by perturbing each point."""
    cp = rand_gregory()
    us = np.linspace(0.1, 0.9, 5)
    edges = {  # edge -> (parameter map, derivative index, inner points used)
        "v0": (lambda s: (s, 0.0), 2, {5: "u", 6: "u"}),
        "v1": (lambda s: (s, 1.0), 2, {9: "u", 10: "u"}),
        "u0": (lambda s: (0.0, s), 1, {5: "v", 9: "v"}),
        "u1": (lambda s: (1.0, s), 1, {6: "v", 10: "v"}),
    }
    pv_slot = {5: 16, 6: 17, 9: 18, 10: 19}
    for name, (uv, deriv, used) in edges.items():
        base = [O.patch_eval(cp, True, *uv(s)) for s in us]
        for slot in (5, 6, 9, 10):
            for which, sl in (("u", slot), ("v", pv_slot[slot])):
                c2 = cp.copy()
                c2[sl] += 0.37
                pert = [O.patch_eval(c2, True, *uv(s)) for s in us]
                same_point = all(np.allclose(a[0], b[0], atol=1e-14) for a, b in zip(base, pert))
                assert same_point, (name, sl)  # inner points never move the boundary curve
                same_cross = all(np.allclose(a[deriv], b[deriv], atol=1e-12) for a, b in zip(base, pert))
                should_move = used.get(slot) == which
                assert same_cross != should_move, (name, slot, which)


def test_gregory_weight_table_and_extremes():
    """Signs of the weight derivatives (the table of Sec. 2.2) and A/B as the blends at
    the two extreme corners; every blend over D lies between them."""
    h = 1e-7
    for k in range(4):
        i, j = (1 if k % 2 == 0 else 2), (1 if k < 2 else 2)
        # paper weight on P^u in Sec. 2.2 (printed form): g = dv / (du + dv)
        def g(u, v):
            du = u if i == 1 else 1 - u
            dv = v if j == 1 else 1 - v
            return dv / (du + dv)
        table = {(1, 1): (-1, +1), (2, 1): (+1, +1), (1, 2): (-1, -1), (2, 2): (+1, -1)}[(i, j)]
        for _ in range(100):
            u, v = RNG.uniform(0.01, 0.99, size=2)
            su = np.sign(g(u + h, v) - g(u - h, v))
            sv = np.sign(g(u, v + h) - g(u, v - h))
            assert su in (table[0], 0) and sv in (table[1], 0)
    for _ in range(40):
        cp = rand_gregory()
        u0, u1 = np.sort(RNG.uniform(size=2))
        v0, v1 = np.sort(RNG.uniform(size=2))
        A, B = O.inner_extremes(cp, u0, u1, v0, v1)
        for k in range(4):
            i, j = (1 if k % 2 == 0 else 2), (1 if k < 2 else 2)
            # the smallest weight on P^u is at small du and large dv, the largest opposite
            ua = u0 if i == 1 else u1
            va = v1 if j == 1 else v0
            ub = u1 if i == 1 else u0
            vb = v0 if j == 1 else v1
            np.testing.assert_allclose(A[k], gregory_blend_point(cp, k, ua, va), atol=1e-12)
            np.testing.assert_allclose(B[k], gregory_blend_point(cp, k, ub, vb), atol=1e-12)
            lo, hi = np.minimum(A[k], B[k]), np.maximum(A[k], B[k])
            for s in np.linspace(0, 1, 33):
                for t in np.linspace(0, 1, 33):
                    p = gregory_blend_point(cp, k, u0 + s * (u1 - u0), v0 + t * (v1 - v0))
                    assert np.all(p >= lo - 1e-12) and np.all(p <= hi + 1e-12)


def test_bernstein_weight_maxima():
    b1 = lambda t: 3 * t * (1 - t) ** 2
    b2 = lambda t: 3 * t * t * (1 - t)
    assert O.wbar(1, 0.0, 1.0) == pytest.approx(4.0 / 9.0, abs=4e-16)
    assert O.wbar(2, 0.0, 1.0) == pytest.approx(4.0 / 9.0, abs=4e-16)
    assert b1(1 / 3) == pytest.approx(4 / 9) and b2(2 / 3) == pytest.approx(4 / 9)
    for _ in range(500):
        t0, t1 = np.sort(RNG.uniform(size=2))
        ts = np.linspace(t0, t1, 2001)
        for k, b in ((1, b1), (2, b2)):
            w = O.wbar(k, t0, t1)
            assert w >= b(ts).max() - 1e-15
            assert w <= b(ts).max() + 1e-6  # attained up to sampling


# ------------------------------------------------------------------- bounding
def random_domain(L, rng=RNG):
    """A random dyadic domain at a random depth 0..2L (alternating u, v splits)."""
    depth = int(rng.integers(0, 2 * L + 1))
    su, sv = 1 << 23, 1 << 23
    pu = pv = 0
    for k in range(depth):
        if k % 2 == 0:
            su >>= 1
            pu += su * int(rng.integers(0, 2))
        else:
            sv >>= 1
            pv += sv * int(rng.integers(0, 2))
    s = 2.0 ** -23
    return pu * s, (pu + su) * s, pv * s, (pv + sv) * s, depth


def box_of(q, d):
    return q.min(axis=0), q.max(axis=0) + d


def test_boxes_are_conservative_and_bezier_boxes_nest(c1):
    rng = np.random.default_rng(7)
    idx = np.concatenate([np.where(c1.types == 1)[0][:12], np.where(c1.types == 0)[0][:6]])
    for pid in idx:
        cp = c1.cp[pid].astype(np.float64)
        greg = bool(c1.types[pid])
        ext = np.ptp(cp.reshape(-1, 3), axis=0).max()
        for _ in range(12):
            u0, u1, v0, v1, depth = random_domain(c1.leaf_depth, rng)
            q, d = O.calc_points_and_d(cp, greg, u0, u1, v0, v1)
            lo, hi = box_of(q, d)
            axis = depth % 2
            L, R = O.split(q, axis)
            halves = ((u0, (u0 + u1) / 2, v0, v1), ((u0 + u1) / 2, u1, v0, v1)) if axis == 0 else \
                ((u0, u1, v0, (v0 + v1) / 2), (u0, u1, (v0 + v1) / 2, v1))
            for s in np.linspace(0, 1, 33):
                for t in np.linspace(0, 1, 33):
                    uu, vv = u0 + s * (u1 - u0), v0 + t * (v1 - v0)
                    f = O.patch_eval(cp, greg, uu, vv)[0]
                    assert np.all(f >= lo - 1e-12 * ext) and np.all(f <= hi + 1e-12 * ext)
                    for child, (a0, a1, b0, b1) in zip((L, R), halves):
                        if a0 <= uu <= a1 and b0 <= vv <= b1:
                            clo, chi = box_of(child, d)
                            assert np.all(f >= clo - 1e-12 * ext) and np.all(f <= chi + 1e-12 * ext)
            if not greg:
                for child in (L, R):
                    clo, chi = box_of(child, 0)
                    assert np.all(clo >= lo - 1e-15 * ext) and np.all(chi <= hi + 1e-15 * ext)


def test_alg3_leaf_box_bounds_its_leaf(c1, c1_oracle):
    """The box a leaf is recorded by (Alg. 3: its half of the parent's lower grid,
    grown by the parent's displacement) bounds the surface over the leaf's domain
    (Sec. 3.2); for a Bezier patch it is the leaf's own crop box (split halves are
    crops, Alg. 1), and leaf_entry is finite exactly when a slab test of the box hits."""
    from oracle.parity import _path_in_box
    rng = np.random.default_rng(17)
    L = c1.leaf_depth
    n = 2 ** L
    loc = O.Scene(c1.cp, c1.types, L, local_frames=True)
    idx = np.concatenate([np.where(c1.types == 1)[0][:8], np.where(c1.types == 0)[0][:4]])
    for pid in idx:
        cp = c1.cp[pid].astype(np.float64)
        greg = bool(c1.types[pid])
        ext = np.ptp(cp.reshape(-1, 3), axis=0).max()
        R = loc.patch_frame(pid)
        for _ in range(6):
            iu, iv = rng.integers(0, n, 2)
            uc, vc = (iu + 0.5) / n, (iv + 0.5) / n
            for sc, rot in ((c1_oracle, np.eye(3)), (loc, R)):
                lo, hi = sc.leaf_box_alg3(pid, uc, vc)
                assert np.all(hi >= lo)
                for s in np.linspace(0, 1, 9):
                    for t in np.linspace(0, 1, 9):
                        f = rot @ O.patch_eval(cp, greg, (iu + s) / n, (iv + t) / n)[0]
                        assert np.all(f >= lo - 1e-12 * ext) and np.all(f <= hi + 1e-12 * ext)
                if not greg:
                    olo, ohi = sc.leaf_box(pid, uc, vc)
                    assert np.allclose(lo, olo, rtol=0, atol=1e-12 * ext)
                    assert np.allclose(hi, ohi, rtol=0, atol=1e-12 * ext)
            # rays through the box's centre hit it; rays passing beside it miss
            lo, hi = c1_oracle.leaf_box_alg3(pid, uc, vc)
            c = 0.5 * (lo + hi)
            for off, want in ((0.0, True), (1.5, False)):
                d = rng.normal(size=3)
                d /= np.linalg.norm(d)
                side = np.cross(d, rng.normal(size=3))
                side /= np.linalg.norm(side)
                p = c + off * np.linalg.norm(hi - lo) * side
                ray = np.array([*(p - 2.0 * d), 0.0, *d, np.inf], np.float32)
                e = c1_oracle.leaf_entry(pid, ray, uc, vc)
                assert np.isfinite(e) == want
                assert (_path_in_box(ray, lo, hi) >= 0) == want
                if want:
                    assert abs(e - 2.0) <= 0.5 * np.linalg.norm(hi - lo) + 1e-6


def test_displacement_vanishes_towards_corners_and_edges(c1):
    pid = int(np.where(c1.types == 1)[0][0])
    cp = c1.cp[pid].astype(np.float64)
    for corner in ((0, 0), (1, 0), (0, 1), (1, 1), (0.5, 0), (0, 0.5), (0.37, 0.61)):
        ds = []
        for k in range(1, 20):
            s = 2.0 ** -k
            u0 = min(max(corner[0] - s / 2, 0.0), 1.0 - s)
            v0 = min(max(corner[1] - s / 2, 0.0), 1.0 - s)
            _, d = O.calc_points_and_d(cp, True, u0, u0 + s, v0, v0 + s)
            ds.append(np.abs(d).max())
        ds = np.array(ds)
        assert ds[-1] < 1e-4 * ds[0] + 1e-14
        assert np.all(ds[1:] <= ds[:-1] * 1.0 + 1e-15)  # non-increasing along the chain


# ---------------------------------------------------- whole intersector pins
def affine_patch(a, e1, e2):
    g = np.zeros((16, 3))
    for j in range(4):
        for i in range(4):
            g[4 * j + i] = a + (i / 3.0) * e1 + (j / 3.0) * e2
    return g


@pytest.mark.parametrize("L", [3, 7, 12, 17, 22])
def test_affine_patch_closed_form(L):
    """f = a + u e1 + v e2 exactly (degree elevation of a plane).  With (u*, v*, t*) the
    closed-form ray/plane solution, the reported hit obeys the method's error bound:
    the entered leaf box precedes the surface by at most its thickness along the
    normal, and the leaf lies within that distance plus its box diagonal of (u*, v*)."""
    rng = np.random.default_rng(L)
    checked = 0
    for trial in range(60):
        # a and the per-index steps e1 / 3, e2 / 3 on a 2^-10 grid: every control point
        # a + i e1/3 + j e2/3 is exact in fp32, so the patch is exactly the plane even at
        # leaf depths where rounding a point off the plane would exceed a leaf's thickness
        a, q1, q2 = (np.round(rng.normal(size=3) * 1024.0) / 1024.0 for _ in range(3))
        g = np.array([a + i * q1 + j * q2 for j in range(4) for i in range(4)])
        cp = np.concatenate([g, g[[5, 6, 9, 10]]]).astype(np.float32)
        assert np.array_equal(cp.astype(np.float64), np.concatenate([g, g[[5, 6, 9, 10]]]))
        sc = O.Scene(cp[None], np.array([trial % 2], np.uint8), L)
        c64 = cp.astype(np.float64)
        a32, e1, e2 = c64[0], c64[3] - c64[0], c64[12] - c64[0]
        nrm = np.cross(e1, e2)
        nrm /= np.linalg.norm(nrm)
        us, vs = rng.uniform(0.02, 0.98, size=2)
        d = rng.normal(size=3)
        if abs(np.dot(d, nrm)) < 0.2 * np.linalg.norm(d):
            continue
        ray = np.array([*(a32 + us * e1 + vs * e2 - 3.0 * d), 0.0, *d, np.inf], np.float32)
        o64, d64 = ray[:3].astype(np.float64), ray[4:7].astype(np.float64)
        u_s, v_s, t_s = np.linalg.solve(np.stack([e1, e2, -d64], axis=1), o64 - a32)
        h = sc.intersect(ray[None])
        assert h["id"][0] == 0
        leaf = 2.0 ** -L
        diag = np.linalg.norm(leaf * (np.abs(e1) + np.abs(e2)))
        gap = t_s - h["t"][0]
        assert -1e-12 <= gap <= diag / abs(np.dot(d64, nrm)) + 1e-12
        du = max(0.0, abs(h["u"][0] - u_s) - leaf / 2)
        dv = max(0.0, abs(h["v"][0] - v_s) - leaf / 2)
        smin = np.linalg.svd(np.stack([e1, e2], axis=1), compute_uv=False).min()
        assert np.hypot(du, dv) <= (gap * np.linalg.norm(d64) + diag) / smin + 1e-12
        checked += 1
    assert checked >= 20


def test_axis_aligned_plane_gives_exact_t():
    L = 10
    g = affine_patch(np.array([-1.0, -1.0, 0.5]), np.array([2.0, 0, 0]), np.array([0, 2.0, 0]))
    cp = np.concatenate([g, g[[5, 6, 9, 10]]]).astype(np.float32)
    sc = O.Scene(cp[None], np.array([0], np.uint8), L)
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = np.array([*rng.normal(scale=0.1, size=2), -1.0])
        o = np.array([*rng.uniform(-0.8, 0.8, size=2), 0.5]) - 2.5 * d
        ray = np.array([*o, 0.0, *d, np.inf], np.float32)
        h = sc.intersect(ray[None])
        t_exact = (np.float64(np.float32(0.5)) - np.float64(ray[2])) / np.float64(ray[6])
        assert h["id"][0] == 0 and h["t"][0] == t_exact


def test_special_rays():
    """Zero direction components, origin inside a box, tmin > tmax, zero direction."""
    L = 6
    g = affine_patch(np.array([-1.0, -1.0, 0.0]), np.array([2.0, 0, 0]), np.array([0, 2.0, 0]))
    cp = np.concatenate([g, g[[5, 6, 9, 10]]]).astype(np.float32)
    sc = O.Scene(cp[None], np.array([0], np.uint8), L)
    rays = np.array([
        [0.25, 0.25, 1.0, 0.0, 0.0, 0.0, -1.0, np.inf],   # axis-aligned, hits at t=1
        [0.25, 0.25, 1.0, 0.0, 0.0, 0.0, 1.0, np.inf],    # away from the plane
        [2.0, 0.25, 1.0, 0.0, 0.0, 0.0, -1.0, np.inf],    # outside the slab in x
        [0.25, 0.25, 1.0, 2.0, 0.0, 0.0, -1.0, 1.5],      # tmin > tmax
        [0.25, 0.25, 1.0, 0.0, 0.0, 0.0, 0.0, np.inf],    # zero direction
        [0.25, 0.25, 1.0, 0.0, 0.0, 0.0, -1.0, 0.5],      # tmax before the plane
        [0.25, 0.25, 1.0, 0.0, 0.0, 0.0, -1.0, 1.0],      # tmax exactly at the plane
    ], np.float32)
    h = sc.intersect(rays)
    assert h["id"][0] == 0 and h["t"][0] == 1.0
    assert list(h["id"][1:6]) == [O.NO_HIT] * 5
    assert h["id"][6] == 0 and h["t"][6] == 1.0
