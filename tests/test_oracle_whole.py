"""Pins of the whole FP64 intersector: the bit-trail loop of Alg. 3 visits the same
domains as the explicit-stack recursion, dense tessellation (512 x 512 per patch)
agrees within the method's error bound (Sec. 3.4: false positives only), rays
through shared edges and corners never miss, and secondary rays follow the
offset rule of Sec. 3.3 in closed form."""
import numpy as np
import pytest

import oracle as O
from paper_1811_03510_amd import scenes as S


def rays_at_patches(cp, types, n, rng, spread=3.0):
    """Rays aimed at random surface points from random directions (some pass near)."""
    idx = rng.integers(0, cp.shape[0], size=n)
    u, v = rng.uniform(size=n), rng.uniform(size=n)
    x = S.surface_points(cp, types, idx, u, v)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x += rng.normal(size=(n, 3)) * 0.01 * (rng.uniform(size=(n, 1)) < 0.3)
    o = x - spread * rng.uniform(0.2, 1.0, size=(n, 1)) * d
    r = np.zeros((n, 8), np.float32)
    r[:, :3], r[:, 4:7], r[:, 7] = o, d, np.inf
    return r, idx


@pytest.fixture(scope="module", params=["world", "local"])
def oracle_any(request, c1, c1_oracle):
    """The oracle in world coordinates and with patch-local frames (Sec. 3.4)."""
    if request.param == "world":
        return c1_oracle
    return O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=True)


def test_bit_trail_loop_visits_the_recursion_sequence(c1, oracle_any):
    c1_oracle = oracle_any
    """Alg. 3 (pos/size/trail registers, ctz backtracking) and the explicit-stack
    recursion produce identical split sequences and hits on random ray-patch pairs."""
    rng = np.random.default_rng(11)
    rays, idx = rays_at_patches(c1.cp, c1.types, 60000, rng)
    greg = np.where(c1.types == 1)[0]
    # weight Gregory patches up (10^5 pairs in all)
    rays2, idx2 = rays_at_patches(c1.cp[greg], c1.types[greg], 40000, rng)
    rays = np.concatenate([rays, rays2])
    idx = np.concatenate([idx, greg[idx2]])
    caps = np.where(rng.uniform(size=len(rays)) < 0.3, rng.uniform(0.5, 3.0, size=len(rays)), np.inf)
    n_steps = n_hits = 0
    for k in range(len(rays)):
        a, ha = c1_oracle.trace_patch(idx[k], rays[k], caps[k])
        b, hb = c1_oracle.trace_patch_alg3(idx[k], rays[k], caps[k])
        assert a.shape == b.shape and np.array_equal(a, b), k
        # same leaf; t differs only by rounding (a cropped vs a split grid after backtracking)
        assert ha[1] == hb[1] and ha[2] == hb[2] and ha[3] == hb[3], k
        assert ha[0] == hb[0] or abs(ha[0] - hb[0]) <= 1e-12 * max(1.0, abs(ha[0])), k
        n_steps += len(a)
        n_hits += ha[1] != O.NO_HIT
    assert n_hits > 10000 and n_steps > 500000


def test_counters_are_consistent(c1, c1_oracle):
    r = c1_oracle.intersect(c1.primary, counters=True)
    c = r["counters"].astype(np.int64)
    hit = r["id"] != O.NO_HIT
    L = c1.leaf_depth
    # a recorded leaf needs 2L split steps on its path
    assert np.all(c[hit, 2] >= 2 * L)
    assert np.all(c[hit, 5] >= 1)
    assert np.all(c[~hit, 5] == 0)
    # every backtrack resumes a second child: at most one per split step
    assert np.all(c[:, 3] <= c[:, 2])


@pytest.mark.slow
def test_dense_tessellation_agrees_within_the_method_error_bound(c1, oracle_any):
    c1_oracle = oracle_any
    L = c1.leaf_depth
    rays = np.concatenate([c1.primary, c1.diffuse])  # every ray of the torus workload
    o = c1_oracle.intersect(rays)
    bf = c1_oracle.bruteforce(rays, res=512)
    eps_tess = 1e-6 * c1.diameter
    hit_o = o["id"] != O.NO_HIT
    hit_b = bf["id"] != O.NO_HIT
    assert hit_b.sum() > 10000
    # (i) no false negatives: a surface hit always has a method hit at or before it
    assert np.all(hit_o[hit_b])
    assert np.all(o["t"][hit_b] <= bf["t"][hit_b] + eps_tess)
    # every reported hit: the entry point lies within the leaf box diagonal of the
    # surface point at the leaf centre (both are in the leaf box)
    for k in np.where(hit_o)[0]:
        lo, hi = c1_oracle.leaf_box(o["id"][k], o["u"][k], o["v"][k])
        diag = np.linalg.norm(hi - lo)
        x = rays[k, :3].astype(np.float64) + o["t"][k] * rays[k, 4:7].astype(np.float64)
        f = O.patch_eval(c1.cp[o["id"][k]], bool(c1.types[o["id"][k]]), o["u"][k], o["v"][k])[0]
        assert np.linalg.norm(x - f) <= diag * (1 + 1e-9) + 1e-12, k
    # (ii) well-conditioned rays away from seams: same patch, t within the leaf
    # thickness along the normal, (u, v) within the distance that allows
    margin = 2.0 * 2.0 ** -L
    good = 0
    for k in np.where(hit_b)[0]:
        pid, ub, vb = bf["id"][k], bf["u"][k], bf["v"][k]
        if not (margin < ub < 1 - margin and margin < vb < 1 - margin):
            continue
        _, fu, fv = O.patch_eval(c1.cp[pid], bool(c1.types[pid]), ub, vb)
        nrm = np.cross(fu, fv)
        nrm /= np.linalg.norm(nrm)
        d = rays[k, 4:7].astype(np.float64)
        cosv = abs(np.dot(d, nrm)) / np.linalg.norm(d)
        if cosv < 0.1:
            continue
        good += 1
        assert o["id"][k] == pid, k
        lo, hi = c1_oracle.leaf_box(pid, o["u"][k], o["v"][k])
        diag = np.linalg.norm(hi - lo)
        gap = bf["t"][k] - o["t"][k]
        assert -eps_tess <= gap <= (diag + eps_tess) / (cosv * np.linalg.norm(d)), k
        smin = np.linalg.svd(np.stack([fu, fv], axis=1), compute_uv=False).min()
        leaf = 2.0 ** -L
        du = max(0.0, abs(o["u"][k] - ub) - leaf / 2)
        dv = max(0.0, abs(o["v"][k] - vb) - leaf / 2)
        assert np.hypot(du, dv) <= 1.5 * (gap * np.linalg.norm(d) + diag) / smin + 1e-9, k
    assert good > 8000


def test_rays_through_shared_edges_and_corners_never_miss(c1, oracle_any):
    c1_oracle = oracle_any
    rng = np.random.default_rng(21)
    nv = 16
    rays, targets = [], []
    for _ in range(1500):
        i, j = rng.integers(0, 32), rng.integers(0, nv)
        a = i * nv + j
        kind = rng.integers(0, 3)
        s = rng.uniform()
        if kind == 0:    # u-seam between (i, j) and (i+1, j)
            x = S.surface_points(c1.cp, c1.types, np.array([a]), np.array([1.0]), np.array([s]))[0]
        elif kind == 1:  # v-seam between (i, j) and (i, j+1)
            x = S.surface_points(c1.cp, c1.types, np.array([a]), np.array([s]), np.array([1.0]))[0]
        else:            # corner shared by four patches
            x = c1.cp[a, 15].astype(np.float64)
        if rng.uniform() < 0.5:
            o = np.array(c1.eye, np.float64)
            d = x - o
        else:
            d = rng.normal(size=3)
            o = x - rng.uniform(0.5, 2.0) * d
        d = d / np.linalg.norm(d)
        rays.append([*o, 0.0, *d, np.inf])
        targets.append(x)
    rays = np.array(rays, np.float32)
    targets = np.array(targets)
    h = c1_oracle.intersect(rays)
    o64, d64 = rays[:, :3].astype(np.float64), rays[:, 4:7].astype(np.float64)
    t_target = np.einsum("ij,ij->i", targets - o64, d64) / np.einsum("ij,ij->i", d64, d64)
    assert np.all(h["id"] != O.NO_HIT)
    assert np.all(h["t"] <= t_target + 1e-9 * c1.diameter)


def flat_patch_scene(L):
    g = np.zeros((16, 3))
    for j in range(4):
        for i in range(4):
            g[4 * j + i] = (-1.0 + 2.0 * i / 3.0, -1.0 + 2.0 * j / 3.0, 0.5)
    cp = np.concatenate([g, g[[5, 6, 9, 10]]]).astype(np.float32)
    return O.Scene(cp[None], np.array([0], np.uint8), L)


def test_bounce_closed_form_on_a_flat_patch():
    """Plane z = 0.5 over [-1, 1]^2: the leaf box is the leaf square, so the origin
    moves up by its L1 size 2 * 2 * 2^-L; u1 = 0 leaves along the normal."""
    L = 8
    sc = flat_patch_scene(L)
    leaf = 2.0 ** -L
    u, v = (37 + 0.5) * leaf, (200 + 0.5) * leaf
    x = np.array([-1 + 2 * u, -1 + 2 * v, 0.5])
    d = np.array([0.3, -0.2, -1.0])
    o = x - 2.0 * d
    ray = np.array([[*o, 0, *d, np.inf]], np.float32)
    t = float(np.float32(2.0))
    hit = np.array([[t, 0, u, v]], np.float32)
    hit[0, 1] = np.array([0], np.uint32).view(np.float32)[0]
    out = sc.bounce(ray, hit, np.array([[0.0, 0.25]], np.float32))
    xx = ray[0, :3].astype(np.float64) + t * ray[0, 4:7].astype(np.float64)
    np.testing.assert_allclose(out[0, :3], xx + np.array([0, 0, 4 * leaf]), atol=1e-15)
    np.testing.assert_allclose(out[0, 4:7], [0, 0, 1], atol=1e-15)
    assert out[0, 3] == 0 and out[0, 7] == np.inf
    # a miss gives an inactive ray (tmin > tmax)
    miss = np.array([[np.inf, 0, 0, 0]], np.float32)
    miss[0, 1] = np.array([0xFFFFFFFF], np.uint32).view(np.float32)[0]
    out = sc.bounce(ray, miss, np.array([[0.5, 0.5]], np.float32))
    assert out[0, 3] > out[0, 7]


def test_bounce_directions_are_cosine_weighted():
    L = 8
    sc = flat_patch_scene(L)
    n = 20000
    rng = np.random.default_rng(4)
    leaf = 2.0 ** -L
    u = (rng.integers(0, 1 << L, n) + 0.5) * leaf
    v = (rng.integers(0, 1 << L, n) + 0.5) * leaf
    x = np.stack([-1 + 2 * u, -1 + 2 * v, np.full(n, 0.5)], 1)
    d = np.tile([0.0, 0.0, -1.0], (n, 1))
    rays = np.zeros((n, 8), np.float32)
    rays[:, :3], rays[:, 4:7], rays[:, 7] = x + d * -1.5, d, np.inf
    hits = np.zeros((n, 4), np.float32)
    hits[:, 0], hits[:, 2], hits[:, 3] = 1.5, u, v
    out = sc.bounce(rays, hits, rng.uniform(size=(n, 2)).astype(np.float32))
    cz = out[:, 6]
    assert np.all(cz >= 0)
    np.testing.assert_allclose(np.linalg.norm(out[:, 4:7], axis=1), 1.0, atol=1e-6)
    # cosine-weighted: E[cos] = 2/3, E[cos^2] = 1/2
    assert abs(cz.mean() - 2 / 3) < 0.01 and abs((cz ** 2).mean() - 0.5) < 0.01


def test_gregory_patches_with_coincident_pairs_intersect_as_bezier(c1, oracle_any):
    """A Gregory patch whose paired inner points coincide is its Bézier patch (Sec. 3.2):
    on the torus with every patch tagged Gregory and P^v = P^u, Alg. 2 gives d = 0
    and the Bézier lower grid on every domain, so every ray gets the hit of the same
    scene tagged Bézier (same patch and leaf; t to the rounding of a crop against a
    split grid)."""
    cp = c1.cp.copy()
    cp[:, 16:20] = cp[:, [5, 6, 9, 10]]
    rays = np.concatenate([c1.primary, c1.diffuse])
    res = []
    for tag in (1, 0):
        osc = O.Scene(cp, np.full(len(cp), tag, np.uint8), c1.leaf_depth, local_frames=oracle_any.local_frames)
        res.append(osc.intersect(rays))
    g, b = res
    hit = b["id"] != O.NO_HIT
    assert hit.sum() > 10000
    assert np.array_equal(g["id"], b["id"]) and np.array_equal(g["u"], b["u"]) and np.array_equal(g["v"], b["v"])
    assert np.allclose(g["t"][hit], b["t"][hit], rtol=1e-12, atol=1e-14)
