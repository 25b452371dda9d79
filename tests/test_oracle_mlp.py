"""Pins of the FP64 reference of the ordering network and of its inputs:
finite differences, closed forms of small networks, rounding cases of bfloat16,
the first Adam step, and the geometric meaning of every policy input."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from oracle import policy as P
from paper_1811_03510_amd import scenes as S


def _rand(seed, n=64):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.4, M.N_PARAMS)
    X = rng.normal(0, 1, (n, 16))
    y = rng.integers(0, 4, n).astype(np.uint8)
    y[::7] = M.NO_LABEL
    return theta, X, y


def test_layout_counts():
    assert sum(int(np.prod(s)) for _, s in M.LAYOUT) == M.N_PARAMS == S.N_POLICY_PARAMS
    th = np.arange(M.N_PARAMS, dtype=np.float64)
    assert np.array_equal(M.pack(M.unpack(th)), th)
    p = M.unpack(th)
    assert p["W1"][0, 1] == 1 and p["b1"][0] == 512 and p["W2"][0, 0] == 544 and p["b3"][3] == 1731


def test_gradient_matches_central_differences():
    theta, X, y = _rand(1)
    _, g = M.loss_and_grad(theta, X, y)
    h = 1e-6
    fd = np.zeros_like(theta)
    for k in range(M.N_PARAMS):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (M.loss(theta + e, X, y) - M.loss(theta - e, X, y)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_zero_network_closed_form():
    _, X, y = _rand(2)
    z, _ = M.forward(np.zeros(M.N_PARAMS), X)
    assert np.all(z == 0)
    L, g = M.loss_and_grad(np.zeros(M.N_PARAMS), X, y)
    assert abs(L - np.log(4.0)) < 1e-15
    m = y != M.NO_LABEL
    onehot = np.eye(4)[y[m].astype(int)]
    gp = M.unpack(g)
    assert np.allclose(gp["b3"], (0.25 - onehot).mean(axis=0), atol=1e-16, rtol=0)
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert np.all(gp[k] == 0)


def test_single_path_network_by_hand():
    p = {k: np.zeros(s) for k, s in M.LAYOUT}
    p["W1"][0, 0], p["W2"][0, 0], p["W3"][1, 0] = 2.0, 3.0, 0.5
    th = M.pack(p)
    X = np.zeros((2, 16))
    X[0, 0], X[1, 0] = 1.5, -1.5
    z, _ = M.forward(th, X)
    assert np.allclose(z[0], [0, 4.5, 0, 0]) and np.all(z[1] == 0)  # ReLU closes the path for x0 < 0
    L = M.loss(th, X[:1], np.array([1], np.uint8))
    assert abs(L - (-4.5 + np.log(3 + np.exp(4.5)))) < 1e-14
    # dL/dW3[1,0] = (p1 - 1) h2_0 with h2_0 = 9
    _, g = M.loss_and_grad(th, X[:1], np.array([1], np.uint8))
    p1 = np.exp(4.5) / (3 + np.exp(4.5))
    assert abs(M.unpack(g)["W3"][1, 0] - (p1 - 1) * 9.0) < 1e-14


def test_unlabelled_samples_carry_nothing():
    theta, X, y = _rand(3)
    L, g = M.loss_and_grad(theta, X, np.full_like(y, M.NO_LABEL))
    assert L == 0 and np.all(g == 0)
    # adding unlabelled samples changes neither loss nor gradient
    m = y != M.NO_LABEL
    L1, g1 = M.loss_and_grad(theta, X[m], y[m])
    L2, g2 = M.loss_and_grad(theta, X, y)
    assert abs(L1 - L2) < 1e-14 and np.max(np.abs(g1 - g2)) < 1e-15


def test_softmax_shift_invariance():
    theta, X, y = _rand(4)
    _, g = M.loss_and_grad(theta, X, y)
    assert abs(M.unpack(g)["b3"].sum()) < 1e-15
    p = M.unpack(theta)
    p2 = dict(p, b3=p["b3"] + 7.25)
    assert abs(M.loss(M.pack(p2), X, y) - M.loss(theta, X, y)) < 1e-12


def test_bf16_rounding_cases():
    one = 1.0
    cases = [(one, one), (1 + 2**-8, 1.0), (1 + 3 * 2**-8, 1 + 2**-6), (1 + 2**-8 + 2**-20, 1 + 2**-7),
             (-(1 + 3 * 2**-8), -(1 + 2**-6)), (3.0, 3.0), (2**-130, 2**-130), (65504.0, 65536.0)]
    for x, want in cases:
        assert M.bf16_round(np.float32(x)) == want, x


def test_bf16_mode_is_exact_on_representable_values():
    rng = np.random.default_rng(5)
    th = rng.integers(-4, 5, M.N_PARAMS).astype(np.float64) / 8.0
    X = rng.integers(-3, 4, (32, 16)).astype(np.float64) / 4.0
    # weights and inputs are exact in bfloat16; where the hidden values are too (8
    # significant bits), the bf16 network must equal the exact one bit for bit
    z0, c = M.forward(th, X)
    z1, c1 = M.forward(th, X, bf16=True)
    rows = np.all(M.bf16_round(c["h1"].astype(np.float32)) == c["h1"], axis=1)
    rows &= np.all(M.bf16_round(c["h2"].astype(np.float32)) == c["h2"], axis=1)
    assert rows.sum() >= 4
    assert np.array_equal(z0[rows], z1[rows])
    # the rounding is idempotent
    assert np.array_equal(M.bf16_round(c1["h1"].astype(np.float32)), c1["h1"])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(6)
    th, g = rng.normal(size=50), rng.normal(size=50)
    t1, m, v = M.adam_step(th, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_order_projection():
    z = np.array([[0, 1, 2, 3], [3, 0, 0, 0], [1, 1, 0, 0], [0, 0, 5, 5], [0, 2, 0, 1]], float)
    u, v = M.predict_order(z)
    assert list(u) == [1, 0, 0, 1, 0] and list(v) == [1, 0, 0, 0, 1]


def test_init_is_seeded_and_scaled():
    a, b = S.mlp_init(), S.mlp_init()
    assert a.dtype == np.float32 and np.array_equal(a, b)
    p = M.unpack(a)
    assert np.abs(p["W1"]).max() <= np.sqrt(6 / 16) and np.abs(p["W2"]).max() <= np.sqrt(6 / 32)
    assert np.all(p["b1"] == 0) and 0.3 < p["W1"].std() < 0.4  # a / sqrt(3) for U(-a, a), a = 0.61


# ------------------------------------------------------------ policy inputs
def test_onb_is_orthonormal_and_right_handed():
    rng = np.random.default_rng(7)
    ns = [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]), np.array([1.0, 0, 0])]
    ns += [v / np.linalg.norm(v) for v in rng.normal(size=(200, 3))]
    for n in ns:
        e1, e2 = P.onb(n)
        B = np.stack([e1, e2, n])
        assert np.allclose(B @ B.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(e1, e2), n, atol=1e-12)


def _scene_ray(seed):
    cp, types = S.torus_scene()
    rng = np.random.default_rng(seed)
    k = int(rng.integers(0, len(cp)))
    u, v = rng.uniform(0.1, 0.9, 2)
    greg = bool(types[k])
    x = O.patch_eval(cp[k], greg, u, v)[0]
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    o = x - 0.7 * d
    ray = np.array([*o, 0.0, *d, np.inf])
    return cp[k], greg, ray


def test_corner_inputs_reconstruct_the_surface_corners():
    checked = 0
    for seed in range(40):
        cp20, greg, ray = _scene_ray(seed)
        for k, (u0, v0, size) in enumerate([(0.0, 0.0, 1.0), (0.5, 0.25, 0.25), (0.375, 0.625, 0.125)]):
            f, ok = P.node_features(cp20, greg, ray, u0, v0, size, 2 * k, 12, np.inf)
            if not ok:
                continue
            # rebuild the frame and the entry point independently of the feature code
            q, disp = O.calc_points_and_d(cp20, greg, u0, u0 + size, v0, v0 + size)
            lo_a = O.crop(q, 0.0, 0.5, 0.0, 1.0).min(axis=0)
            hi_a = O.crop(q, 0.0, 0.5, 0.0, 1.0).max(axis=0) + disp
            lo_b = O.crop(q, 0.5, 1.0, 0.0, 1.0).min(axis=0)
            hi_b = O.crop(q, 0.5, 1.0, 0.0, 1.0).max(axis=0) + disp
            o, d = ray[:3], ray[4:7]
            ent = []
            for lo, hi in ((lo_a, hi_a), (lo_b, hi_b)):
                t0, t1 = (lo - o) / d, (hi - o) / d
                ent.append((max(0.0, np.minimum(t0, t1).max()), np.maximum(t0, t1).min()))
            p = o + min(ent[0][0], ent[1][0]) * d
            e1, e2 = P.onb(d)
            loc = f[:12].reshape(4, 3)
            # a Bezier node's corners are surface points; a Gregory node's are those of
            # its lower bounding grid (Alg. 2), evaluated at the corners of [0, 1]^2
            if greg:
                corners = [O.bezier_eval(q, uu, vv)[0] for uu, vv in ((0, 0), (1, 0), (0, 1), (1, 1))]
            else:
                corners = [O.patch_eval(cp20, greg, uu, vv)[0] for uu, vv in
                           ((u0, v0), (u0 + size, v0), (u0, v0 + size), (u0 + size, v0 + size))]
            rel = np.array([[np.dot(c - p, e1), np.dot(c - p, e2), np.dot(c - p, d)] for c in corners])
            s = np.abs(rel).max()
            assert np.allclose(loc * s, rel, atol=1e-9 * max(1, s))
            assert abs(np.abs(loc).max() - 1.0) < 1e-12
            dl = np.linalg.norm(d)
            assert abs(f[12] - np.clip((ent[0][0] - ent[1][0]) * dl / s, -4, 4) / 4) < 1e-9
            assert abs(f[13] - np.clip((ent[0][1] - ent[1][1]) * dl / s, -4, 4) / 4) < 1e-9
            assert f[14] == 2 * k / 24 and f[15] == float(greg)
            checked += 1
    assert checked >= 20


def test_inputs_invariant_under_translation_and_scaling():
    for seed in range(10):
        cp20, greg, ray = _scene_ray(100 + seed)
        f0, ok0 = P.node_features(cp20, greg, ray, 0.0, 0.0, 1.0, 0, 12, np.inf)
        shift = np.array([3.0, -2.0, 5.0])
        cp2 = (cp20.astype(np.float64) * 4.0 + shift)
        ray2 = ray.copy()
        ray2[:3] = ray[:3] * 4.0 + shift
        f1, ok1 = P.node_features(cp2, greg, ray2, 0.0, 0.0, 1.0, 0, 12, np.inf)
        assert ok0 == ok1
        if ok0:
            assert np.allclose(f0, f1, atol=1e-12)


def test_path_labels_name_the_leaf():
    cp20, greg, ray = _scene_ray(300)
    L = 6
    u, v = (37 + 0.5) / 64, (10 + 0.5) / 64
    _, labels = P.path_records(cp20, greg, ray, u, v, L, np.inf)
    iu = iv = 0
    for k in range(L):
        lab = labels[k]
        if lab == P.NO_LABEL:  # not a decision: recover the bits from (u, v) itself
            lab = 2 * ((37 >> (L - 1 - k)) & 1) + ((10 >> (L - 1 - k)) & 1)
        iu, iv = 2 * iu + (lab >> 1), 2 * iv + (lab & 1)
    assert (iu, iv) == (37, 10)
