"""The learned child ordering on the GPU against the FP64 references: network
inference on the matrix cores, loss gradients (fp32 and bfloat16), training
records, the traversal with the learned order (oracle gate for any weights,
launch-independent results), and what a trained network changes."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from oracle import policy as OP
from oracle.parity import assert_gate, gate
from paper_1811_03510_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ccs():
    from paper_1811_03510_amd import ccs as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


@pytest.fixture(scope="module")
def c1_gpu(ccs, c1):
    return ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth)


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    th = S.mlp_init(S.STREAM_MLP + seed).astype(np.float64) * scale
    th[M.N_PARAMS - 36:] += rng.normal(0, 0.1, 36)  # nonzero biases of the last layers too
    p = M.unpack(th)
    p["b1"] = rng.normal(0, 0.1, 32)
    p["b2"] = rng.normal(0, 0.1, 32)
    return M.pack(p).astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_inference_matches_the_reference(ccs):
    rng = np.random.default_rng(1)
    for n in (1, 15, 64, 100, 1000):
        th = _params(n)
        X = rng.uniform(-1, 1, (n, 16)).astype(np.float32)
        _say(f"inference on {n} rows")
        z = ccs.policy_infer(_dev(th), _dev(X)).cpu().numpy()
        zr, _ = M.forward(th, X, bf16=True)
        err = np.abs(z - zr)
        # fp32 sums instead of exact ones can move a hidden value across a bfloat16
        # rounding boundary (one unit in the last place, 2^-8 relative)
        assert np.all(err <= 2e-2 * np.maximum(1.0, np.abs(zr))), (n, err.max())
        assert np.median(err) <= 1e-4
        top = np.argmax(z, axis=1)
        srt = np.sort(zr, axis=1)
        clear = srt[:, -1] - srt[:, -2] > 0.05
        assert np.array_equal(top[clear], np.argmax(zr, axis=1)[clear])


def test_inference_layout_with_one_hot_paths(ccs):
    """Every input reaches every logit through one chosen unit per layer: a wrong
    operand layout would route it elsewhere."""
    for i in range(16):
        for o in range(4):
            p = {k: np.zeros(s) for k, s in M.LAYOUT}
            h1, h2 = (5 * i + o) % 32, (7 * i + 3 * o + 1) % 32
            p["W1"][h1, i] = 1.0
            p["W2"][h2, h1] = 2.0
            p["W3"][o, h2] = 0.5
            th = M.pack(p).astype(np.float32)
            X = np.zeros((64, 16), np.float32)
            X[:, i] = np.arange(64) / 8.0
            z = ccs.policy_infer(_dev(th), _dev(X)).cpu().numpy()
            want = np.zeros((64, 4))
            want[:, o] = np.arange(64) / 8.0
            assert np.array_equal(z, want), (i, o)


def _records(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (n, 16)).astype(np.float32)
    y = rng.integers(0, 4, n).astype(np.uint8)
    y[rng.random(n) < 0.2] = M.NO_LABEL
    return X, y


@pytest.mark.parametrize("n", [1, 63, 1000, 4161])
def test_gradient_fp32_matches_the_reference(ccs, n):
    th = _params(7)
    X, y = _records(n, n)
    loss, g = ccs.policy_grad(_dev(th), _dev(X), _dev(y), bf16=False)
    g = g.cpu().numpy()
    lr, gr = M.loss_and_grad(th, X, y)
    assert abs(loss - lr) <= 1e-5 * max(1.0, abs(lr))
    # fp32 sums of up to n terms: relative error of order sqrt(n) 2^-24 of the terms,
    # and a ReLU gate within rounding of zero can flip one sample's path (1/n)
    scale = max(np.abs(gr).max(), 1e-30)
    assert np.abs(g - gr).max() <= 1e-4 * scale, np.abs(g - gr).max() / scale
    if np.linalg.norm(gr) > 0:
        assert np.linalg.norm(g - gr) <= 2e-5 * np.linalg.norm(gr)


def test_gradient_bf16_matches_the_reference(ccs):
    th = _params(8)
    X, y = _records(3000, 9)
    loss, g = ccs.policy_grad(_dev(th), _dev(X), _dev(y), bf16=True)
    g = g.cpu().numpy()
    lr, gr = M.loss_and_grad(th, X, y, bf16=True)
    assert abs(loss - lr) <= 1e-2 * max(1.0, abs(lr))
    assert np.linalg.norm(g - gr) <= 1e-2 * np.linalg.norm(gr)


def test_gradient_of_no_labels_is_zero(ccs):
    th = _params(3)
    X, _ = _records(100, 3)
    loss, g = ccs.policy_grad(_dev(th), _dev(X), _dev(np.full(100, 255, np.uint8)))
    assert loss == 0.0 and not g.abs().max().item()


def test_training_is_deterministic_and_learns(ccs):
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (20000, 16)).astype(np.float32)
    y = (2 * (X[:, 12] > 0) + (X[:, 3] > X[:, 5])).astype(np.uint8)  # a learnable rule
    th0 = S.mlp_init()
    runs = []
    for _ in range(2):
        th = _dev(th0.copy())
        hist = ccs.policy_train(th, _dev(X), _dev(y), steps=400, batch=1024, lr=3e-3, seed=11, bf16=True)
        runs.append((th.cpu().numpy(), hist.cpu().numpy()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    hist = runs[0][1]
    _say(f"loss {hist[:10].mean():.3f} -> {hist[-10:].mean():.3f}")
    assert hist[-20:].mean() < 0.5 * hist[:10].mean()
    acc = (np.argmax(M.forward(runs[0][0], X, bf16=True)[0], axis=1) == y).mean()
    assert acc > 0.9, acc


def test_first_training_step_is_one_adam_update(ccs):
    th0 = _params(5)
    X, y = _records(512, 5)
    th = _dev(th0.copy())
    ccs.policy_train(th, _dev(X), _dev(y), steps=1, batch=512, lr=1e-3, seed=0, bf16=False)
    _, g = M.loss_and_grad(th0, X, y)
    want, _, _ = M.adam_step(th0.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS), g, 1, 1e-3)
    got = th.cpu().numpy()
    # the first Adam step moves each weight by lr * g / (|g| + eps): lr * sign(g) where |g| >> eps
    big = np.abs(g) > 1e-5
    assert np.allclose(got[big], want[big], rtol=0, atol=2e-6)


def test_second_step_carries_adams_moments(ccs):
    # step 1 from a fresh state, then step 2 resumed from the returned state: the
    # moments must follow the reference update from the state of step 1
    th0 = _params(6)
    X, y = _records(512, 6)
    th = _dev(th0.copy())
    adam = ccs.Adam()
    ccs.policy_train(th, _dev(X), _dev(y), steps=1, batch=512, lr=1e-3, seed=0, bf16=False, state=adam)
    assert adam.t == 1
    th1, m1, v1 = (a.cpu().numpy().astype(np.float64) for a in (th, adam.m, adam.v))
    ccs.policy_train(th, _dev(X), _dev(y), steps=1, batch=512, lr=1e-3, seed=0, bf16=False, state=adam)
    assert adam.t == 2
    _, g = M.loss_and_grad(th1, X, y)
    want, wm, wv = M.adam_step(th1, m1, v1, g, 2, 1e-3)
    big = np.abs(g) > 1e-3
    assert big.sum() > 100
    assert np.allclose(adam.m.cpu().numpy()[big], wm[big], rtol=1e-4, atol=0)
    assert np.allclose(adam.v.cpu().numpy()[big], wv[big], rtol=2e-4, atol=0)
    assert np.allclose(th.cpu().numpy()[big], want[big], rtol=0, atol=2e-6)


def test_training_resumes_bit_exactly_from_a_checkpoint(ccs, tmp_path):
    from paper_1811_03510_amd import checkpoint
    rng = np.random.default_rng(8)
    X = rng.uniform(-1, 1, (20000, 16)).astype(np.float32)
    y = (2 * (X[:, 1] > X[:, 2]) + (X[:, 7] > 0)).astype(np.uint8)
    kw = dict(batch=1024, lr=3e-3, seed=5, bf16=True)  # 19 steps an epoch: the cut falls inside the second
    th_a = _dev(S.mlp_init())
    hist_a = ccs.policy_train(th_a, _dev(X), _dev(y), steps=50, **kw).cpu().numpy()
    th_b = _dev(S.mlp_init())
    adam = ccs.Adam()
    h1 = ccs.policy_train(th_b, _dev(X), _dev(y), steps=23, state=adam, **kw).cpu().numpy()
    path = str(tmp_path / "policy.npz")
    checkpoint.save_training(path, th_b, adam, hyper=kw)
    del th_b, adam
    th_c, adam_c, hyper = checkpoint.load_training(path)
    assert adam_c.t == 23 and hyper == kw
    h2 = ccs.policy_train(th_c, _dev(X), _dev(y), steps=27, state=adam_c, **hyper).cpu().numpy()
    assert adam_c.t == 50
    assert np.array_equal(np.concatenate([h1, h2]).view(np.uint32), hist_a.view(np.uint32))
    assert np.array_equal(th_c.cpu().numpy().view(np.uint32), th_a.cpu().numpy().view(np.uint32))


def test_records_match_the_reference(ccs, c1, c1_gpu):
    rays = c1.diffuse[:3000]
    r = _dev(rays)
    h = c1_gpu.intersect(r)
    f, y = c1_gpu.record(r, h)
    hits, f, y = h.cpu().numpy(), f.cpu().numpy(), y.cpu().numpy()
    L = c1.leaf_depth
    ids = hits[:, 1].view(np.uint32)
    agree = total = 0
    worst = 0.0
    for i in np.flatnonzero(ids != O.NO_HIT)[:400]:
        p = int(ids[i])
        ff, yy = OP.path_records(c1.cp[p], bool(c1.types[p]), rays[i].astype(np.float64), float(hits[i, 2]),
                                 float(hits[i, 3]), L)
        gy = y[i * L:(i + 1) * L]
        gf = f[i * L:(i + 1) * L]
        both = (gy != 255) & (yy != 255)
        total += L
        agree += int(np.sum((gy != 255) == (yy != 255)))
        assert np.array_equal(gy[both], yy[both])
        if both.any():
            worst = max(worst, float(np.abs(gf[both] - ff[both]).max()))
    for i in np.flatnonzero(ids == O.NO_HIT)[:50]:
        assert np.all(y[i * L:(i + 1) * L] == 255) and np.all(f[i * L:(i + 1) * L] == 0)
    _say(f"decision flags agree on {agree}/{total}; worst input difference {worst:.2e}")
    assert agree >= 0.99 * total
    assert worst <= 2e-3


@pytest.mark.parametrize("kind", ["random", "contrarian"])
def test_learned_order_passes_the_gate_for_any_weights(ccs, c1, c1_gpu, c1_oracle, kind):
    """The order never decides a hit: even an untrained or adversarial network
    yields the oracle's hits to the gate's tolerance."""
    if kind == "random":
        th = _params(21, scale=3.0)
    else:  # always rank the grandchild farthest along the plain order first
        p = {k: np.zeros(s) for k, s in M.LAYOUT}
        p["W1"][0, 12], p["W1"][1, 12] = 4.0, -4.0
        p["W2"][0, 0], p["W2"][1, 1] = 1.0, 1.0
        p["W3"][0, 0], p["W3"][3, 1] = 1.0, 1.0  # lower u-half entered later -> pick it; else upper
        th = M.pack(p).astype(np.float32)
    rays = np.concatenate([c1.primary, c1.diffuse])
    r = _dev(rays)
    plain = c1_gpu.intersect(r).cpu().numpy()
    c1_gpu.set_policy(_dev(th))
    try:
        learned = c1_gpu.intersect(r).cpu().numpy()
        _, cnt_l = c1_gpu.intersect_counted(r)
        cnt_l = cnt_l.cpu().numpy()
    finally:
        c1_gpu.set_policy(None)
    _, cnt_p = c1_gpu.intersect_counted(r)
    cnt_p = cnt_p.cpu().numpy()
    same = np.mean(np.all(learned.view(np.uint32) == plain.view(np.uint32), axis=1))
    _say(f"{kind}: identical to closest-first on {same:.5f} of rays; splits/ray "
         f"{cnt_p[:, 2].mean():.2f} -> {cnt_l[:, 2].mean():.2f}")
    o = c1_oracle.intersect(rays)
    assert_gate(gate(learned, o, rays, c1_oracle, c1.diameter, c1.leaf_depth, label=f"learned-{kind}"))


def test_learned_order_is_launch_independent(ccs, c1, c1_gpu):
    rays = _dev(np.concatenate([c1.primary, c1.diffuse]))
    c1_gpu.set_policy(_dev(_params(22, scale=2.0)))
    try:
        c1_gpu.set_launch()
        base = c1_gpu.intersect(rays).cpu().numpy()
        for cfg in ((1, 1, 1, 1, 0, 1), (0, 64, 64, 64, 1, 64), (2, 8, 32, 4, 3, 3), (0, 33, 2, 7, 5, 17)):
            _say(f"learned launch {cfg}")
            c1_gpu.set_launch(*cfg)
            assert np.array_equal(c1_gpu.intersect(rays).cpu().numpy().view(np.uint32), base.view(np.uint32)), cfg
        # a ragged sub-launch gives the same per-ray results
        idx = np.random.default_rng(3).choice(rays.shape[0], 1001, replace=False)
        part = c1_gpu.intersect(rays[torch.from_numpy(idx).cuda()].contiguous()).cpu().numpy()
        assert np.array_equal(part.view(np.uint32), base[idx].view(np.uint32))
    finally:
        c1_gpu.set_launch()
        c1_gpu.set_policy(None)


def test_trained_network_against_closest_first(ccs, c1, c1_gpu, c1_oracle):
    """Trains on records from secondary rays of the torus (a seeded stream apart
    from the evaluation rays) and compares with the closest-first order: the
    u-half choice accuracy on held-out records, subdivision steps per ray and the
    oracle gate on the torus workload."""
    train_rays = _dev(S.policy_training_rays(1 << 17))
    h = c1_gpu.intersect(train_rays)
    f, y = c1_gpu.record(train_rays, h)
    keep = (y != 255).nonzero().squeeze(1)
    f, y = f[keep].contiguous(), y[keep].contiguous()
    n = f.shape[0]
    cut = int(0.9 * n)
    _say(f"{n} labelled records")
    th = _dev(S.mlp_init())
    hist = ccs.policy_train(th, f[:cut].contiguous(), y[:cut].contiguous(), steps=1500, batch=4096, lr=3e-3,
                            seed=1, bf16=True).cpu().numpy()
    _say(f"training loss {hist[:20].mean():.4f} -> {hist[-50:].mean():.4f}")
    assert hist[-50:].mean() < hist[:20].mean()
    fv, yv = f[cut:], y[cut:].cpu().numpy()
    z = ccs.policy_infer(th, fv.contiguous()).cpu().numpy()
    learned_u = np.argmax(z, axis=1) >> 1
    plain_u = (fv[:, 12].cpu().numpy() > 0).astype(np.int64)  # closest first: upper iff the lower is entered later
    true_u = yv >> 1
    acc_l, acc_p = (learned_u == true_u).mean(), (plain_u == true_u).mean()
    _say(f"u-half choice accuracy on held-out records: closest-first {acc_p:.4f}, learned {acc_l:.4f}")
    assert acc_l >= acc_p - 0.01
    rays = np.concatenate([c1.primary, c1.diffuse])
    r = _dev(rays)
    _, cp = c1_gpu.intersect_counted(r)
    c1_gpu.set_policy(th)
    try:
        hl, cl = c1_gpu.intersect_counted(r)
    finally:
        c1_gpu.set_policy(None)
    cp, cl = cp.cpu().numpy(), cl.cpu().numpy()
    o = c1_oracle.intersect(rays)
    assert_gate(gate(hl.cpu().numpy(), o, rays, c1_oracle, c1.diameter, c1.leaf_depth, label="learned-trained"))

    def mrays(policy):  # both ray classes of the torus workload in one launch, median of 7
        c1_gpu.set_policy(policy)
        try:
            hits = torch.empty((r.shape[0], 4), dtype=torch.float32, device="cuda")
            c1_gpu.intersect(r, hits)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(7)]
            for a, b in ev:
                a.record()
                c1_gpu.intersect(r, hits)
                b.record()
            torch.cuda.synchronize()
        finally:
            c1_gpu.set_policy(None)
        return r.shape[0] / np.median([a.elapsed_time(b) for a, b in ev]) / 1e3

    m_cf, m_l = mrays(None), mrays(th)
    s_cf, s_l = cp[:, 2].mean(), cl[:, 2].mean()
    _say(f"torus512, {r.shape[0]} rays: splits/ray closest-first {s_cf:.3f}, learned {s_l:.3f}; "
         f"re-crops/ray {cp[:, 6].mean():.3f} vs {cl[:, 6].mean():.3f}; "
         f"MRays/s closest-first {m_cf:.1f}, learned {m_l:.1f} ({m_l / m_cf:.3f}x)")
    # No child order saves more than 2 % of closest-first's split steps (the oracle's
    # hindsight and lookahead orders, test_oracle_order_bound.py), so a trained order
    # cannot either; and a sane network does not inflate the work by more than 10 %.
    assert 0.98 * s_cf <= s_l <= 1.10 * s_cf
    assert m_l > 0.3 * m_cf


def test_learned_order_in_local_frames_passes_the_gate(ccs, c1):
    """Learned order on a scene subdivided in patch-local frames: records, training
    and traversal in that frame; hits against the oracle in the same frame."""
    g = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth,
                  local_frames=True)
    osc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=True)
    tr = _dev(S.policy_training_rays(1 << 15))
    f, y = g.record(tr, g.intersect(tr))
    keep = (y != 255).nonzero().squeeze(1)
    f, y = f[keep].contiguous(), y[keep].contiguous()
    th = _dev(S.mlp_init())
    ccs.policy_train(th, f, y, steps=300, batch=2048, lr=3e-3, seed=2, bf16=True)
    rays = np.concatenate([c1.primary, c1.diffuse])
    g.set_policy(th)
    h = g.intersect(_dev(rays)).cpu().numpy()
    g.set_policy(None)
    assert_gate(gate(h, osc.intersect(rays), rays, osc, c1.diameter, c1.leaf_depth, label="learned-local"))
