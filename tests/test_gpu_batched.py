"""Frames, batched launches and HIP-graph replay (animation playback): hits of a
batched launch equal single-batch launches of the same rays bitwise, each frame
matches the oracle on that frame's geometry, and a captured frame loop replays
to the eager result every time."""
import numpy as np
import pytest

import oracle as O
from oracle.parity import assert_gate, gate, ids_of
from paper_1811_03510_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def anim():
    return S.config3(n_frames=4, lo=1 << 10, hi=1 << 14)


@pytest.fixture(scope="module", params=["world", "local"])
def scene(anim, request):
    from paper_1811_03510_amd import ccs
    g = ccs.Scene(torch.from_numpy(anim.cp0).cuda(), torch.from_numpy(anim.types).cuda(), anim.leaf_depth,
                  local_frames=request.param == "local")
    g.set_frames(len(anim.frames))
    for f, cp in enumerate(anim.frames):
        g.refit_frame(f, torch.from_numpy(cp).cuda())
    torch.cuda.synchronize()
    return g


def test_frames_match_the_oracle(anim, scene):
    for f, (cp, rays) in enumerate(zip(anim.frames, anim.rays)):
        _say(f"frame {f}: {len(rays)} rays")
        (h,) = scene.intersect_batched([(f, torch.from_numpy(rays).cuda(), None)])
        torch.cuda.synchronize()
        osc = O.Scene(cp, anim.types, anim.leaf_depth, local_frames=scene.local_frames)
        assert_gate(gate(h.cpu().numpy(), osc.intersect(rays), rays, osc, anim.diameter, anim.leaf_depth,
                         label=f"anim-frame{f}"))


def test_batched_launch_equals_single_batches(anim, scene):
    rng = np.random.default_rng(9)
    parts = []
    for f, rays in enumerate(anim.rays):
        cut = np.sort(rng.choice(len(rays), size=3, replace=False))
        for a, b in zip([0, *cut], [*cut, len(rays)]):
            parts.append((f, rays[a:b]))
    parts.append((1, anim.rays[1][:0]))  # an empty batch
    rng.shuffle(parts)
    parts = parts[:32]
    dev = [(f, torch.from_numpy(np.ascontiguousarray(r)).cuda(), None) for f, r in parts]
    _say(f"batched launch of {len(dev)} batches")
    many = scene.intersect_batched(dev)
    singles = [scene.intersect_batched([d])[0] for d in dev]
    torch.cuda.synchronize()
    for a, b in zip(many, singles):
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))


def test_frame0_batch_equals_intersect(anim, scene):
    r = torch.from_numpy(anim.rays[0]).cuda()
    a = scene.intersect(r)
    (b,) = scene.intersect_batched([(0, r, None)])
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))


def test_batch_limits(anim, scene):
    from paper_1811_03510_amd import ccs
    r = torch.from_numpy(anim.rays[0][:10]).cuda()
    with pytest.raises(ccs.CcsError):
        scene.intersect_batched([(0, r, None)] * 33)
    with pytest.raises(ccs.CcsError):
        scene.intersect_batched([(len(anim.frames), r, None)])


def test_graph_captured_frame_loop_replays(anim, scene):
    """[refit every frame -> one batched launch] captured once, replayed three times
    with eager work and synchronizations between the replays."""
    cps = [torch.from_numpy(cp).cuda() for cp in anim.frames]
    rays = [torch.from_numpy(r).cuda() for r in anim.rays]
    hits = [torch.empty((r.shape[0], 4), dtype=torch.float32, device="cuda") for r in rays]
    batches = [(f, rays[f], hits[f]) for f in range(len(rays))]

    def loop():
        for f, cp in enumerate(cps):
            scene.refit_frame(f, cp)
        scene.intersect_batched(batches)

    loop()
    torch.cuda.synchronize()
    eager = [h.cpu().numpy().copy() for h in hits]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        loop()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        loop()
    for rep in range(3):
        for h in hits:
            h.fill_(-1.0)
        x = torch.randn(1 << 20, device="cuda")  # eager work between replays
        (x * 2).sum().item()
        _say(f"graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        for e, h in zip(eager, hits):
            assert np.array_equal(e.view(np.uint32), h.cpu().numpy().view(np.uint32))


def test_autotuner_picks_a_setting_and_caches_it(anim, scene, tmp_path, monkeypatch):
    from paper_1811_03510_amd import autotune
    monkeypatch.setenv("CCS_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    rays = [torch.from_numpy(r).cuda() for r in anim.rays]
    batches = [(f, r, None) for f, r in enumerate(rays)]
    ref = [h.cpu().numpy() for h in scene.intersect_batched(batches)]
    small = dict(waves_per_cu=[0, 4], fetch_min=[8, 16], traverse_min=[1], grid_min=[16], traverse_steps=[1, 2])
    monkeypatch.setattr(autotune, "SPACE", small)
    p = autotune.tuned(scene, batches, name="anim-test", reps=1, log=_say)

    def same(q):
        cur = scene.get_launch()
        return all(cur[k] == v for k, v in q.items() if not (k == "waves_per_cu" and v == 0))
    assert same(p)
    assert (tmp_path / "tune.json").exists()
    scene.set_launch()  # defaults
    q = autotune.tuned(scene, batches, name="anim-test", reps=1, log=_say)  # from the cache
    assert q == p and same(p)
    got = [h.cpu().numpy() for h in scene.intersect_batched(batches)]
    scene.set_launch()
    for a, b in zip(ref, got):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_bounce_on_a_frame_uses_that_frames_geometry(anim, scene):
    """Secondary rays from hits on frame f follow frame f's surface (oracle on that frame)."""
    rng = np.random.default_rng(17)
    f = len(anim.frames) - 1
    cp = anim.frames[f]
    n, L = 2000, anim.leaf_depth
    idx = rng.integers(0, cp.shape[0], n)
    leaf = 2.0 ** -L
    u = (rng.integers(0, 1 << L, n) + 0.5) * leaf
    v = (rng.integers(0, 1 << L, n) + 0.5) * leaf
    x = S.surface_points(cp, anim.types, idx, u, v)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t = rng.uniform(0.5, 2.0, size=n)
    rays = np.zeros((n, 8), np.float32)
    rays[:, :3], rays[:, 4:7], rays[:, 7] = x - t[:, None] * d, d, np.inf
    hits = np.zeros((n, 4), np.float32)
    hits[:, 0], hits[:, 2], hits[:, 3] = t, u, v
    hits[:, 1] = idx.astype(np.uint32).view(np.float32)
    w = rng.uniform(size=(n, 2)).astype(np.float32)
    ref = O.Scene(cp, anim.types, L, local_frames=scene.local_frames).bounce(rays, hits, w)
    out = scene.bounce(torch.from_numpy(rays).cuda(), torch.from_numpy(hits).cuda(), torch.from_numpy(w).cuda(),
                       frame=f)
    out0 = scene.bounce(torch.from_numpy(rays).cuda(), torch.from_numpy(hits).cuda(), torch.from_numpy(w).cuda())
    out, out0 = out.cpu().numpy().astype(np.float64), out0.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(out[:, :3], ref[:, :3], atol=2e-6 * anim.diameter)
    np.testing.assert_allclose(out[:, 4:7], ref[:, 4:7], atol=2e-5)
    assert np.abs(out0[:, :3] - ref[:, :3]).max() > 1e-4  # frame 0's geometry is elsewhere
    from paper_1811_03510_amd import ccs
    with pytest.raises(ccs.CcsError):
        scene.bounce(torch.from_numpy(rays).cuda(), torch.from_numpy(hits).cuda(), torch.from_numpy(w).cuda(),
                     frame=len(anim.frames))


def test_graph_captured_refit_intersect_bounce_loop(anim, scene):
    """[refit every frame -> one batched launch -> bounce rays on every frame ->
    one batched launch of the bounces] captured once and replayed three times,
    each replay bitwise equal to the eager loop; the bounce hits pass the oracle
    gate on every frame."""
    F = len(anim.frames)
    cps = [torch.from_numpy(cp).cuda() for cp in anim.frames]
    rays = [torch.from_numpy(r).cuda() for r in anim.rays]
    hits = [torch.empty((r.shape[0], 4), dtype=torch.float32, device="cuda") for r in rays]
    bray = [torch.empty_like(r) for r in rays]
    bhit = [torch.empty_like(h) for h in hits]
    rng = np.random.default_rng(8)
    unif = [torch.from_numpy(rng.uniform(size=(r.shape[0], 2)).astype(np.float32)).cuda() for r in rays]

    def loop():
        for f in range(F):
            scene.refit_frame(f, cps[f])
        scene.intersect_batched([(f, rays[f], hits[f]) for f in range(F)])
        for f in range(F):
            scene.bounce(rays[f], hits[f], unif[f], out=bray[f], frame=f)
        scene.intersect_batched([(f, bray[f], bhit[f]) for f in range(F)])

    loop()
    torch.cuda.synchronize()
    eager = [h.cpu().numpy().copy() for h in bhit]
    eager_rays = [r.cpu().numpy().copy() for r in bray]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        loop()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        loop()
    for rep in range(3):
        for h, r in zip(bhit, bray):
            h.fill_(-1.0)
            r.fill_(0.0)
        (torch.randn(1 << 20, device="cuda") * 3).sum().item()  # eager work between replays
        _say(f"bounce-loop graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        for e, er, h, r in zip(eager, eager_rays, bhit, bray):
            assert np.array_equal(er.view(np.uint32), r.cpu().numpy().view(np.uint32))
            assert np.array_equal(e.view(np.uint32), h.cpu().numpy().view(np.uint32))
    for f in range(F):
        osc = O.Scene(anim.frames[f], anim.types, anim.leaf_depth, local_frames=scene.local_frames)
        r = eager_rays[f]
        assert_gate(gate(eager[f], osc.intersect(r), r, osc, anim.diameter, anim.leaf_depth,
                         label=f"bounce-frame{f}"))


def test_combined_pipeline_with_learned_order(anim, scene):
    """The combined workload in small: every frame refit, one batched launch of the
    primary rays of all frames, then two bounce levels, each generated per frame from
    the previous level's hits and intersected in one batched launch, with the learned
    child order on (an untrained network: the order never decides a hit).  Every
    (frame, level) passes the oracle gate on that frame's geometry."""
    from paper_1811_03510_amd import ccs
    F, levels = len(anim.frames), 3
    rng = np.random.default_rng(31)
    theta = torch.from_numpy((rng.normal(size=ccs.POLICY_PARAMS) * 0.5).astype(np.float32)).cuda()
    cps = [torch.from_numpy(cp).cuda() for cp in anim.frames]
    rays = [[torch.from_numpy(r).cuda() for r in anim.rays]]
    hits = []
    scene.set_policy(theta)
    try:
        for f in range(F):
            scene.refit_frame(f, cps[f])
        for b in range(levels):
            if b > 0:
                nxt = []
                for f in range(F):
                    w = torch.from_numpy(rng.uniform(size=(rays[b - 1][f].shape[0], 2)).astype(np.float32)).cuda()
                    nxt.append(scene.bounce(rays[b - 1][f], hits[b - 1][f], w, frame=f))
                rays.append(nxt)
            hits.append(list(scene.intersect_batched([(f, rays[b][f], None) for f in range(F)])))
        torch.cuda.synchronize()
    finally:
        scene.set_policy(None)
    for b in range(levels):
        for f in (0, F - 1):
            r, h = rays[b][f].cpu().numpy(), hits[b][f].cpu().numpy()
            osc = O.Scene(anim.frames[f], anim.types, anim.leaf_depth, local_frames=scene.local_frames)
            _say(f"combined: level {b}, frame {f}: {len(r)} rays")
            assert_gate(gate(h, osc.intersect(r), r, osc, anim.diameter, anim.leaf_depth,
                             label=f"combined-level{b}-frame{f}"))


def test_combined_pipeline_at_one_million_patches():
    """The combined pipeline at the 1M-patch scale: two animation frames of the
    1M-patch scene (the seeded displacement), each refit on the GPU, the 1920x1080
    primary rays of both frames in one batched launch, then one bounce level
    generated per frame from those hits and intersected in one batched launch with
    the learned order on (an untrained network: the order never decides a hit).
    Each (frame, level) passes the oracle gate on 32,768 seeded rays of that frame's
    geometry, and the counted batched launch gives bitwise the same hits."""
    from paper_1811_03510_amd import ccs
    w = S.config2(with_diffuse=False)
    F = 2
    frames = [S.animate(w.cp, f, 8) for f in (0, 5)]
    _say("1M combined: building the scene and two frames")
    sc = ccs.Scene(torch.from_numpy(w.cp).cuda(), torch.from_numpy(w.types).cuda(), w.leaf_depth, local_frames=True)
    sc.set_frames(F)
    cps = [torch.from_numpy(c).cuda() for c in frames]
    for f in range(F):
        sc.refit_frame(f, cps[f])
    prim = torch.from_numpy(w.primary).cuda()
    h0 = sc.intersect_batched([(f, prim, None) for f in range(F)])
    rng = np.random.default_rng(41)
    brays = []
    for f in range(F):
        u = torch.from_numpy(rng.uniform(size=(prim.shape[0], 2)).astype(np.float32)).cuda()
        brays.append(sc.bounce(prim, h0[f], u, frame=f))
    theta = torch.from_numpy((rng.normal(size=ccs.POLICY_PARAMS) * 0.5).astype(np.float32)).cuda()
    sc.set_policy(theta)
    try:
        _say("1M combined: bounce level, learned order")
        h1 = sc.intersect_batched([(f, brays[f], None) for f in range(F)])
        torch.cuda.synchronize()
    finally:
        sc.set_policy(None)
    hc, _ = sc.intersect_batched([(f, prim, None) for f in range(F)], counted=True)
    torch.cuda.synchronize()
    for f in range(F):
        assert np.array_equal(hc[f].cpu().numpy().view(np.uint32), h0[f].cpu().numpy().view(np.uint32))
    # the bounce level compacted to its active rays (ccs_compact_rays) and traced in one batched
    # launch gives, closest-first, the full level's hits at the kept rays and misses elsewhere
    full = sc.intersect_batched([(f, brays[f], None) for f in range(F)])
    packed = [ccs.compact_rays(brays[f]) for f in range(F)]
    torch.cuda.synchronize()
    m = [int(wk[0].item()) for _, _, wk in packed]
    part = sc.intersect_batched([(f, packed[f][0][:m[f]], None) for f in range(F)])
    torch.cuda.synchronize()
    for f in range(F):
        idx = packed[f][1][:m[f]].cpu().numpy()
        fh = full[f].cpu().numpy()
        _say(f"1M combined: frame {f}, bounce level compacted to {m[f]} of {len(fh)} rays")
        assert 0.2 * len(fh) < m[f] < len(fh)
        assert np.array_equal(part[f].cpu().numpy().view(np.uint32), fh[idx].view(np.uint32))
        rest = np.ones(len(fh), bool)
        rest[idx] = False
        assert (ids_of(fh[rest]) == O.NO_HIT).all()
    for f in range(F):
        osc = O.Scene(frames[f], w.types, w.leaf_depth, local_frames=True)
        for lvl, (r, h) in enumerate(((prim, h0[f]), (brays[f], h1[f]))):
            r_np, h_np = r.cpu().numpy(), h.cpu().numpy()
            active = np.flatnonzero(r_np[:, 3] <= r_np[:, 7])  # rays of missed pixels are inactive
            sel = active[S.sample_indices(len(active), min(32768, len(active)), seed=300 + 10 * f + lvl)]
            _say(f"1M combined: frame {f}, level {lvl}: gate on {len(sel)} of {len(active)} active rays")
            rep = gate(h_np[sel], osc.intersect(r_np[sel]), r_np[sel], osc, w.diameter, w.leaf_depth,
                       label=f"1M-combined-frame{f}-level{lvl}")
            assert_gate(rep)
            assert rep["oracle_hits"] > 1000
        del osc
