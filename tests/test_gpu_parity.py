"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the
same seeded inputs, at sizes spanning many waves with ragged tails, and at the
full 1M-patch / 1920x1080 size on a seeded sample of rays."""
import numpy as np
import pytest

import oracle as O
from paper_1811_03510_amd import scenes as S

from oracle.parity import assert_gate, gate, ids_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# rays per class the oracle checks at full size (same hit/miss and patch on >= 99.99 %)
GATE_RAYS = 131072


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ccs():
    from paper_1811_03510_amd import ccs as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


@pytest.fixture(scope="module", params=["world", "local"])
def frames(request):
    """Subdivision in world coordinates, or in patch-local frames (Sec. 3.4)."""
    return request.param == "local"


@pytest.fixture(scope="module")
def c1_gpu(ccs, c1, frames):
    _say(f"building the 512-patch torus scene on the GPU (local frames: {frames})")
    return ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth,
                     local_frames=frames)


@pytest.fixture(scope="module")
def c1_ref(c1, c1_oracle, frames):
    """The oracle in the same frames as c1_gpu."""
    return O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=True) if frames else c1_oracle


def run(scene, rays_np):
    r = torch.from_numpy(np.ascontiguousarray(rays_np, dtype=np.float32)).cuda()
    h = scene.intersect(r)
    torch.cuda.synchronize()
    return h.cpu().numpy()


@pytest.mark.parametrize("cls", ["primary", "diffuse"])
def test_torus512_all_rays(ccs, c1, c1_ref, c1_gpu, cls):
    c1_oracle = c1_ref
    rays = c1.primary if cls == "primary" else c1.diffuse
    _say(f"torus512 {cls}: {len(rays)} rays")
    g = run(c1_gpu, rays)
    o = c1_oracle.intersect(rays)
    assert_gate(gate(g, o, rays, c1_oracle, c1.diameter, c1.leaf_depth, label=f"torus512-{cls}"))


@pytest.mark.parametrize("L", [17, 18, 20])
def test_torus512_deep_leaf_depths(ccs, c1, L, frames):
    """Leaf depths above 16 (64-bit path and trail words): every torus ray against the
    oracle at the same L, in both frame modes; the variants kept to 32-bit words refuse
    such a scene."""
    rays = np.concatenate([c1.primary, c1.diffuse])
    gsc = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), L, local_frames=frames)
    osc = O.Scene(c1.cp, c1.types, L, local_frames=frames)
    _say(f"torus512 at L = {L}: {len(rays)} rays")
    g = run(gsc, rays)
    o = osc.intersect(rays)
    assert_gate(gate(g, o, rays, osc, c1.diameter, L, label=f"torus512-L{L}"))
    hit = ids_of(g) != O.NO_HIT
    assert hit.sum() > 10000
    # reported (u, v) are centres of leaves of size 2^-L
    k = g[hit, 2:4].astype(np.float64) * 2.0 ** L - 0.5
    assert np.array_equal(k, np.round(k))
    theta = torch.zeros(ccs.POLICY_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(ccs.CcsError):
        gsc.set_policy(theta)
    with pytest.raises(ccs.CcsError):
        gsc.debug_grids(np.zeros(1, np.uint32), np.zeros(1, np.uint32), np.zeros(1, np.uint32))
    with pytest.raises(ccs.CcsError):
        ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), L, single_box=True)


def test_ragged_launches_are_bitwise_identical(ccs, c1, c1_gpu):
    """Per-ray results do not depend on the launch size or the ray's position in it."""
    rays = c1.diffuse
    full = run(c1_gpu, rays)
    rng = np.random.default_rng(3)
    for n in (1, 63, 64, 65, 1000, 4097):
        idx = rng.choice(len(rays), size=n, replace=False)
        _say(f"ragged launch of {n} rays")
        part = run(c1_gpu, rays[idx])
        assert np.array_equal(part.view(np.uint32), full[idx].view(np.uint32)), n


def test_launch_configuration_never_changes_results(ccs, c1, c1_gpu):
    """Persistent waves, phase thresholds and waves per CU only change speed."""
    rays = np.concatenate([c1.primary, c1.diffuse])
    c1_gpu.set_launch()
    base = run(c1_gpu, rays)
    for w, f, t, g, k in ((1, 1, 1, 1, 0), (0, 64, 64, 64, 1), (2, 8, 32, 4, 3), (0, 1, 64, 1, 0), (3, 33, 2, 64, 7)):
        _say(f"launch waves/CU={w} fetch>={f} traverse>={t} grid>={g} steps={k}")
        c1_gpu.set_launch(w, f, t, g, k)
        assert np.array_equal(run(c1_gpu, rays).view(np.uint32), base.view(np.uint32)), (w, f, t, g, k)
    c1_gpu.set_launch()
    with pytest.raises(ccs.CcsError):
        c1_gpu.set_launch(0, 0, 16, 16)


def test_counted_kernel_gives_the_same_hits(ccs, c1, c1_gpu, c1_ref):
    c1_oracle = c1_ref
    r = torch.from_numpy(c1.primary).cuda()
    h0 = c1_gpu.intersect(r)
    h1, cnt = c1_gpu.intersect_counted(r)
    torch.cuda.synchronize()
    h0, h1, cnt = h0.cpu().numpy(), h1.cpu().numpy(), cnt.cpu().numpy().astype(np.int64)
    assert np.array_equal(h0.view(np.uint32), h1.view(np.uint32))
    hit = ids_of(h1) != O.NO_HIT
    L = c1.leaf_depth
    assert np.all(cnt[hit, 2] >= 2 * L) and np.all(cnt[hit, 5] >= 1) and np.all(cnt[~hit, 5] == 0)
    # same algorithm: totals of the per-patch work agree with the oracle's to a few percent
    oc = c1_oracle.intersect(c1.primary, counters=True)["counters"].astype(np.int64)
    for k in (2, 3, 4, 5, 6, 7):
        a, b = cnt[:, k].sum(), oc[:, k].sum()
        assert abs(a - b) <= 0.05 * max(a, b) + 10, (k, a, b)


def test_empty_inputs(ccs, c1, c1_gpu):
    r = torch.zeros((0, 8), dtype=torch.float32, device="cuda")
    h = c1_gpu.intersect(r)
    assert h.shape == (0, 4)
    empty = ccs.Scene(torch.zeros((0, 20, 3), dtype=torch.float32).cuda(),
                      torch.zeros((0,), dtype=torch.uint8).cuda(), 12)
    g = run(empty, c1.primary[:100])
    assert np.all(ids_of(g) == O.NO_HIT) and np.all(np.isinf(g[:, 0]))


def affine_cp(rng):
    a, e1, e2 = rng.normal(size=3), rng.normal(size=3), rng.normal(size=3)
    g = np.array([[a + (i / 3) * e1 + (j / 3) * e2 for i in range(4)] for j in range(4)]).reshape(16, 3)
    return np.concatenate([g, g[[5, 6, 9, 10]]])


@pytest.mark.parametrize("L", [1, 4, 12, 16, 17, 20])
def test_single_patches_and_special_rays(ccs, L, frames):
    rng = np.random.default_rng(L)
    for trial in range(4):
        cp = affine_cp(rng) if trial < 2 else S.config1(8, 8, False).cp[rng.integers(0, 512)].astype(np.float64)
        cp = cp.astype(np.float32)[None]
        ty = np.array([trial % 2], np.uint8)
        osc = O.Scene(cp, ty, L, local_frames=frames)
        gsc = ccs.Scene(torch.from_numpy(cp).cuda(), torch.from_numpy(ty).cuda(), L, local_frames=frames)
        x = S.surface_points(cp, ty, np.zeros(256, np.int64), rng.uniform(size=256), rng.uniform(size=256))
        d = rng.normal(size=(256, 3))
        rays = np.zeros((256 + 6, 8), np.float32)
        rays[:256, :3], rays[:256, 4:7], rays[:256, 7] = x - 2.0 * d, d, np.inf
        c = x[0]
        rays[256:] = [[c[0], c[1], c[2] + 5, 0, 0, 0, -1, np.inf],      # axis-aligned
                      [c[0], c[1], c[2] + 5, 0, 0, 0, 0, np.inf],       # zero direction
                      [c[0], c[1], c[2] + 5, 3, 0, 0, -1, 2],           # tmin > tmax
                      [np.nan, 0, 0, 0, 0, 0, 1, np.inf],               # non-finite origin
                      [c[0], c[1], c[2], 0, 1, 0, 0, np.inf],           # origin on the surface
                      [c[0], c[1], c[2] + 5, 0, 0, 0, -1, 0.5]]         # tmax too short
        _say(f"single patch L={L} trial {trial}")
        g = run(gsc, rays)
        o = osc.intersect(rays)
        diam = float(np.linalg.norm(np.ptp(cp.reshape(-1, 3).astype(np.float64), axis=0)))
        assert_gate(gate(g, o, rays, osc, diam, L, label=f"single-L{L}-{trial}"))
        assert np.all(ids_of(g)[[257, 258, 259]] == O.NO_HIT)


def test_rays_through_shared_edges_never_miss(ccs, c1, c1_gpu):
    rng = np.random.default_rng(5)
    nv = 16
    pts = []
    for _ in range(4000):
        i, j = rng.integers(0, 32), rng.integers(0, nv)
        a = np.array([i * nv + j])
        kind, s = rng.integers(0, 3), rng.uniform()
        if kind == 0:
            x = S.surface_points(c1.cp, c1.types, a, np.array([1.0]), np.array([s]))[0]
        elif kind == 1:
            x = S.surface_points(c1.cp, c1.types, a, np.array([s]), np.array([1.0]))[0]
        else:
            x = c1.cp[a[0], 15].astype(np.float64)
        pts.append(x)
    pts = np.array(pts)
    o = np.array(c1.eye)[None] + rng.normal(size=(len(pts), 3)) * 0.3
    d = pts - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((len(pts), 8), np.float32)
    rays[:, :3], rays[:, 4:7], rays[:, 7] = o, d, np.inf
    g = run(c1_gpu, rays)
    t_target = np.einsum("ij,ij->i", pts - rays[:, :3], rays[:, 4:7].astype(np.float64))
    missed = ids_of(g) == O.NO_HIT
    assert missed.sum() == 0, np.where(missed)[0][:10]
    assert np.all(g[:, 0] <= t_target + 1e-4 * c1.diameter)


def test_bounce_matches_oracle(ccs, c1, c1_ref, c1_gpu):
    c1_oracle = c1_ref
    """Secondary rays from the same (ray, hit, uniforms) inputs on both sides."""
    rng = np.random.default_rng(8)
    n = 4096
    idx = rng.integers(0, 512, size=n)
    L = c1.leaf_depth
    leaf = 2.0 ** -L
    u = (rng.integers(0, 1 << L, n) + 0.5) * leaf
    v = (rng.integers(0, 1 << L, n) + 0.5) * leaf
    x = S.surface_points(c1.cp, c1.types, idx, u, v)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t = rng.uniform(0.5, 2.0, size=n)
    rays = np.zeros((n, 8), np.float32)
    rays[:, :3], rays[:, 4:7], rays[:, 7] = x - t[:, None] * d, d, np.inf
    hits = np.zeros((n, 4), np.float32)
    hits[:, 0], hits[:, 2], hits[:, 3] = t, u, v
    hits[:, 1] = idx.astype(np.uint32).view(np.float32)
    hits[::17, 1] = np.array([O.NO_HIT], np.uint32).view(np.float32)[0]
    hits[::17, 0] = np.inf
    w = rng.uniform(size=(n, 2)).astype(np.float32)
    ref = c1_oracle.bounce(rays, hits, w)
    out = c1_gpu.bounce(torch.from_numpy(rays).cuda(), torch.from_numpy(hits).cuda(), torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    active = ref[:, 3] <= ref[:, 7]
    assert np.array_equal(active, out[:, 3] <= out[:, 7])
    np.testing.assert_allclose(out[active, :3], ref[active, :3], atol=2e-6 * c1.diameter)
    np.testing.assert_allclose(out[active, 4:7], ref[active, 4:7], atol=2e-5)


def test_refit_matches_oracle_on_moved_scene(ccs, c1, frames):
    """Moving the control points (a smooth displacement field: shared points move
    together) and refitting gives the oracle's hits on the moved scene; refitting
    back gives bitwise the original hits."""
    cp0 = c1.cp.astype(np.float64)
    x = cp0.reshape(-1, 3)
    k = np.array([[0.9, 0.3, 0.1], [0.2, -0.7, 0.5], [0.1, 0.4, -0.9]]) * 2 * np.pi
    disp = 0.01 * np.sin(x @ k.T + np.array([0.3, 1.1, 2.0]))
    cp1 = (x + disp).reshape(cp0.shape).astype(np.float32)
    gsc = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth,
                    local_frames=frames)
    base = run(gsc, c1.primary)
    _say("refit to moved control points")
    gsc.refit(torch.from_numpy(cp1).cuda())
    g = run(gsc, c1.primary)
    osc = O.Scene(cp1, c1.types, c1.leaf_depth, local_frames=frames)
    o = osc.intersect(c1.primary)
    assert_gate(gate(g, o, c1.primary, osc, c1.diameter, c1.leaf_depth, label="torus512-refit"))
    gsc.refit(torch.from_numpy(c1.cp))  # host input
    back = run(gsc, c1.primary)
    assert np.array_equal(back.view(np.uint32), base.view(np.uint32))


def test_instanced_1m_full_size_sampled(ccs, frames):
    """1,000,000 patches, 1920x1080 primary + secondary rays, one launch per class and
    both classes in one launch as the benchmark times them, closest-first and learned
    order; the oracle checks a seeded sample of 131,072 rays of each class."""
    _say("generating the 1M-patch scene")
    w = S.config2()
    gsc = ccs.Scene(torch.from_numpy(w.cp).cuda(), torch.from_numpy(w.types).cuda(), w.leaf_depth,
                    local_frames=frames)
    osc = O.Scene(w.cp, w.types, w.leaf_depth, local_frames=frames)
    classes = (("primary", w.primary), ("diffuse", w.diffuse))
    single = {}
    for cls, rays in classes:
        _say(f"1M {cls}: {len(rays)} rays on the GPU")
        g = single[cls] = run(gsc, rays)
        sel = S.sample_indices(len(rays), GATE_RAYS, seed=77 if cls == "primary" else 78)
        o = osc.intersect(rays[sel])
        rep = gate(g[sel], o, rays[sel], osc, w.diameter, w.leaf_depth, label=f"1M-{cls}-sample")
        assert_gate(rep)
        assert rep["oracle_hits"] > 500
    # the benchmark's launch: both classes in one batched launch, bitwise the same hits;
    # then the same launch with the learned child order (an untrained network) on the
    # same samples against the oracle
    dev = [torch.from_numpy(r).cuda() for _, r in classes]
    both = gsc.intersect_batched([(0, r, None) for r in dev])
    torch.cuda.synchronize()
    for (cls, _), h in zip(classes, both):
        assert np.array_equal(h.cpu().numpy().view(np.uint32), single[cls].view(np.uint32)), cls
    rng = np.random.default_rng(23)
    gsc.set_policy(torch.from_numpy((rng.normal(size=ccs.POLICY_PARAMS) * 0.5).astype(np.float32)).cuda())
    try:
        _say("1M: learned order, both classes in one launch")
        learned = gsc.intersect_batched([(0, r, None) for r in dev])
        torch.cuda.synchronize()
    finally:
        gsc.set_policy(None)
    for (cls, rays), h in zip(classes, learned):
        sel = S.sample_indices(len(rays), GATE_RAYS, seed=77 if cls == "primary" else 78)
        rep = gate(h.cpu().numpy()[sel], osc.intersect(rays[sel]), rays[sel], osc, w.diameter, w.leaf_depth,
                   label=f"1M-{cls}-learned-sample")
        assert_gate(rep)


def test_instanced_1m_refit_to_an_animation_frame(ccs, frames):
    """The 1M-patch scene refit to a frame of the seeded animation (every level of
    its 27-deep BVH refit in its own launch) against the oracle on that frame."""
    _say("generating the 1M-patch scene and an animation frame")
    w = S.config2(with_diffuse=False)
    cp1 = S.animate(w.cp, 5, 16)
    gsc = ccs.Scene(torch.from_numpy(w.cp).cuda(), torch.from_numpy(w.types).cuda(), w.leaf_depth,
                    local_frames=frames)
    gsc.refit(torch.from_numpy(cp1).cuda())
    sel = S.sample_indices(len(w.primary), GATE_RAYS, seed=79)
    rays = w.primary[sel]
    g = run(gsc, rays)
    osc = O.Scene(cp1, w.types, w.leaf_depth, local_frames=frames)
    rep = gate(g, osc.intersect(rays), rays, osc, w.diameter, w.leaf_depth, label="1M-refit-frame5")
    assert_gate(rep)
    assert rep["oracle_hits"] > 1000
