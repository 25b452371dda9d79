"""Ray compaction (ccs_compact_rays) for the bounce levels of a path tracer
(Sec. 4): the kept rays, their order and indices against the rule written out
here in numpy, the rule against the intersection kernel's own decision (its
node counter is zero exactly for the rays it does not trace), and a compacted
bounce level traced to the same hits as the full one."""
import numpy as np
import pytest

import oracle as O
from oracle.parity import assert_gate, gate, ids_of

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


def traced_rule(r: np.ndarray) -> np.ndarray:
    """Rays an intersection entry point traces: finite origin and direction, tmin
    and tmax not NaN, a nonzero direction and tmin <= tmax (inputs without
    denormals, where flushing them changes nothing)."""
    o, d, tmin, tmax = r[:, 0:3], r[:, 4:7], r[:, 3], r[:, 7]
    with np.errstate(invalid="ignore"):
        return (np.isfinite(o).all(1) & np.isfinite(d).all(1) & ~np.isnan(tmin) & ~np.isnan(tmax)
                & (d != 0).any(1) & (tmin <= tmax))


def mixed_rays(n: int, seed: int, denormals: bool = False) -> np.ndarray:
    """Rays toward the unit torus scene's extent, a third of them spoiled in one of
    the ways the rule rejects (and some edge cases it accepts)."""
    rng = np.random.default_rng(seed)
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = rng.uniform(-4, 4, (n, 3))
    r[:, 4:7] = rng.normal(size=(n, 3))
    r[:, 3] = 0.0
    r[:, 7] = np.inf
    kind = rng.integers(0, 16, n)
    col = rng.integers(0, 3, n)
    nan, inf = np.float32(np.nan), np.float32(np.inf)
    r[kind == 1, 0] = nan                                    # NaN origin
    r[kind == 2, 4 + col[kind == 2]] = inf                   # infinite direction component
    r[kind == 3, 1] = -inf                                   # infinite origin
    r[kind == 4, 3] = nan                                    # NaN tmin
    r[kind == 5, 7] = nan                                    # NaN tmax
    r[np.ix_(kind == 6, [4, 5, 6])] = 0.0                    # zero direction
    r[np.ix_(kind == 7, [4, 5, 6])] = -0.0                   # negative zero direction
    k8 = kind == 8                                            # tmin > tmax (an inactive bounce)
    r[k8, 3], r[k8, 7] = 1.0, -1.0
    k9 = kind == 9                                            # tmin == tmax: traced
    r[k9, 3] = r[k9, 7] = 0.5
    r[kind == 10, 3] = -inf                                  # tmin = -inf: traced
    r[np.ix_(kind == 11, [4, 5])] = 0.0                      # one nonzero direction component: traced
    r[kind == 12, 4 + col[kind == 12]] = np.float32(np.nan)  # NaN direction component
    if denormals:
        k13 = kind == 13                                     # only denormal direction components
        r[np.ix_(k13, [4, 5, 6])] = np.float32(1e-40)
        k14 = kind == 14                                     # denormal tmin above a zero tmax
        r[k14, 3], r[k14, 7] = np.float32(1e-40), 0.0
    return r


def _compact(ccs, rays):
    out, index, work = ccs.compact_rays(torch.from_numpy(rays).cuda())
    torch.cuda.synchronize()
    m = int(work[0].item())
    return out[:m].cpu().numpy(), index[:m].cpu().numpy().view(np.uint32), m


@pytest.mark.parametrize("n", [1, 255, 256, 257, 5000, (1 << 22) + 17])
def test_kept_rays_order_and_indices(ccs, n):
    rays = mixed_rays(n, seed=n)
    keep = traced_rule(rays)
    out, idx, m = _compact(ccs, rays)
    _say(f"n = {n}: {m} of {n} rays kept (rule: {int(keep.sum())})")
    assert m == int(keep.sum())
    assert np.array_equal(idx, np.flatnonzero(keep).astype(np.uint32))
    assert np.array_equal(out.view(np.uint32), rays[keep].view(np.uint32))


def test_empty_input_sets_the_count(ccs):
    work = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    ccs.compact_rays(torch.empty((0, 8), dtype=torch.float32, device="cuda"), work=work)
    torch.cuda.synchronize()
    assert int(work[0].item()) == 0


def test_rule_is_the_intersection_kernels(ccs, c1):
    """Rays the compaction drops are exactly those the intersection kernel does not
    trace (no node visited), denormal directions and limits included."""
    rays = mixed_rays(20000, seed=3, denormals=True)
    scene = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth,
                      local_frames=True)
    _, cnt = scene.intersect_counted(torch.from_numpy(rays).cuda())
    torch.cuda.synchronize()
    traced = cnt[:, 0].cpu().numpy() > 0
    _, idx, m = _compact(ccs, rays)
    kept = np.zeros(len(rays), bool)
    kept[idx] = True
    _say(f"kept {m} of {len(rays)}; traced by the intersection kernel {int(traced.sum())}")
    assert np.array_equal(kept, traced)
    assert 0 < m < len(rays)


@pytest.mark.parametrize("local", [False, True], ids=["world", "local"])
def test_compacted_bounce_level_traces_to_the_full_levels_hits(ccs, c1, local):
    """Primary hits -> one cosine bounce per ray -> the bounce level traced in full
    and compacted: the same hits bitwise for the kept rays, misses for the others,
    and the compacted level passes the gate against the oracle."""
    scene = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth,
                      local_frames=local)
    prim = torch.from_numpy(c1.primary).cuda()
    hp = scene.intersect(prim)
    u = torch.from_numpy(np.random.default_rng(17).uniform(0, 1, (len(c1.primary), 2)).astype(np.float32)).cuda()
    b = scene.bounce(prim, hp, u)
    full = scene.intersect(b)
    out, index, work = ccs.compact_rays(b)
    torch.cuda.synchronize()
    m = int(work[0].item())
    part = scene.intersect(out[:m])
    torch.cuda.synchronize()
    idx = index[:m].cpu().numpy()
    fh, ph = full.cpu().numpy(), part.cpu().numpy()
    _say(f"bounce level: {m} of {len(c1.primary)} rays active")
    assert 1000 < m < len(c1.primary)
    assert np.array_equal(ph.view(np.uint32), fh[idx].view(np.uint32))
    rest = np.ones(len(fh), bool)
    rest[idx] = False
    assert (ids_of(fh[rest]) == O.NO_HIT).all()
    rays = out[:m].cpu().numpy()
    osc = O.Scene(c1.cp, c1.types, c1.leaf_depth, local_frames=local)
    assert_gate(gate(ph, osc.intersect(rays), rays, osc, c1.diameter, c1.leaf_depth, label="compacted-bounce"))
