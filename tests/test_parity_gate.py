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
        assert not rep["ok"] and rep["excused"]["hard"] >= 0.9 * len(hit), (kind, rep["excused"])


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
