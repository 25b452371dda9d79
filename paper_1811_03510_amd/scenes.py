"""Seeded synthetic workloads for ray / Catmull-Clark patch intersection.

This module only *describes inputs*: control cages, their conversion to bicubic
patches in OpenSubdiv's patch form (16-point Bezier, 20-point Gregory), camera
rays and secondary-ray sets.  It performs no step of the intersection method
(no subdivision, no patch bounds, no ray/box test); the HIP library and the FP64
oracle both consume what it returns and nothing else is shared between them.

Patch layout (20 points x 3 floats, fp32), slot order:
  * slots 0..15: the 4x4 grid, slot(i, j) = 4*j + i, i along u and j along v;
  * inner slots 5, 6, 9, 10 hold P^u of the inner points (1,1), (2,1), (1,2), (2,2);
  * slots 16..19 hold P^v of the same four inner points.  A Bezier patch stores a
    copy of its inner points there, so that reading it as a Gregory patch with
    coincident pairs gives the same surface (Sec. 2.2 of the paper).
Gregory blend convention: the inner point (i, j) is
  (du * P^u + dv * P^v) / (du + dv), du = u (i=1) or 1-u (i=2), dv = v (j=1) or 1-v (j=2),
which is the weighting used by the bound computation of Alg. 2.

Random streams: SplitMix64 in counter form (draw k of a stream with seed s is
mix(s + (k+1) * 0x9E3779B97F4A7C15)), uniforms from the top 53 bits, normals by
Box-Muller.  Everything is computed in float64 and rounded to float32 once.
"""
from __future__ import annotations

import dataclasses
import math

import os

import numpy as np

SEED = 1811035
STREAM_SCENE = SEED + 1
STREAM_GREGORY_CHOICE = SEED + 2
STREAM_GREGORY_JITTER = SEED + 3
STREAM_PLACEMENT = SEED + 4
STREAM_ANIMATION = SEED + 5
STREAM_BOUNCE = SEED + 6
STREAM_BATCH = SEED + 7
STREAM_MLP = SEED + 8

INNER_SLOTS = (5, 6, 9, 10)
PV_SLOTS = (16, 17, 18, 19)
BEZIER = 0
GREGORY = 1

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


# --------------------------------------------------------------------------- RNG
def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Draws start .. start+n-1 of the SplitMix64 stream seeded with ``seed``."""
    k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def substream(seed: int, k: int) -> int:
    """Seed of the k-th independent sub-stream of ``seed``."""
    return int(splitmix64(seed, 1, k)[0])


def uniform(seed: int, n: int, start: int = 0) -> np.ndarray:
    """n uniforms in [0, 1) (float64)."""
    return (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, n: int) -> np.ndarray:
    """n standard normals by Box-Muller (one normal per uniform pair)."""
    u = uniform(seed, 2 * n).reshape(n, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))  # 1-u in (0, 1]
    return r * np.cos(2.0 * np.pi * u[:, 1])


# ------------------------------------------------------------------ cages, patches
def torus_frame(n_theta: int, n_phi: int):
    """Unit ring points (cos t, sin t, 0) and tube normals on an n_theta x n_phi grid."""
    th = 2.0 * np.pi * np.arange(n_theta) / n_theta
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    T, P = np.meshgrid(th, ph, indexing="ij")
    nrm = np.stack((np.cos(P) * np.cos(T), np.cos(P) * np.sin(T), np.sin(P)), axis=-1)
    ring = np.stack((np.cos(T), np.sin(T), np.zeros_like(T)), axis=-1)
    return ring, nrm


def torus_cage(n_theta: int, n_phi: int, R: float, r: float):
    """Vertices (n_theta, n_phi, 3) of a torus control cage and their tube normals."""
    ring, nrm = torus_frame(n_theta, n_phi)
    return R * ring + r * nrm, nrm


def _end(a, b, c):
    # uniform cubic B-spline -> Bezier end point; the same operand order on both
    # sides of a shared edge keeps shared boundary points bit-identical
    return (a + 4.0 * b + c) / 6.0


def _third(b, c):
    return (2.0 * b + c) / 3.0


def bspline_to_bezier(cage: np.ndarray) -> np.ndarray:
    """Periodic bicubic B-spline cage (..., nu, nv, 3) -> Bezier grids (..., nu*nv, 16, 3).

    Quad (i, j) spans cage vertices i..i+1 along u and j..j+1 along v; its 4x4
    B-spline neighbourhood is rows i-1..i+2, columns j-1..j+2 (indices mod the
    cage size).  All cage vertices have valence 4, so each grid is exactly the
    Catmull-Clark limit patch of its quad.  Conversion is applied along u, then v.
    """
    nu, nv = cage.shape[-3], cage.shape[-2]
    iu = np.arange(nu)
    cm1, c0 = cage[..., (iu - 1) % nu, :, :], cage
    c1, c2 = cage[..., (iu + 1) % nu, :, :], cage[..., (iu + 2) % nu, :, :]
    U = np.stack((_end(cm1, c0, c1), _third(c0, c1), _third(c1, c0), _end(c0, c1, c2)),
                 axis=-2)  # (..., nu, nv, 4[a], 3)
    iv = np.arange(nv)
    um1, u0 = U[..., :, (iv - 1) % nv, :, :], U
    u1, u2 = U[..., :, (iv + 1) % nv, :, :], U[..., :, (iv + 2) % nv, :, :]
    P = np.stack((_end(um1, u0, u1), _third(u0, u1), _third(u1, u0), _end(u0, u1, u2)),
                 axis=-2)  # (..., nu, nv, 4[a], 4[b], 3)
    P = np.swapaxes(P, -3, -2)  # [..., b, a, 3] -> slot 4*b + a
    return P.reshape(P.shape[:-5] + (nu * nv, 16, 3))


def patch_cell(grid16: np.ndarray) -> np.ndarray:
    """Mean length of the four corner-to-corner edges p00p30, p03p33, p00p03, p30p33."""
    p00, p30, p03, p33 = grid16[:, 0], grid16[:, 3], grid16[:, 12], grid16[:, 15]
    e = [p30 - p00, p33 - p03, p03 - p00, p33 - p30]
    return sum(np.linalg.norm(x, axis=-1) for x in e) / 4.0


def to_twenty(grid16: np.ndarray) -> np.ndarray:
    cp = np.empty((grid16.shape[0], 20, 3), dtype=np.float64)
    cp[:, :16] = grid16
    cp[:, 16:] = grid16[:, list(INNER_SLOTS)]
    return cp


def gregory_split(cp: np.ndarray, sel: np.ndarray, jitter_seed: int, rel: float = 0.05) -> None:
    """Turn the patches ``sel`` (sorted indices) into Gregory patches in place.

    Every inner point p becomes the pair P^u = p + e, P^v = p - e with
    e ~ N(0, (rel * cell)^2 I_3), cell = ``patch_cell`` of the patch.
    """
    if len(sel) == 0:
        return
    cell = patch_cell(cp[sel, :16])
    e = normal(jitter_seed, len(sel) * 12).reshape(len(sel), 4, 3) * (rel * cell)[:, None, None]
    base = cp[sel][:, list(INNER_SLOTS)]
    cp[np.ix_(sel, list(INNER_SLOTS))] = base + e
    cp[np.ix_(sel, list(PV_SLOTS))] = base - e


def choose(seed: int, n: int, k: int) -> np.ndarray:
    """A seeded subset of k out of n indices (sorted)."""
    perm = np.argsort(uniform(seed, n), kind="stable")
    return np.sort(perm[:k])


# --------------------------------------------------------------------------- rays
def pinhole_rays(eye, target, up, vfov_deg: float, width: int, height: int) -> np.ndarray:
    """(height*width, 8) float32 rays {o, tmin=0, d (unit), tmax=+inf}, row-major from the top."""
    eye, target, up = (np.asarray(x, dtype=np.float64) for x in (eye, target, up))
    f = target - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    upv = np.cross(r, f)
    th = math.tan(math.radians(vfov_deg) / 2.0)
    aspect = width / height
    x = (2.0 * (np.arange(width) + 0.5) / width - 1.0) * th * aspect
    y = (1.0 - 2.0 * (np.arange(height) + 0.5) / height) * th
    X, Y = np.meshgrid(x, y, indexing="xy")
    d = f[None, None, :] + X[..., None] * r + Y[..., None] * upv
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    d = d.reshape(-1, 3)
    out = np.zeros((d.shape[0], 8), dtype=np.float64)
    out[:, 0:3] = eye
    out[:, 4:7] = d
    out[:, 7] = np.inf
    return out.astype(np.float32)


def _bern(t):
    s = 1.0 - t
    return np.stack((s * s * s, 3 * t * s * s, 3 * t * t * s, t * t * t), axis=-1)


def _blended_grids(cp: np.ndarray, types: np.ndarray, idx: np.ndarray):
    g = cp[idx].astype(np.float64)
    return g, types[idx] == GREGORY


def _eval_gathered(g: np.ndarray, greg: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    grid = g[:, :16]
    if np.any(greg):
        grid = grid.copy()
        for k, (slot, pv) in enumerate(zip(INNER_SLOTS, PV_SLOTS)):
            i, j = (1 if k % 2 == 0 else 2), (1 if k < 2 else 2)
            du = u[greg] if i == 1 else 1.0 - u[greg]
            dv = v[greg] if j == 1 else 1.0 - v[greg]
            den = du + dv
            lam = np.where(den > 0, du / np.where(den > 0, den, 1.0), 0.5)
            grid[greg, slot] = lam[:, None] * g[greg, slot] + (1.0 - lam[:, None]) * g[greg, pv]
    bu, bv = _bern(u), _bern(v)
    w = (bv[:, :, None] * bu[:, None, :]).reshape(-1, 16)  # slot 4*j + i
    return np.einsum("ns,nsc->nc", w, grid)


def surface_points(cp: np.ndarray, types: np.ndarray, idx: np.ndarray, u: np.ndarray,
                   v: np.ndarray) -> np.ndarray:
    """Surface points of patches ``idx`` at (u, v), float64 (the patch definition of Sec. 2)."""
    g, greg = _blended_grids(cp, types, idx)
    return _eval_gathered(g, greg, np.asarray(u, np.float64), np.asarray(v, np.float64))


def onb(n: np.ndarray):
    """Orthonormal tangents (t, b) for unit normals n (Duff et al. 2017, branch-free)."""
    sign = np.where(n[:, 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t = np.stack((1.0 + sign * n[:, 0] ** 2 * a, sign * b, -sign * n[:, 0]), axis=-1)
    bb = np.stack((b, sign + n[:, 1] ** 2 * a, -n[:, 1]), axis=-1)
    return t, bb


def cosine_dirs(n: np.ndarray, u1: np.ndarray, u2: np.ndarray) -> np.ndarray:
    """Cosine-weighted directions about unit normals n (Malley's method, polar disk map)."""
    r = np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    z = np.sqrt(np.maximum(0.0, 1.0 - u1))
    t, b = onb(n)
    return (r * np.cos(phi))[:, None] * t + (r * np.sin(phi))[:, None] * b + z[:, None] * n


def surface_bounce_rays(cp: np.ndarray, types: np.ndarray, leaf_depth: int, eye, n: int,
                        seed: int = STREAM_BOUNCE, chunk: int = 1 << 16) -> np.ndarray:
    """Secondary-ray stand-in: one cosine-weighted bounce from n seeded surface points.

    A patch is drawn uniformly, (u, v) uniformly in [0.01, 0.99]^2; the normal is
    taken from central differences of the surface, turned towards the eye; the
    origin is pushed off the surface along it by 2^-L times the L1 size of the
    patch's bounding box (a leaf-sized offset).  Directions are cosine-weighted.
    """
    npatch = cp.shape[0]
    s = [substream(seed, k) for k in range(5)]
    idx_all = np.minimum((uniform(s[0], n) * npatch).astype(np.int64), npatch - 1)
    u_all = 0.01 + 0.98 * uniform(s[1], n)
    v_all = 0.01 + 0.98 * uniform(s[2], n)
    w1_all, w2_all = uniform(s[3], n), uniform(s[4], n)
    out = np.zeros((n, 8), dtype=np.float32)
    eye = np.asarray(eye, dtype=np.float64)
    h = 1e-6

    def one_chunk(b):  # chunks are independent: their uniforms are drawn above
        e = min(n, b + chunk)
        idx, u, v = idx_all[b:e], u_all[b:e], v_all[b:e]
        g, greg = _blended_grids(cp, types, idx)
        x = _eval_gathered(g, greg, u, v)
        fu = _eval_gathered(g, greg, u + h, v) - _eval_gathered(g, greg, u - h, v)
        fv = _eval_gathered(g, greg, u, v + h) - _eval_gathered(g, greg, u, v - h)
        nrm = np.cross(fu, fv)
        nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
        nrm *= np.where(np.sum(nrm * (eye[None, :] - x), axis=-1) < 0, -1.0, 1.0)[:, None]
        ext = (g.max(axis=1) - g.min(axis=1)).sum(axis=-1)
        o = x + (ext * 2.0 ** -leaf_depth)[:, None] * nrm
        d = cosine_dirs(nrm, w1_all[b:e], w2_all[b:e])
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        out[b:e, 0:3] = o
        out[b:e, 4:7] = d

    starts = range(0, n, chunk)
    if len(starts) > 4:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(one_chunk, starts))
    else:
        for b in starts:
            one_chunk(b)
    out[:, 7] = np.inf
    return out


# ------------------------------------------------------------------------ configs
@dataclasses.dataclass
class Workload:
    name: str
    cp: np.ndarray          # (n, 20, 3) float32
    types: np.ndarray       # (n,) uint8, 0 Bezier / 1 Gregory
    leaf_depth: int
    eye: tuple
    primary: np.ndarray     # (Np, 8) float32
    diffuse: np.ndarray     # (Nd, 8) float32

    @property
    def diameter(self) -> float:
        c = self.cp.reshape(-1, 3).astype(np.float64)
        return float(np.linalg.norm(c.max(axis=0) - c.min(axis=0)))


def torus_scene(n_theta=32, n_phi=16, R=1.0, r=0.35, noise=0.02, gregory_frac=0.10,
                seed_offset: int = 0):
    """One displaced torus: cage n_theta x n_phi, radial N(0, noise^2) per vertex."""
    cage, nrm = torus_cage(n_theta, n_phi, R, r)
    cage = cage + nrm * (noise * normal(STREAM_SCENE + seed_offset, n_theta * n_phi)
                         ).reshape(n_theta, n_phi, 1)
    cp = to_twenty(bspline_to_bezier(cage))
    n = cp.shape[0]
    types = np.zeros(n, dtype=np.uint8)
    sel = choose(STREAM_GREGORY_CHOICE + seed_offset, n, int(round(gregory_frac * n)))
    types[sel] = GREGORY
    gregory_split(cp, sel, STREAM_GREGORY_JITTER + seed_offset)
    return cp.astype(np.float32), types


def config1(width: int = 128, height: int = 128, with_diffuse: bool = True) -> Workload:
    """Displaced torus (R=1, r=0.35, 32x16 cage, 512 patches, 10% Gregory), L=12,
    128x128 pinhole primary rays, one secondary ray per pixel."""
    cp, types = torus_scene()
    eye = (0.0, -3.2, 2.0)
    prim = pinhole_rays(eye, (0, 0, 0), (0, 0, 1), 40.0, width, height)
    diff = (surface_bounce_rays(cp, types, 12, eye, width * height) if with_diffuse
            else np.zeros((0, 8), np.float32))
    return Workload("torus-512p-L12", cp, types, 12, eye, prim, diff)


def quat_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices (n, 3, 3) from unit quaternions (w, x, y, z)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack((
        np.stack((1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)), -1),
        np.stack((2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)), -1),
        np.stack((2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)), -1),
    ), axis=1)


def instanced_scene(n_objects: int = 2000, n_theta: int = 25, n_phi: int = 20,
                    gregory_frac: float = 0.25, extent: float = 40.0, noise: float = 0.02):
    """Randomly placed, scaled and rotated displaced tori and near-spherical 'apple'
    tori (R=0.55, r=0.5; closed and regular, so no extraordinary vertex appears).
    n_objects x n_theta*n_phi patches; a seeded ``gregory_frac`` become Gregory."""
    ps = [substream(STREAM_PLACEMENT, k) for k in range(6)]
    kind = uniform(ps[0], n_objects) < 0.5
    scale = np.exp(np.log(0.5) + (np.log(2.0) - np.log(0.5)) * uniform(ps[1], n_objects))
    q = normal(ps[2], 4 * n_objects).reshape(n_objects, 4)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    centre = (2.0 * uniform(ps[3], 3 * n_objects) - 1.0).reshape(n_objects, 3) * extent
    ring, nrm = torus_frame(n_theta, n_phi)
    R = np.where(kind, 1.0, 0.55)[:, None, None, None]
    r = np.where(kind, 0.35, 0.5)[:, None, None, None]
    cages = R * ring[None] + r * nrm[None]
    nz = normal(substream(STREAM_SCENE, 1), n_objects * n_theta * n_phi)
    cages = cages + nrm[None] * (noise * nz).reshape(n_objects, n_theta, n_phi, 1)
    rot = quat_rot(q)
    per = n_theta * n_phi
    cp = np.empty((n_objects * per, 20, 3), dtype=np.float64)
    for b in range(0, n_objects, 128):  # object chunks keep the temporaries cache-sized
        e = min(n_objects, b + 128)
        rb, cb = rot[b:e, None, None], cages[b:e]
        cg = np.stack([rb[..., a, 0] * cb[..., 0] + rb[..., a, 1] * cb[..., 1] + rb[..., a, 2] * cb[..., 2]
                       for a in range(3)], axis=-1)
        cg = cg * scale[b:e, None, None, None] + centre[b:e, None, None, :]
        cp[b * per:e * per] = to_twenty(bspline_to_bezier(cg).reshape(-1, 16, 3))
    n = cp.shape[0]
    types = np.zeros(n, dtype=np.uint8)
    sel = choose(STREAM_GREGORY_CHOICE, n, int(round(gregory_frac * n)))
    types[sel] = GREGORY
    gregory_split(cp, sel, STREAM_GREGORY_JITTER)
    return cp.astype(np.float32), types


def config2(width: int = 1920, height: int = 1080, n_objects: int = 2000,
            with_diffuse: bool = True) -> Workload:
    """1,000,000 patches (2000 objects x 500, 25% Gregory), L=10, 1920x1080 primary
    rays from (0,-110,30) towards the origin, one secondary ray per pixel."""
    cp, types = instanced_scene(n_objects)
    eye = (0.0, -110.0, 30.0)
    prim = pinhole_rays(eye, (0, 0, 0), (0, 0, 1), 50.0, width, height)
    diff = (surface_bounce_rays(cp, types, 10, eye, width * height) if with_diffuse
            else np.zeros((0, 8), np.float32))
    return Workload(f"instanced-{cp.shape[0]}p-L10", cp, types, 10, eye, prim, diff)


def sample_indices(n: int, k: int, seed: int = SEED) -> np.ndarray:
    """A seeded sorted sample of k distinct indices out of n (k <= n)."""
    k = min(k, n)
    return choose(seed, n, k)


# -------------------------------------------------------------- animation
def animate(cp: np.ndarray, frame: int, n_frames: int = 16, seed: int = STREAM_ANIMATION,
            amp_rel: float = 0.05, chunk: int = 1 << 18) -> np.ndarray:
    """Frame ``frame`` of a seeded animation: every control point x (all 20 slots) moves by
    A (sin(k1.x + 2 pi f/F + p1), sin(k2.x + 2 pi f/F + p2), sin(k3.x + 2 pi f/F + p3)),
    A = amp_rel * mean patch cell, k_i = 2 pi * seeded unit vectors, p_i seeded.  The
    displacement is a function of the rest position, so points shared by neighbouring
    patches move together and seams stay closed.  Patches are processed in chunks."""
    s = [substream(seed, k) for k in range(2)]
    k = normal(s[0], 9).reshape(3, 3)
    k = 2.0 * np.pi * k / np.linalg.norm(k, axis=1, keepdims=True)
    phase = 2.0 * np.pi * uniform(s[1], 3)
    n = cp.shape[0]
    cell = 0.0
    for b in range(0, n, chunk):
        cell += float(np.sum(patch_cell(cp[b:b + chunk, :16].astype(np.float64))))
    amp = amp_rel * cell / max(n, 1)
    out = np.empty(cp.shape, dtype=np.float32)

    def one(b):
        x = cp[b:b + chunk].astype(np.float64).reshape(-1, 3)
        # k . x as elementwise products and sums: a matrix product here would go to BLAS,
        # whose concurrent calls from the pool's threads have given corrupted results
        arg = np.stack([(x[:, 0] * k[i, 0] + x[:, 1] * k[i, 1]) + x[:, 2] * k[i, 2] for i in range(3)], axis=1)
        arg = arg + phase[None, :] + 2.0 * np.pi * frame / n_frames
        out[b:b + chunk] = (x + amp * np.sin(arg)).reshape(-1, 20, 3).astype(np.float32)

    from concurrent.futures import ThreadPoolExecutor  # elementwise: any chunk order gives the same bits
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(one, range(0, n, chunk)))
    return out


@dataclasses.dataclass
class Animation:
    name: str
    cp0: np.ndarray
    types: np.ndarray
    leaf_depth: int
    frames: list          # per frame: control points (n, 20, 3) float32
    rays: list            # per frame: (N_f, 8) float32, primary rays first
    n_primary: list       # per frame: number of primary rays at the front of rays[f]

    @property
    def diameter(self) -> float:
        c = self.cp0.reshape(-1, 3).astype(np.float64)
        return float(np.linalg.norm(c.max(axis=0) - c.min(axis=0)))


def config3(n_frames: int = 16, lo: int = 1 << 16, hi: int = 1 << 21, seed: int = STREAM_BATCH) -> Animation:
    """The 512-patch torus animated over n_frames frames; per frame a log-uniform
    number of rays in [lo, hi]: half primary from an orbiting camera (square image),
    half secondary rays from that frame's surface."""
    cp0, types = torus_scene()
    sizes = np.round(np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * uniform(seed, n_frames))).astype(np.int64)
    frames, rays, n_prim = [], [], []
    for f in range(n_frames):
        cp = animate(cp0, f, n_frames)
        ang = 2.0 * np.pi * f / n_frames
        eye = (3.2 * np.sin(ang), -3.2 * np.cos(ang), 2.0)
        side = max(8, int(round(np.sqrt(sizes[f] / 2))))
        prim = pinhole_rays(eye, (0, 0, 0), (0, 0, 1), 40.0, side, side)
        diff = surface_bounce_rays(cp, types, 12, eye, int(max(0, sizes[f] - side * side)),
                                   seed=substream(STREAM_BOUNCE, 100 + f))
        frames.append(cp)
        rays.append(np.concatenate([prim, diff]))
        n_prim.append(len(prim))
    return Animation(f"torus512-anim{n_frames}", cp0, types, 12, frames, rays, n_prim)


# --------------------------------------------------- child-ordering network
N_POLICY_PARAMS = 1732  # 16 -> 32 -> 32 -> 4: W1 (32x16), b1, W2 (32x32), b2, W3 (4x32), b3


def mlp_init(seed: int = STREAM_MLP) -> np.ndarray:
    """Seeded initial weights, fp32, flat in the order W1, b1, W2, b2, W3, b3:
    weights uniform in +-sqrt(6 / fan_in) (He et al. 2015), biases zero."""
    shapes = ((32, 16), (32,), (32, 32), (32,), (4, 32), (4,))
    out = []
    for k, shp in enumerate(shapes):
        if len(shp) == 1:
            out.append(np.zeros(shp))
        else:
            lim = np.sqrt(6.0 / shp[1])
            out.append((2.0 * uniform(substream(seed, k), int(np.prod(shp))) - 1.0) * lim)
    return np.concatenate([o.reshape(-1) for o in out]).astype(np.float32)


def policy_training_rays(n: int, seed: int = STREAM_MLP) -> np.ndarray:
    """Secondary rays on the 512-patch torus for recording ordering traces: the
    same recipe as its diffuse workload, from a stream of their own."""
    cp, types = torus_scene()
    return surface_bounce_rays(cp, types, 12, (0.0, -3.2, 2.0), n, seed=substream(seed, 100))


# ----------------------------------------------------------- combined run
@dataclasses.dataclass
class Combined:
    name: str
    cp: np.ndarray          # frame 0 (rest) control points, (n, 20, 3) float32
    types: np.ndarray
    leaf_depth: int
    eye: tuple
    primary: np.ndarray     # (W*H, 8) float32
    n_frames: int
    bounces: int

    def frame(self, f: int) -> np.ndarray:
        return animate(self.cp, f, self.n_frames)

    def bounce_uniforms(self, frame: int, bounce: int, n: int) -> np.ndarray:
        """Seeded uniforms for secondary-ray generation (ccs_bounce): 2 n values, pair i for ray i."""
        return uniform(substream(STREAM_BOUNCE, 1000 + 16 * frame + bounce), 2 * n).astype(np.float32)

    @property
    def diameter(self) -> float:
        c = self.cp.reshape(-1, 3)
        return float(np.linalg.norm(c.max(axis=0).astype(np.float64) - c.min(axis=0)))


def config5(n_objects: int = 16000, width: int = 3840, height: int = 2160, n_frames: int = 8,
            bounces: int = 3) -> Combined:
    """8,000,000 patches (16000 objects x 500, 30% Gregory) in [-80, 80]^3, L=10,
    3840x2160 primary rays from (0,-220,60), each followed by `bounces` diffuse
    bounces generated from the hits (ccs_bounce), over `n_frames` animation frames."""
    cp, types = instanced_scene(n_objects, gregory_frac=0.30, extent=80.0)
    eye = (0.0, -220.0, 60.0)
    prim = pinhole_rays(eye, (0, 0, 0), (0, 0, 1), 50.0, width, height)
    return Combined(f"instanced-{cp.shape[0]}p-L10-anim{n_frames}", cp, types, 10, eye, prim, n_frames, bounces)
