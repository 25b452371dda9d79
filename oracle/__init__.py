"""FP64 CPU oracle for ray / Bezier-Gregory patch intersection (TEST INFRASTRUCTURE).

A plain, slow, independent implementation of what the HIP path computes, used
only by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py``.  It shares no code with the library; it reads the same seeded
inputs (patch control points, type tags, leaf depth, rays) and nothing else.
See ``oracle.cpp`` for the conventions and the passages of the paper each
function follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
NO_HIT = 0xFFFFFFFF
COUNTER_NAMES = ("node", "cand", "split", "backtrack", "greg", "leaf", "crop", "cand_greg")


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB names another build of oracle.cpp (the planted-mistake builds of
        # tests/test_oracle_mutants.py); by default the one oracle/build.py makes
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        d, u32, i32, vp = C.c_double, C.c_uint32, C.c_int, C.c_void_p
        P = C.POINTER
        L.orc_patch_eval.argtypes = [P(d), i32, d, d, P(d), P(d), P(d)]
        L.orc_bezier_eval.argtypes = [P(d), d, d, P(d)]
        L.orc_split.argtypes = [P(d), i32, P(d), P(d)]
        L.orc_crop.argtypes = [P(d), d, d, d, d, P(d)]
        L.orc_wbar.argtypes = [i32, d, d]
        L.orc_wbar.restype = d
        L.orc_inner_extremes.argtypes = [P(d), d, d, d, d, P(d), P(d)]
        L.orc_calc_points_and_d.argtypes = [P(d), i32, d, d, d, d, P(d), P(d)]
        L.orc_scene_create.argtypes = [P(C.c_float), P(C.c_uint8), u32, i32, i32, i32]
        L.orc_patch_frame.argtypes = [vp, u32, P(d)]
        L.orc_scene_create.restype = vp
        L.orc_scene_destroy.argtypes = [vp]
        L.orc_scene_nodes.argtypes = [vp]
        L.orc_scene_nodes.restype = u32
        L.orc_intersect.argtypes = [vp, P(C.c_float), u32, i32, P(d), P(u32), P(d), P(d), P(u32)]
        L.orc_intersect_f64.argtypes = [vp, P(d), u32, i32, P(d), P(u32), P(d), P(d)]
        L.orc_intersect_hinted.argtypes = [vp, P(C.c_float), u32, i32, i32, P(u32), P(d), P(d), P(d), P(u32),
                                           P(d), P(d), P(u32)]
        L.orc_trace_patch.argtypes = [vp, u32, P(C.c_float), d, P(u32), i32, P(d)]
        L.orc_trace_patch.restype = i32
        L.orc_trace_patch_alg3.argtypes = [vp, u32, P(C.c_float), d, P(u32), i32, P(d)]
        L.orc_trace_patch_alg3.restype = i32
        L.orc_bruteforce.argtypes = [vp, P(C.c_float), u32, i32, i32, P(d), P(u32), P(d), P(d)]
        L.orc_bounce.argtypes = [vp, P(C.c_float), P(C.c_float), P(C.c_float), u32, P(d)]
        L.orc_leaf_entry.argtypes = [vp, u32, P(C.c_float), u32, u32]
        L.orc_leaf_entry.restype = d
        L.orc_domain_box.argtypes = [vp, u32, u32, u32, u32, u32, P(d)]
        L.orc_leaf_box_alg3.argtypes = [vp, u32, u32, u32, P(d)]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ------------------------------------------------------------------ patch math
def patch_eval(cp20, gregory: bool, u: float, v: float):
    """(f, f_u, f_v) of a Bezier or Gregory patch at (u, v)."""
    cp = _f64(cp20, (20, 3))
    f, fu, fv = (np.zeros(3) for _ in range(3))
    lib().orc_patch_eval(_p(cp, C.c_double), int(gregory), u, v, _p(f, C.c_double),
                         _p(fu, C.c_double), _p(fv, C.c_double))
    return f, fu, fv


def bezier_eval(grid16, u: float, v: float):
    """(f, f_u, f_v, f_uv) of a 16-point Bezier grid at (u, v)."""
    g = _f64(grid16, (16, 3))
    out = np.zeros((4, 3))
    lib().orc_bezier_eval(_p(g, C.c_double), u, v, _p(out, C.c_double))
    return out


def split(grid16, axis: int):
    g = _f64(grid16, (16, 3))
    L, R = np.zeros((16, 3)), np.zeros((16, 3))
    lib().orc_split(_p(g, C.c_double), axis, _p(L, C.c_double), _p(R, C.c_double))
    return L, R


def crop(grid16, u0, u1, v0, v1):
    g = _f64(grid16, (16, 3))
    q = np.zeros((16, 3))
    lib().orc_crop(_p(g, C.c_double), u0, u1, v0, v1, _p(q, C.c_double))
    return q


def wbar(k: int, t0: float, t1: float) -> float:
    return lib().orc_wbar(k, t0, t1)


def inner_extremes(cp20, u0, u1, v0, v1):
    cp = _f64(cp20, (20, 3))
    A, B = np.zeros((4, 3)), np.zeros((4, 3))
    lib().orc_inner_extremes(_p(cp, C.c_double), u0, u1, v0, v1, _p(A, C.c_double), _p(B, C.c_double))
    return A, B


def calc_points_and_d(cp20, gregory: bool, u0, u1, v0, v1):
    cp = _f64(cp20, (20, 3))
    q, d = np.zeros((16, 3)), np.zeros(3)
    lib().orc_calc_points_and_d(_p(cp, C.c_double), int(gregory), u0, u1, v0, v1,
                                _p(q, C.c_double), _p(d, C.c_double))
    return q, d


# --------------------------------------------------------------------- scenes
class Scene:
    """Oracle scene: patches (n, 20, 3) float32, tags (n,) uint8, per-axis leaf depth L."""

    def __init__(self, cp, types, leaf_depth: int, use_bvh: bool = True, local_frames: bool = False):
        self.cp = np.ascontiguousarray(cp, dtype=np.float32).reshape(-1, 20, 3)
        self.types = np.ascontiguousarray(types, dtype=np.uint8)
        assert self.types.shape[0] == self.cp.shape[0]
        self.n = self.cp.shape[0]
        self.leaf_depth = int(leaf_depth)
        self.local_frames = bool(local_frames)
        self._h = lib().orc_scene_create(_p(self.cp, C.c_float), _p(self.types, C.c_uint8), self.n,
                                         self.leaf_depth, int(use_bvh), int(self.local_frames))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_scene_destroy(h)
            self._h = None

    def patch_frame(self, k: int) -> np.ndarray:
        """Rows (3 x 3) of patch k's local frame (the identity unless local_frames)."""
        r = np.zeros(9)
        lib().orc_patch_frame(self._h, int(k), _p(r, C.c_double))
        return r.reshape(3, 3)

    @property
    def n_nodes(self) -> int:
        return int(lib().orc_scene_nodes(self._h))

    def intersect(self, rays, nthreads: int = 0, counters: bool = False):
        """Closest hits: dict(t, id, u, v[, counters (n, 8), see COUNTER_NAMES])."""
        r = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
        n = r.shape[0]
        t, u, v = np.zeros(n), np.zeros(n), np.zeros(n)
        ids = np.zeros(n, dtype=np.uint32)
        cnt = np.zeros((n, 8), dtype=np.uint32) if counters else None
        lib().orc_intersect(self._h, _p(r, C.c_float), n, nthreads, _p(t, C.c_double),
                            _p(ids, C.c_uint32), _p(u, C.c_double), _p(v, C.c_double),
                            _p(cnt, C.c_uint32) if counters else None)
        out = dict(t=t, id=ids, u=u, v=v)
        if counters:
            out["counters"] = cnt
        return out

    def intersect_f64(self, rays, nthreads: int = 0):
        """Closest hits of rays given in double precision (n, 8): dict(t, id, u, v)."""
        r = np.ascontiguousarray(rays, dtype=np.float64).reshape(-1, 8)
        n = r.shape[0]
        t, u, v = np.zeros(n), np.zeros(n), np.zeros(n)
        ids = np.zeros(n, dtype=np.uint32)
        lib().orc_intersect_f64(self._h, _p(r, C.c_double), n, nthreads, _p(t, C.c_double), _p(ids, C.c_uint32),
                                _p(u, C.c_double), _p(v, C.c_double))
        return dict(t=t, id=ids, u=u, v=v)

    def intersect_hinted(self, rays, hint=None, nthreads: int = 0, lookahead: bool = False):
        """Closest hits and counters in another child order, to bound what a learned order
        can save.  Where both halves of a split are hit (not the leaf pair): with a hint
        (a dict(id, u, v) of closest hits, e.g. intersect's own) the half holding the
        hinted leaf goes first on the hinted patch (hindsight); with lookahead, on every
        patch, the half whose first visit costs fewer split steps over the node's subtree."""
        r = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
        n = r.shape[0]
        if hint is None:
            hint = dict(id=np.full(n, NO_HIT, np.uint32), u=np.zeros(n), v=np.zeros(n))
        hid = np.ascontiguousarray(hint["id"], dtype=np.uint32)
        hu, hv = _f64(hint["u"]), _f64(hint["v"])
        t, u, v = np.zeros(n), np.zeros(n), np.zeros(n)
        ids = np.zeros(n, dtype=np.uint32)
        cnt = np.zeros((n, 8), dtype=np.uint32)
        lib().orc_intersect_hinted(self._h, _p(r, C.c_float), n, nthreads, int(lookahead), _p(hid, C.c_uint32),
                                   _p(hu, C.c_double), _p(hv, C.c_double), _p(t, C.c_double),
                                   _p(ids, C.c_uint32), _p(u, C.c_double), _p(v, C.c_double),
                                   _p(cnt, C.c_uint32))
        return dict(t=t, id=ids, u=u, v=v, counters=cnt)

    def intersect_retest(self, rays, nthreads: int = 0):
        """Closest hits and counters when a pending sibling is skipped on resumption if its
        box's entry (tested when its parent was split) lies beyond the best distance found
        since; Alg. 3 resumes it without re-testing.  dict(t, id, u, v, counters)."""
        return self._mode(rays, 3, nthreads)

    def _mode(self, rays, mode, nthreads):
        r = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
        n = r.shape[0]
        zero = np.zeros(n)
        hid = np.full(n, NO_HIT, np.uint32)
        t, u, v = np.zeros(n), np.zeros(n), np.zeros(n)
        ids = np.zeros(n, dtype=np.uint32)
        cnt = np.zeros((n, 8), dtype=np.uint32)
        lib().orc_intersect_hinted(self._h, _p(r, C.c_float), n, nthreads, mode, _p(hid, C.c_uint32),
                                   _p(zero, C.c_double), _p(zero, C.c_double), _p(t, C.c_double),
                                   _p(ids, C.c_uint32), _p(u, C.c_double), _p(v, C.c_double), _p(cnt, C.c_uint32))
        return dict(t=t, id=ids, u=u, v=v, counters=cnt)

    def intersect_single_box(self, rays, nthreads: int = 0):
        """Closest hits and counters when every subdivision node tests only its own box
        (Sec. 3.3's alternative to the two-box test): dict(t, id, u, v, counters)."""
        return self._mode(rays, 2, nthreads)

    def _trace(self, fn, patch, ray8, cap, max_seq):
        r = np.ascontiguousarray(ray8, dtype=np.float32).reshape(8)
        seq = np.zeros((max_seq, 4), dtype=np.uint32)
        hit = np.zeros(4)
        n = fn(self._h, int(patch), _p(r, C.c_float), float(cap), _p(seq, C.c_uint32), max_seq,
               _p(hit, C.c_double))
        return seq[:min(n, max_seq)], hit

    def trace_patch(self, patch, ray8, cap=np.inf, max_seq=4096):
        """Split sequence (pos_u, pos_v, size_u, size_v) and hit (t, id, u, v) of one ray-patch pair."""
        return self._trace(lib().orc_trace_patch, patch, ray8, cap, max_seq)

    def trace_patch_alg3(self, patch, ray8, cap=np.inf, max_seq=4096):
        """The same, from the bit-trail loop of Alg. 3 (control-logic equivalence test)."""
        return self._trace(lib().orc_trace_patch_alg3, patch, ray8, cap, max_seq)

    def bruteforce(self, rays, res: int = 512, nthreads: int = 0):
        r = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
        n = r.shape[0]
        t, u, v = np.zeros(n), np.zeros(n), np.zeros(n)
        ids = np.zeros(n, dtype=np.uint32)
        lib().orc_bruteforce(self._h, _p(r, C.c_float), n, res, nthreads, _p(t, C.c_double),
                             _p(ids, C.c_uint32), _p(u, C.c_double), _p(v, C.c_double))
        return dict(t=t, id=ids, u=u, v=v)

    def bounce(self, rays, hits, uniforms):
        """Secondary rays (n, 8) float64 from hits (n, 4) float32 records {t, id bits, u, v}."""
        r = np.ascontiguousarray(rays, dtype=np.float32).reshape(-1, 8)
        h = np.ascontiguousarray(hits, dtype=np.float32).reshape(-1, 4)
        w = np.ascontiguousarray(uniforms, dtype=np.float32).reshape(-1, 2)
        out = np.zeros((r.shape[0], 8))
        lib().orc_bounce(self._h, _p(r, C.c_float), _p(h, C.c_float), _p(w, C.c_float), r.shape[0],
                         _p(out, C.c_double))
        return out

    def leaf_entry(self, patch, ray8, u, v):
        """Entry distance into the Alg. 3 box of the leaf containing (u, v) (inf if missed)."""
        r = np.ascontiguousarray(ray8, dtype=np.float32).reshape(8)
        _, pu, pv = self._leaf_corner(u, v)
        return lib().orc_leaf_entry(self._h, int(patch), _p(r, C.c_float), pu, pv)

    def domain_box(self, patch, u0, v0, size_u, size_v):
        """[lo, hi] of the lower grid + displacement on an integer domain (units 2^-23)."""
        box = np.zeros(6)
        lib().orc_domain_box(self._h, int(patch), int(u0), int(v0), int(size_u), int(size_v),
                             _p(box, C.c_double))
        return box[:3], box[3:]

    def _leaf_corner(self, u, v):
        leaf = (1 << 23) >> self.leaf_depth
        pu = min(int(np.floor(u * 2.0 ** 23)) & ~(leaf - 1), (1 << 23) - leaf)
        pv = min(int(np.floor(v * 2.0 ** 23)) & ~(leaf - 1), (1 << 23) - leaf)
        return leaf, pu, pv

    def leaf_box(self, patch, u, v):
        """[lo, hi] of the leaf containing (u, v) bounded on its own domain (calcPointsAndD)."""
        leaf, pu, pv = self._leaf_corner(u, v)
        return self.domain_box(patch, pu, pv, leaf, leaf)

    def leaf_box_alg3(self, patch, u, v):
        """[lo, hi] of the leaf containing (u, v) as Alg. 3 tests it: its half of the
        parent's grid, grown by the parent's displacement."""
        _, pu, pv = self._leaf_corner(u, v)
        box = np.zeros(6)
        lib().orc_leaf_box_alg3(self._h, int(patch), pu, pv, _p(box, C.c_double))
        return box[:3], box[3:]
