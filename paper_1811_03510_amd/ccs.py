"""Python binding of libccs (include/ccs.h): argument marshalling only.

Every step of the intersection runs in the HIP library; PyTorch provides device
memory and the current stream.  Importing works without a GPU (the library
loads), but building a scene needs a gfx950 device.  If the library has not been
built, ``lib()`` raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccs.so")

CCS_OK, CCS_ERR_INVALID_ARG, CCS_ERR_OOM, CCS_ERR_HIP, CCS_ERR_UNSUPPORTED = range(5)
CCS_BEZIER, CCS_GREGORY = 0, 1
CCS_HOST, CCS_DEVICE = 0, 1
CCS_FLAG_LOCAL_FRAMES = 1
CCS_FLAG_SINGLE_BOX = 2
NO_HIT = 0xFFFFFFFF
COUNTER_NAMES = ("node", "cand", "split", "backtrack", "greg", "leaf", "crop", "cand_greg")

EXPORTS = ("ccs_scene_create", "ccs_refit", "ccs_intersect", "ccs_intersect_counted", "ccs_bounce",
           "ccs_scene_info_get", "ccs_scene_destroy", "ccs_last_error", "ccs_scene_set_launch",
           "ccs_scene_get_launch", "ccs_scene_set_frames", "ccs_refit_frame", "ccs_intersect_batched",
           "ccs_scene_set_policy", "ccs_policy_record", "ccs_policy_infer", "ccs_policy_grad", "ccs_policy_train",
           "ccs_bounce_frame", "ccs_device_bytes_in_use", "ccs_debug_grids", "ccs_policy_grad_noalloc",
           "ccs_intersect_batched_counted", "ccs_compact_rays")
MAX_BATCHES = 32
MAX_RAYS = (1 << 31) - 1  # per call
POLICY_PARAMS = 1732
NO_LABEL = 255
DEBUG_GRID_FLOATS = 160
GRAD_NOALLOC_MAX_ROWS = 16384


class CcsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ccs status {status}: {message}")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [("control_points", C.c_void_p), ("patch_types", C.c_void_p), ("n_patches", C.c_uint32),
                ("location", C.c_int32), ("leaf_depth", C.c_uint32), ("flags", C.c_uint32),
                ("stream", C.c_void_p)]


class SceneInfo(C.Structure):
    _fields_ = [("n_patches", C.c_uint32), ("n_nodes", C.c_uint32), ("leaf_depth", C.c_uint32),
                ("bvh_depth", C.c_uint32), ("device_bytes", C.c_uint64), ("lo", C.c_float * 3),
                ("hi", C.c_float * 3), ("build_seconds", C.c_double), ("n_frames", C.c_uint32)]


class Batch(C.Structure):
    _fields_ = [("frame", C.c_uint32), ("n", C.c_uint32), ("rays", C.c_void_p), ("hits", C.c_void_p)]


class LaunchParams(C.Structure):
    _fields_ = [("waves_per_cu", C.c_uint32), ("fetch_min", C.c_uint32), ("traverse_min", C.c_uint32),
                ("grid_min", C.c_uint32), ("traverse_steps", C.c_uint32), ("decide_min", C.c_uint32)]


class TrainParams(C.Structure):
    _fields_ = [("steps", C.c_uint32), ("batch", C.c_uint32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64), ("bf16", C.c_uint32),
                ("reserved", C.c_uint32)]


class AdamState(C.Structure):
    _fields_ = [("m", C.c_void_p), ("v", C.c_void_p), ("t", C.c_uint64)]


_lib = None


def lib():
    """The loaded libccs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python paper_1811_03510_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, u32, i32 = C.c_void_p, C.c_uint32, C.c_int32
        L.ccs_scene_create.argtypes = [C.POINTER(SceneDesc), C.POINTER(vp)]
        L.ccs_refit.argtypes = [vp, vp, i32, vp]
        L.ccs_intersect.argtypes = [vp, vp, u32, vp, vp]
        L.ccs_intersect_counted.argtypes = [vp, vp, u32, vp, vp, vp]
        L.ccs_bounce.argtypes = [vp, vp, vp, vp, u32, vp, vp]
        L.ccs_bounce_frame.argtypes = [vp, u32, vp, vp, vp, u32, vp, vp]
        L.ccs_scene_info_get.argtypes = [vp, C.POINTER(SceneInfo)]
        L.ccs_scene_destroy.argtypes = [vp]
        L.ccs_scene_destroy.restype = None
        L.ccs_last_error.restype = C.c_char_p
        L.ccs_scene_set_launch.argtypes = [vp, C.POINTER(LaunchParams)]
        L.ccs_scene_set_frames.argtypes = [vp, u32]
        L.ccs_refit_frame.argtypes = [vp, u32, vp, i32, vp]
        L.ccs_intersect_batched.argtypes = [vp, C.POINTER(Batch), u32, vp]
        L.ccs_intersect_batched_counted.argtypes = [vp, C.POINTER(Batch), u32, vp, vp]
        L.ccs_scene_get_launch.argtypes = [vp, C.POINTER(LaunchParams)]
        L.ccs_scene_set_policy.argtypes = [vp, vp, vp]
        L.ccs_policy_record.argtypes = [vp, vp, vp, u32, vp, vp, vp]
        L.ccs_policy_infer.argtypes = [vp, vp, u32, vp, vp]
        L.ccs_policy_grad.argtypes = [vp, vp, vp, u32, u32, vp, vp, vp]
        L.ccs_policy_grad_noalloc.argtypes = [vp, vp, vp, u32, u32, vp, vp, vp]
        L.ccs_policy_train.argtypes = [vp, vp, vp, u32, C.POINTER(TrainParams), C.POINTER(AdamState), vp, vp]
        L.ccs_debug_grids.argtypes = [vp, u32, vp, vp, vp, u32, vp, vp]
        L.ccs_compact_rays.argtypes = [vp, u32, vp, vp, vp, vp]
        L.ccs_device_bytes_in_use.argtypes = []
        for name in EXPORTS:
            if name not in ("ccs_scene_destroy", "ccs_last_error", "ccs_device_bytes_in_use"):
                getattr(L, name).restype = C.c_int
        L.ccs_device_bytes_in_use.restype = C.c_uint64
        _lib = L
    return _lib


def _check(status: int):
    if status != CCS_OK:
        raise CcsError(status, lib().ccs_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Scene:
    """A patch scene on the current GPU.

    control_points: (n, 20, 3) float32 (torch tensor on cuda or cpu, or numpy);
    patch_types: (n,) uint8 (0 Bezier, 1 Gregory); leaf_depth: L in [1, 20] (above 16: closest-first order only).
    local_frames: subdivide in patch-local frames; single_box: the one-box-per-step
    ablation of Sec. 3.3 (measurement only).
    """

    def __init__(self, control_points, patch_types, leaf_depth: int, stream=None, local_frames: bool = False,
                 single_box: bool = False):
        import torch
        cp = torch.as_tensor(control_points)
        ty = torch.as_tensor(patch_types)
        if cp.dtype != torch.float32 or ty.dtype != torch.uint8:
            raise TypeError("control_points must be float32 and patch_types uint8")
        cp = cp.reshape(-1, 20, 3).contiguous()
        ty = ty.reshape(-1).contiguous()
        if cp.shape[0] != ty.shape[0]:
            raise ValueError("control_points and patch_types disagree on the patch count")
        on_dev = cp.is_cuda
        if ty.is_cuda != on_dev:
            ty = ty.to(cp.device)
        self.n = int(cp.shape[0])
        self.leaf_depth = int(leaf_depth)
        self.local_frames = bool(local_frames)
        desc = SceneDesc(cp.data_ptr() if self.n else None, ty.data_ptr() if self.n else None, self.n,
                         CCS_DEVICE if on_dev else CCS_HOST, self.leaf_depth,
                         (CCS_FLAG_LOCAL_FRAMES if local_frames else 0) | (CCS_FLAG_SINGLE_BOX if single_box else 0),
                         _stream(stream).value if on_dev else None)
        h = C.c_void_p()
        _check(lib().ccs_scene_create(C.byref(desc), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ccs_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = SceneInfo()
        _check(lib().ccs_scene_info_get(self._h, C.byref(i)))
        return dict(n_patches=i.n_patches, n_nodes=i.n_nodes, leaf_depth=i.leaf_depth, bvh_depth=i.bvh_depth,
                    device_bytes=int(i.device_bytes), lo=list(i.lo), hi=list(i.hi),
                    build_seconds=i.build_seconds, n_frames=i.n_frames)

    def set_frames(self, n_frames: int):
        _check(lib().ccs_scene_set_frames(self._h, int(n_frames)))

    def refit_frame(self, frame: int, control_points, stream=None):
        import torch
        cp = torch.as_tensor(control_points)
        if cp.dtype != torch.float32 or cp.numel() != self.n * 60:
            raise ValueError("refit input must be float32 with n x 20 x 3 values")
        cp = cp.contiguous()
        keep = getattr(self, "_refit_keep_frames", {})
        keep[int(frame)] = cp  # device input must outlive the queued work
        self._refit_keep_frames = keep
        _check(lib().ccs_refit_frame(self._h, int(frame), _ptr(cp), CCS_DEVICE if cp.is_cuda else CCS_HOST,
                                     _stream(stream)))

    def intersect_batched(self, batches, stream=None, counted: bool = False):
        """batches: list of (frame, rays (N, 8) cuda float32, hits (N, 4) cuda float32 or None).
        Returns the list of hit tensors (one launch for all batches), and with counted
        also the (sum N, 8) int32 work counters of the launch's rays in batch order."""
        import torch
        out, arr, total = [], (Batch * max(1, len(batches)))(), 0
        for k, (frame, rays, hits) in enumerate(batches):
            r = self._rays(rays)
            if hits is None:
                hits = torch.empty((r.shape[0], 4), dtype=torch.float32, device=r.device)
            hits = _out(hits, r.shape[0], 4, torch.float32, "hits")
            arr[k] = Batch(int(frame), r.shape[0], r.data_ptr(), hits.data_ptr())
            out.append(hits)
            total += r.shape[0]
        if not counted:
            _check(lib().ccs_intersect_batched(self._h, arr, len(batches), _stream(stream)))
            return out
        cnt = torch.empty((total, 8), dtype=torch.int32, device="cuda")
        _check(lib().ccs_intersect_batched_counted(self._h, arr, len(batches), _ptr(cnt), _stream(stream)))
        return out, cnt

    def set_launch(self, waves_per_cu: int = 0, fetch_min: int = 16, traverse_min: int = 1, grid_min: int = 8,
                   traverse_steps: int = 3, decide_min: int = 8):
        p = LaunchParams(waves_per_cu, fetch_min, traverse_min, grid_min, traverse_steps, decide_min)
        _check(lib().ccs_scene_set_launch(self._h, C.byref(p)))

    def get_launch(self) -> dict:
        p = LaunchParams()
        _check(lib().ccs_scene_get_launch(self._h, C.byref(p)))
        return dict(waves_per_cu=p.waves_per_cu, fetch_min=p.fetch_min, traverse_min=p.traverse_min,
                    grid_min=p.grid_min, traverse_steps=p.traverse_steps, decide_min=p.decide_min)

    def set_policy(self, params=None, stream=None):
        """Learned child order with the network `params` (CUDA float32, 1732 values);
        None returns to the closest-first order."""
        if params is None:
            _check(lib().ccs_scene_set_policy(self._h, None, _stream(stream)))
            return
        p = _params(params)
        self._policy_keep = p
        _check(lib().ccs_scene_set_policy(self._h, _ptr(p), _stream(stream)))

    def record(self, rays, hits, stream=None):
        """Training records of the ordering network: (features (N*L, 16), labels (N*L,) uint8)."""
        import torch
        r = self._rays(rays)
        h = torch.as_tensor(hits)
        if not h.is_cuda or h.dtype != torch.float32 or tuple(h.shape) != (r.shape[0], 4) or not h.is_contiguous():
            raise ValueError("hits must be a contiguous (N, 4) float32 CUDA tensor")
        L = self.info()["leaf_depth"]
        f = torch.empty((r.shape[0] * L, 16), dtype=torch.float32, device=r.device)
        y = torch.empty((r.shape[0] * L,), dtype=torch.uint8, device=r.device)
        _check(lib().ccs_policy_record(self._h, _ptr(r), _ptr(h), r.shape[0], _ptr(f), _ptr(y), _stream(stream)))
        return f, y

    @staticmethod
    def _rays(rays):
        import torch
        r = torch.as_tensor(rays)
        if not r.is_cuda or r.dtype != torch.float32 or r.dim() != 2 or r.shape[1] != 8 or not r.is_contiguous():
            raise ValueError("rays must be a contiguous (N, 8) float32 CUDA tensor")
        if r.shape[0] > MAX_RAYS:
            raise ValueError(f"at most {MAX_RAYS} rays per call")
        return r

    def intersect(self, rays, hits=None, stream=None):
        """Closest hits (N, 4) float32 {t, patch id bits, u, v}; ``hits_ids(h)`` reads the ids."""
        import torch
        r = self._rays(rays)
        n = r.shape[0]
        if hits is None:
            hits = torch.empty((n, 4), dtype=torch.float32, device=r.device)
        hits = _out(hits, n, 4, torch.float32, "hits")
        _check(lib().ccs_intersect(self._h, _ptr(r), n, _ptr(hits), _stream(stream)))
        return hits

    def intersect_counted(self, rays, stream=None):
        import torch
        r = self._rays(rays)
        n = r.shape[0]
        hits = torch.empty((n, 4), dtype=torch.float32, device=r.device)
        cnt = torch.empty((n, 8), dtype=torch.int32, device=r.device)
        _check(lib().ccs_intersect_counted(self._h, _ptr(r), n, _ptr(hits), _ptr(cnt), _stream(stream)))
        return hits, cnt

    def refit(self, control_points, stream=None):  # frame 0
        import torch
        cp = torch.as_tensor(control_points)
        if cp.dtype != torch.float32 or cp.numel() != self.n * 60:
            raise ValueError("refit input must be float32 with n x 20 x 3 values")
        cp = cp.contiguous()
        self._refit_keep = cp  # device input must outlive the queued work
        _check(lib().ccs_refit(self._h, _ptr(cp), CCS_DEVICE if cp.is_cuda else CCS_HOST, _stream(stream)))

    def debug_grids(self, patch_ids, codes, depths, frame: int = 0, stream=None):
        """Rows (N, DEBUG_GRID_FLOATS) float32 of ccs_debug_grids: stored points, the
        recomputed grid and displacement, and the split-chain grid of each subdomain."""
        import torch
        q = [torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.uint32)).view(np.int32)).cuda()
             for x in (patch_ids, codes, depths)]
        n = q[0].numel()
        if any(x.numel() != n for x in q):
            raise ValueError("patch_ids, codes and depths must have the same length")
        out = torch.empty((n, DEBUG_GRID_FLOATS), dtype=torch.float32, device=q[0].device)
        _check(lib().ccs_debug_grids(self._h, int(frame), _ptr(q[0]), _ptr(q[1]), _ptr(q[2]), n, _ptr(out),
                                     _stream(stream)))
        return out

    def bounce(self, rays, hits, uniforms, out=None, stream=None, frame: int = 0):
        """Secondary rays from hits (uniforms: (N, 2) float32 in [0, 1)) on the given frame."""
        import torch
        r = self._rays(rays)
        n = r.shape[0]
        h, u = torch.as_tensor(hits), torch.as_tensor(uniforms)
        if not (h.is_cuda and u.is_cuda and h.is_contiguous() and u.is_contiguous() and h.numel() == 4 * n
                and u.numel() == 2 * n and h.dtype == torch.float32 and u.dtype == torch.float32):
            raise ValueError("hits (N, 4) and uniforms (N, 2) must be contiguous float32 CUDA tensors")
        if out is None:
            out = torch.empty_like(r)
        out = _out(out, n, 8, torch.float32, "out")
        if out.data_ptr() == r.data_ptr():
            raise ValueError("out must not alias rays")
        _check(lib().ccs_bounce_frame(self._h, int(frame), _ptr(r), _ptr(h), _ptr(u), n, _ptr(out), _stream(stream)))
        return out


def compact_work_words(n: int) -> int:
    """Words of the workspace ccs_compact_rays needs for n rays (CCS_COMPACT_WORK_WORDS)."""
    return 1 + (int(n) + 255) // 256


def compact_rays(rays, out=None, index=None, work=None, stream=None):
    """The rays the intersection entry points trace, in input order (ccs_compact_rays).

    rays: (N, 8) float32 CUDA tensor.  out (>= N, 8) float32, index (>= N,) int32 (uint32
    bits) and work (>= compact_work_words(N),) int32 are allocated when not given.  Returns
    (out, index, work); the count m is work[0] (device): out[:m] and index[:m] are valid once
    the stream has reached the call."""
    import torch
    r = Scene._rays(rays)
    n = r.shape[0]
    if out is None:
        out = torch.empty_like(r)
    if index is None:
        index = torch.empty(n, dtype=torch.int32, device=r.device)
    if work is None:
        work = torch.empty(compact_work_words(n), dtype=torch.int32, device=r.device)
    for t, name, dt, ok in ((out, "out", torch.float32, out.dim() == 2 and out.shape[1] == 8 and out.shape[0] >= n),
                            (index, "index", torch.int32, index.dim() == 1 and index.numel() >= n),
                            (work, "work", torch.int32, work.dim() == 1 and work.numel() >= compact_work_words(n))):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and ok):
            raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor of sufficient size")
    if n > 0 and out.data_ptr() == r.data_ptr():
        raise ValueError("out must not alias rays")
    _check(lib().ccs_compact_rays(_ptr(r), n, _ptr(out), _ptr(index), _ptr(work), _stream(stream)))
    return out, index, work


def _out(t, n: int, width: int, dtype, name: str):
    """A caller-supplied output tensor: the kernel writes exactly n x width values into it."""
    import torch
    t = torch.as_tensor(t)
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != (n, width):
        raise ValueError(f"{name} must be a contiguous ({n}, {width}) {dtype} CUDA tensor")
    return t


def _params(params):
    import torch
    p = torch.as_tensor(params)
    if not p.is_cuda or p.dtype != torch.float32 or p.numel() != POLICY_PARAMS or not p.is_contiguous():
        raise ValueError(f"policy parameters must be a contiguous CUDA float32 tensor of {POLICY_PARAMS} values")
    return p


def _rows(x, width, dtype):
    import torch
    t = torch.as_tensor(x)
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or (width and (t.dim() != 2 or t.shape[1] != width)):
        raise ValueError(f"expected a contiguous CUDA {dtype} tensor" + (f" of shape (N, {width})" if width else ""))
    return t


def policy_infer(params, features, stream=None):
    """Logits (N, 4) of the ordering network, computed as during traversal."""
    import torch
    p, f = _params(params), _rows(features, 16, torch.float32)
    z = torch.empty((f.shape[0], 4), dtype=torch.float32, device=f.device)
    _check(lib().ccs_policy_infer(_ptr(p), _ptr(f), f.shape[0], _ptr(z), _stream(stream)))
    return z


def policy_grad(params, features, labels, bf16: bool = False, stream=None):
    """(mean loss, gradient (1732,)) of the ordering network on labelled rows."""
    import torch
    p, f = _params(params), _rows(features, 16, torch.float32)
    y = _rows(labels, 0, torch.uint8)
    if y.numel() != f.shape[0]:
        raise ValueError("one label per row")
    g = torch.empty(POLICY_PARAMS, dtype=torch.float32, device=f.device)
    loss = torch.empty(1, dtype=torch.float32, device=f.device)
    _check(lib().ccs_policy_grad(_ptr(p), _ptr(f), _ptr(y), f.shape[0], int(bf16), _ptr(g), _ptr(loss),
                                 _stream(stream)))
    return float(loss.item()), g


def policy_grad_noalloc(params, features, labels, grad, loss, bf16: bool = False, stream=None):
    """policy_grad into caller-given grad (1732,) and loss (1,) float32 CUDA tensors,
    with the library's preallocated scratch (no device allocation; asynchronous;
    at most GRAD_NOALLOC_MAX_ROWS rows; calls overlapping on one device race)."""
    import torch
    p, f = _params(params), _rows(features, 16, torch.float32)
    y = _rows(labels, 0, torch.uint8)
    if y.numel() != f.shape[0]:
        raise ValueError("one label per row")
    for t, k, name in ((grad, POLICY_PARAMS, "grad"), (loss, 1, "loss")):
        if not (torch.is_tensor(t) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and t.numel() == k):
            raise ValueError(f"{name} must be a contiguous CUDA float32 tensor of {k} values")
    if f.shape[0] > GRAD_NOALLOC_MAX_ROWS:
        raise ValueError(f"at most {GRAD_NOALLOC_MAX_ROWS} rows")
    _check(lib().ccs_policy_grad_noalloc(_ptr(p), _ptr(f), _ptr(y), f.shape[0], int(bf16), _ptr(grad), _ptr(loss),
                                         _stream(stream)))


class Adam:
    """Adam's moments (two CUDA float32 tensors of 1732 values) and its step count,
    carried across policy_train calls."""

    def __init__(self, device="cuda", m=None, v=None, t: int = 0):
        import torch
        self.m = torch.zeros(POLICY_PARAMS, dtype=torch.float32, device=device) if m is None else _params(m)
        self.v = torch.zeros(POLICY_PARAMS, dtype=torch.float32, device=device) if v is None else _params(v)
        self.t = int(t)


def policy_train(params, features, labels, steps: int, batch: int = 4096, lr: float = 3e-3, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, seed: int = 0, bf16: bool = True, state: Adam = None,
                 stream=None):
    """Adam on the ordering network, params updated in place; returns the per-step loss.
    state: None for a fresh start, else an Adam whose moments and step count are used and advanced."""
    import torch
    p, f = _params(params), _rows(features, 16, torch.float32)
    y = _rows(labels, 0, torch.uint8)
    if y.numel() != f.shape[0]:
        raise ValueError("one label per row")
    hist = torch.empty(max(1, steps), dtype=torch.float32, device=f.device)
    tp = TrainParams(steps, batch, lr, beta1, beta2, eps, seed, int(bf16), 0)
    st = None
    if state is not None:
        st = AdamState(_ptr(_params(state.m)), _ptr(_params(state.v)), state.t)
    _check(lib().ccs_policy_train(_ptr(p), _ptr(f), _ptr(y), f.shape[0], C.byref(tp),
                                  C.byref(st) if st is not None else None, _ptr(hist), _stream(stream)))
    if st is not None:
        state.t = int(st.t)
    return hist[:steps]


def device_bytes_in_use() -> int:
    """Device bytes the library holds in this process (every scene and call temporaries)."""
    return int(lib().ccs_device_bytes_in_use())


def hit_ids(hits) -> np.ndarray:
    """Patch ids of a hits tensor/array as uint32 (CCS_NO_HIT for misses)."""
    h = hits.detach().cpu().numpy() if hasattr(hits, "detach") else np.asarray(hits)
    return np.ascontiguousarray(h[:, 1]).view(np.uint32)
