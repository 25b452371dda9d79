"""The C ABI without a GPU: the library loads, exports every declared entry point,
and validates arguments on the host before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1811_03510_amd import ccs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ccs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 8
    lib = ccs.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ccs.EXPORTS)


def test_struct_layouts():
    class Ray(C.Structure):
        _fields_ = [(f, C.c_float) for f in ("ox", "oy", "oz", "tmin", "dx", "dy", "dz", "tmax")]

    class Hit(C.Structure):
        _fields_ = [("t", C.c_float), ("patch_id", C.c_uint32), ("u", C.c_float), ("v", C.c_float)]
    assert C.sizeof(Ray) == 32 and C.sizeof(Hit) == 16
    assert C.sizeof(ccs.SceneDesc) == 40


def create(desc):
    h = C.c_void_p()
    st = ccs.lib().ccs_scene_create(C.byref(desc) if desc is not None else None, C.byref(h))
    return st, ccs.lib().ccs_last_error().decode(), h


def host_desc(cp, ty, L=12, flags=0, location=ccs.CCS_HOST):
    return ccs.SceneDesc(cp.ctypes.data if cp is not None else None, ty.ctypes.data if ty is not None else None,
                         len(ty) if ty is not None else 3, location, L, flags, None)


def test_host_validation_errors():
    cp = np.zeros((3, 20, 3), np.float32)
    ty = np.zeros(3, np.uint8)
    st, msg, _ = create(None)
    assert st == ccs.CCS_ERR_INVALID_ARG and "desc" in msg
    assert ccs.lib().ccs_scene_create(C.byref(host_desc(cp, ty)), None) == ccs.CCS_ERR_INVALID_ARG
    st, msg, h = create(host_desc(None, ty))
    assert st == ccs.CCS_ERR_INVALID_ARG and h.value is None
    for L in (0, 21, 23, 100):
        st, msg, _ = create(host_desc(cp, ty, L=L))
        assert st == ccs.CCS_ERR_INVALID_ARG and "leaf_depth" in msg
    bad = ty.copy()
    bad[1] = 2
    st, msg, _ = create(host_desc(cp, bad))
    assert st == ccs.CCS_ERR_INVALID_ARG and "type" in msg
    for v in (np.nan, np.inf, -np.inf):
        c2 = cp.copy()
        c2[2, 7, 1] = v
        st, msg, _ = create(host_desc(c2, ty))
        assert st == ccs.CCS_ERR_INVALID_ARG and "finite" in msg
    for flags in (4, 0x80000000):  # bits 0 (local frames) and 1 (single-box ablation) are the only flags
        st, msg, _ = create(host_desc(cp, ty, flags=flags))
        assert st == ccs.CCS_ERR_UNSUPPORTED and "flags" in msg
    st, msg, _ = create(host_desc(cp, ty, location=7))
    assert st == ccs.CCS_ERR_INVALID_ARG


def test_null_scene_calls_fail_cleanly():
    L = ccs.lib()
    assert L.ccs_intersect(None, None, 0, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_refit(None, None, 0, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_bounce(None, None, None, None, 4, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_intersect_counted(None, None, 1, None, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_scene_info_get(None, None) == ccs.CCS_ERR_INVALID_ARG
    L.ccs_scene_destroy(None)
    assert "NULL" in L.ccs_last_error().decode()


def test_binding_fails_loudly_without_the_library(monkeypatch):
    monkeypatch.setattr(ccs, "_lib", None)
    monkeypatch.setattr(ccs, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libccs.so"))
    with pytest.raises(ImportError):
        ccs.lib()


def test_new_struct_layouts():
    assert C.sizeof(ccs.LaunchParams) == 24
    assert C.sizeof(ccs.Batch) == 24
    assert C.sizeof(ccs.TrainParams) == 40
    assert ccs.TrainParams.seed.offset == 24


def test_policy_and_batch_entry_points_validate_on_the_host():
    L = ccs.lib()
    fake = C.c_void_p(16)  # never dereferenced: each call fails validation first
    assert L.ccs_scene_set_policy(None, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_policy_record(None, fake, fake, 4, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_policy_infer(None, fake, 4, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_policy_infer(fake, fake, 0, None, None) == ccs.CCS_OK  # empty input is a no-op
    assert L.ccs_policy_grad(None, fake, fake, 4, 0, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_policy_grad(fake, None, fake, 4, 0, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG
    tp = ccs.TrainParams(10, 0, 1e-3, 0.9, 0.999, 1e-8, 1, 1, 0)
    assert L.ccs_policy_train(fake, fake, fake, 100, C.byref(tp), None, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert "batch" in L.ccs_last_error().decode()
    for bad in (dict(lr=0.0), dict(beta1=1.0), dict(beta2=-0.1), dict(eps=0.0)):
        kw = dict(steps=10, batch=64, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=1, bf16=1, reserved=0)
        kw.update(bad)
        tp = ccs.TrainParams(**kw)
        assert L.ccs_policy_train(fake, fake, fake, 100, C.byref(tp), None, None, None) == ccs.CCS_ERR_INVALID_ARG, bad
    tp = ccs.TrainParams(0, 64, 1e-3, 0.9, 0.999, 1e-8, 1, 1, 0)
    assert L.ccs_policy_train(fake, fake, fake, 100, C.byref(tp), None, None, None) == ccs.CCS_OK  # no steps
    assert L.ccs_policy_train(None, fake, fake, 100, C.byref(tp), None, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_intersect_batched(None, None, 1, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_bounce_frame(None, 0, fake, fake, fake, 4, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_scene_set_frames(None, 2) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_refit_frame(None, 0, fake, 1, None) == ccs.CCS_ERR_INVALID_ARG
    p = ccs.LaunchParams(0, 16, 1, 16, 2, 0)
    assert L.ccs_scene_set_launch(None, C.byref(p)) == ccs.CCS_ERR_INVALID_ARG


def test_ray_count_bound_is_checked_before_any_launch():
    # the persistent kernel's 32-bit ray counter must not wrap: 2^31 rays or more
    # are refused on the host (the scene pointer is not dereferenced on this path)
    L = ccs.lib()
    fake = C.c_void_p(16)
    for n in ((1 << 31), (1 << 32) - 1):
        assert L.ccs_intersect(fake, fake, n, fake, None) == ccs.CCS_ERR_INVALID_ARG
        assert "2^31" in L.ccs_last_error().decode()
        assert L.ccs_intersect_counted(fake, fake, n, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG



def test_measurement_and_noalloc_entry_points_validate_on_the_host():
    L = ccs.lib()
    fake = C.c_void_p(16)  # never dereferenced: each call fails validation first
    assert L.ccs_debug_grids(None, 0, fake, fake, fake, 4, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_intersect_batched_counted(None, None, 1, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_intersect_batched_counted(fake, None, 1, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert "counters" in L.ccs_last_error().decode()
    # the entry point that allocates nothing refuses rows beyond its scratch before any device call
    assert L.ccs_policy_grad_noalloc(None, fake, fake, 4, 0, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG
    n = ccs.GRAD_NOALLOC_MAX_ROWS + 1
    assert L.ccs_policy_grad_noalloc(fake, fake, fake, n, 0, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert "scratch" in L.ccs_last_error().decode()


def test_compaction_validates_on_the_host():
    L = ccs.lib()
    fake, other = C.c_void_p(16), C.c_void_p(4096)  # never dereferenced: each call fails validation first
    assert L.ccs_compact_rays(fake, 4, other, fake, None, None) == ccs.CCS_ERR_INVALID_ARG
    assert "work" in L.ccs_last_error().decode()
    assert L.ccs_compact_rays(None, 4, other, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert L.ccs_compact_rays(fake, 4, fake, other, other, None) == ccs.CCS_ERR_INVALID_ARG
    assert "alias" in L.ccs_last_error().decode()
    assert L.ccs_compact_rays(C.c_void_p(24), 4, other, fake, fake, None) == ccs.CCS_ERR_INVALID_ARG
    assert "aligned" in L.ccs_last_error().decode()
    # the workspace: the count and one word per block of 256 rays
    assert [ccs.compact_work_words(n) for n in (0, 1, 256, 257, 2**32 - 1)] == [1, 2, 2, 3, 1 + 2**24]
