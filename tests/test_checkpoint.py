"""Training checkpoints (.npz) and the host-side checks of resumable training."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_1811_03510_amd import ccs, checkpoint


def _arrays(seed):
    g = np.random.default_rng(seed)
    p = g.standard_normal(ccs.POLICY_PARAMS).astype(np.float32)
    p[:4] = [-0.0, np.float32(1e-45), np.float32(-3e-39), np.float32(3.4e38)]  # signed zero, subnormals, near max
    m = g.standard_normal(ccs.POLICY_PARAMS).astype(np.float32) * 1e-3
    v = np.abs(g.standard_normal(ccs.POLICY_PARAMS)).astype(np.float32) * 1e-6
    return p, m, v


def test_round_trip_is_bit_exact(tmp_path):
    p, m, v = _arrays(1)
    path = str(tmp_path / "ckpt.npz")
    hyper = {"lr": 3e-3, "batch": 4096, "seed": 7}
    checkpoint.save(path, p, m, v, t=12345, hyper=hyper)
    c = checkpoint.load(path)
    for k, a in (("params", p), ("adam_m", m), ("adam_v", v)):
        assert c[k].dtype == np.float32 and np.array_equal(c[k].view(np.uint32), a.view(np.uint32)), k
    assert c["adam_t"] == 12345 and c["hyper"] == hyper
    assert os.listdir(tmp_path) == ["ckpt.npz"]  # the temporary file was renamed away


def test_fresh_state_defaults_and_overwrite(tmp_path):
    p, _, _ = _arrays(2)
    path = str(tmp_path / "c.npz")
    checkpoint.save(path, p)
    c = checkpoint.load(path)
    assert c["adam_t"] == 0 and not c["adam_m"].any() and not c["adam_v"].any() and c["hyper"] == {}
    checkpoint.save(path, p + 1, t=3)
    assert checkpoint.load(path)["adam_t"] == 3


def test_rejects_bad_files(tmp_path):
    p, m, v = _arrays(3)
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), p[:10])
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), p, t=-1)
    other = str(tmp_path / "other.npz")
    np.savez(other, format=np.array("something else"), params=p)
    with pytest.raises(ValueError):
        checkpoint.load(other)
    bad = str(tmp_path / "nan.npz")
    m2 = m.copy()
    m2[5] = np.nan
    checkpoint.save(bad, p, m2, v)
    with pytest.raises(ValueError):
        checkpoint.load(bad)


def test_adam_state_layout_and_validation():
    assert C.sizeof(ccs.AdamState) == 24 and ccs.AdamState.t.offset == 16
    L = ccs.lib()
    fake = C.c_void_p(16)  # never dereferenced: each call fails validation first
    tp = ccs.TrainParams(10, 64, 1e-3, 0.9, 0.999, 1e-8, 1, 1, 0)
    st = ccs.AdamState(None, fake.value, 0)
    assert L.ccs_policy_train(fake, fake, fake, 100, C.byref(tp), C.byref(st), None, None) == ccs.CCS_ERR_INVALID_ARG
    assert "moments" in L.ccs_last_error().decode()
    st = ccs.AdamState(fake.value, fake.value, (1 << 32) + 1)
    assert L.ccs_policy_train(fake, fake, fake, 100, C.byref(tp), C.byref(st), None, None) == ccs.CCS_ERR_INVALID_ARG
    assert "2^32" in L.ccs_last_error().decode()


def test_nothing_held_without_a_device():
    assert ccs.device_bytes_in_use() == 0
