"""Device memory accounting and the CCS_MAX_DEVICE_BYTES cap on the GPU: a cap
one byte below what a scene needs refuses it with CCS_ERR_OOM and leaks nothing,
the exact figure admits it, and a policy call's temporaries are refused the same
way without touching the caller's parameters."""
import os

import numpy as np
import pytest

from paper_1811_03510_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ENV = "CCS_MAX_DEVICE_BYTES"


@pytest.fixture(scope="module")
def ccs():
    from paper_1811_03510_amd import ccs as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


@pytest.fixture
def cap():
    old = os.environ.get(ENV)

    def set_cap(v):
        if v is None:
            os.environ.pop(ENV, None)
        else:
            os.environ[ENV] = str(v)
    yield set_cap
    set_cap(old)


@pytest.mark.parametrize("local", [False, True], ids=["world", "local"])
def test_cap_admits_exactly_what_a_scene_needs(ccs, c1, cap, local):
    cp, ty = torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda()
    torch.cuda.synchronize()
    base = ccs.device_bytes_in_use()
    sc = ccs.Scene(cp, ty, c1.leaf_depth, local_frames=local)
    need = sc.info()["device_bytes"]
    assert need > c1.cp.nbytes and ccs.device_bytes_in_use() == base + need
    sc.close()
    assert ccs.device_bytes_in_use() == base
    cap(base + need - 1)
    with pytest.raises(ccs.CcsError) as e:
        ccs.Scene(cp, ty, c1.leaf_depth, local_frames=local)
    assert e.value.status == ccs.CCS_ERR_OOM and ENV in str(e.value)
    assert ccs.device_bytes_in_use() == base  # the failed create freed what it had
    cap(base + need)
    sc = ccs.Scene(cp, ty, c1.leaf_depth, local_frames=local)
    assert sc.info()["device_bytes"] == need
    hits = sc.intersect(torch.from_numpy(c1.primary[:4096]).cuda())  # launches allocate nothing
    torch.cuda.synchronize()
    assert (ccs.hit_ids(hits) != ccs.NO_HIT).any()
    sc.close()
    assert ccs.device_bytes_in_use() == base


def test_frames_and_policy_temporaries_are_capped(ccs, c1, cap):
    cp, ty = torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda()
    sc = ccs.Scene(cp, ty, c1.leaf_depth)
    base = ccs.device_bytes_in_use()
    cap(base + 1000)
    with pytest.raises(ccs.CcsError) as e:
        sc.set_frames(4)
    assert e.value.status == ccs.CCS_ERR_OOM and ccs.device_bytes_in_use() == base
    assert sc.info()["n_frames"] == 1
    th = torch.from_numpy(S.mlp_init()).cuda()
    before = th.clone()
    X = torch.zeros((4096, 16), dtype=torch.float32, device="cuda")
    y = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(ccs.CcsError) as e:
        ccs.policy_train(th, X, y, steps=3, batch=4096)
    assert e.value.status == ccs.CCS_ERR_OOM and ccs.device_bytes_in_use() == base
    assert torch.equal(th, before)
    cap(None)
    sc.set_frames(4)
    held = ccs.device_bytes_in_use()
    assert sc.info()["n_frames"] == 4 and held > base
    ccs.policy_train(th, X, y, steps=3, batch=4096)
    assert not torch.equal(th, before) and ccs.device_bytes_in_use() == held  # temporaries returned
    sc.close()


def test_malformed_cap_is_an_argument_error(ccs, c1, cap):
    cap("12abc")
    with pytest.raises(ccs.CcsError) as e:
        ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth)
    assert e.value.status == ccs.CCS_ERR_INVALID_ARG and ENV in str(e.value)


def test_binding_rejects_outputs_the_kernels_would_overrun(ccs, c1):
    sc = ccs.Scene(torch.from_numpy(c1.cp).cuda(), torch.from_numpy(c1.types).cuda(), c1.leaf_depth)
    rays = torch.from_numpy(c1.primary[:1000]).cuda()
    for bad in (torch.empty((999, 4), device="cuda"), torch.empty((1000, 4), device="cuda", dtype=torch.float64),
                torch.empty((4, 1000), device="cuda").t(), torch.empty((1000, 4))):
        with pytest.raises(ValueError):
            sc.intersect(rays, bad)
        with pytest.raises(ValueError):
            sc.intersect_batched([(0, rays, bad)])
    with pytest.raises(ValueError):
        sc.intersect(rays.reshape(10, 100, 8))
    hits = sc.intersect(rays)
    u = torch.rand((1000, 2), device="cuda")
    with pytest.raises(ValueError):
        sc.bounce(rays, hits, u, out=torch.empty((999, 8), device="cuda"))
    with pytest.raises(ValueError):
        sc.bounce(rays, hits, u, out=rays)
    out = sc.bounce(rays, hits, u)
    torch.cuda.synchronize()
    assert out.shape == (1000, 8) and torch.isfinite(out[:, :3]).all()
    sc.close()
