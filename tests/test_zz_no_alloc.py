"""ccs_policy_grad_noalloc (the gradient entry point that allocates nothing, for
callers under graph capture or in tight loops) against ccs_policy_grad: the same
kernels on the same rows, so the gradient and the loss are bitwise equal; two
calls in a row, the second on fewer rows (the library's scratch keeps the first
call's rows, which the second must not read), then the row limit and an empty
input (zero gradient, a fill kernel rather than a memset)."""
import ctypes as C

import numpy as np
import pytest

from paper_1811_03510_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.normal(size=(n, 16)).astype(np.float32)).cuda()
    y = rng.integers(0, 4, n).astype(np.uint8)
    y[::7] = 255  # unlabelled rows carry nothing
    return X, torch.from_numpy(y).cuda()


def _noalloc(L, th, X, y, bf16, stream):
    g = torch.full((1732,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    st = L.ccs_policy_grad_noalloc(C.c_void_p(th.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()),
                                   X.shape[0], int(bf16), C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr()),
                                   stream)
    return st, g, loss


def test_noalloc_gradient_equals_the_allocating_entry_point():
    from paper_1811_03510_amd import ccs
    L = ccs.lib()
    th = torch.from_numpy(S.mlp_init()).cuda()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, seed, bf16 in ((16384, 1, True), (1000, 2, False), (64, 3, True), (1, 4, False)):
        print(f"no-alloc gradient: {n} rows, bf16 {bf16}", flush=True)
        X, y = _rows(n, seed)
        loss_ref, g_ref = ccs.policy_grad(th, X, y, bf16=bf16)
        st, g, loss = _noalloc(L, th, X, y, bf16, stream)
        assert st == ccs.CCS_OK, L.ccs_last_error().decode()
        torch.cuda.synchronize()
        assert np.array_equal(g.cpu().numpy().view(np.uint32), g_ref.cpu().numpy().view(np.uint32)), n
        assert np.float32(loss.item()).view(np.uint32) == np.float32(loss_ref).view(np.uint32), n
    # beyond the scratch: a clear error, nothing launched
    X, y = _rows(ccs.GRAD_NOALLOC_MAX_ROWS + 1, 5)
    st, g, _ = _noalloc(L, th, X, y, False, stream)
    assert st == ccs.CCS_ERR_INVALID_ARG and "scratch" in L.ccs_last_error().decode()
    torch.cuda.synchronize()
    assert torch.isnan(g).all()
    # no rows: zero gradient and loss
    X0 = torch.empty((0, 16), dtype=torch.float32, device="cuda")
    y0 = torch.empty((0,), dtype=torch.uint8, device="cuda")
    loss_ref, g_ref = ccs.policy_grad(th, X0, y0)
    st, g, loss = _noalloc(L, th, X0, y0, False, stream)
    assert st == ccs.CCS_OK
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), g_ref.cpu().numpy()) and float(loss.item()) == loss_ref
