"""np_net_mse_noalloc (the entry point for callers that cannot allocate)
against np_net_mse with a caller-provided workspace: same kernels, so the
loss and the gradient must agree bit for bit.  Two calls in a row, the
second with a smaller input, so the shared static partials of the first call
are still in place when the second one runs."""
import ctypes

import pytest
import torch

from paper_2001_02327_amd import _lib

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _mse_workspace(L, pred, target, mask, count, stream):
    n = pred.numel()
    ws = L.np_net_workspace_bytes(1, 1, n)
    work = torch.empty(ws // 4 + 1, dtype=torch.float32, device=pred.device)
    grad = torch.empty_like(pred)
    loss = torch.zeros(1, dtype=torch.float32, device=pred.device)
    rc = L.np_net_mse(_p(pred), _p(target), _p(mask), n, count, _p(grad), _p(loss), _p(work), ws, stream)
    assert rc == 0
    return grad, loss


def _mse_noalloc(L, pred, target, mask, count, stream):
    n = pred.numel()
    grad = torch.empty_like(pred)
    loss = torch.zeros(1, dtype=torch.float32, device=pred.device)
    rc = L.np_net_mse_noalloc(_p(pred), _p(target), _p(mask), n, count, _p(grad), _p(loss), stream)
    assert rc == 0, L.nested_poisson_last_error(None)
    return grad, loss


def test_noalloc_mse_matches_workspace_mse():
    L = _lib.lib()
    dev = torch.device("cuda", 0)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    gen = torch.Generator(device="cpu").manual_seed(1234)
    # sizes: several blocks of partials with a ragged tail, then a smaller call
    for n, masked in ((3 * 1000 * 1000 + 77, True), (70001, False)):
        print("np_net_mse_noalloc: n = %d, mask = %s" % (n, masked), flush=True)
        pred = torch.randn(n, generator=gen, dtype=torch.float32).to(dev)
        target = torch.randn(n, generator=gen, dtype=torch.float32).to(dev)
        mask = (torch.rand(n, generator=gen) > 0.3).to(torch.float32).to(dev) if masked else None
        count = float(mask.sum().item()) if masked else float(n)
        g_ref, l_ref = _mse_workspace(L, pred, target, mask, count, stream)
        g_new, l_new = _mse_noalloc(L, pred, target, mask, count, stream)
        torch.cuda.synchronize()
        assert torch.equal(g_new, g_ref)
        assert torch.equal(l_new, l_ref)
        # and both against a plain FP64 evaluation of the definition
        d = (pred.double() - target.double()) * (mask.double() if masked else 1.0)
        assert abs(float(l_new.item()) - float((d * d).sum().item() / count)) <= 1e-5 * float(l_new.item())


def test_noalloc_mse_rejects_oversized_input():
    L = _lib.lib()
    dev = torch.device("cuda", 0)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    x = torch.zeros(4, dtype=torch.float32, device=dev)
    # the size check comes before any device work, so the small buffers are never read
    rc = L.np_net_mse_noalloc(_p(x), _p(x), None, _lib.NP_NET_MSE_NOALLOC_MAX + 1, 1.0, _p(x), _p(x), stream)
    assert rc == _lib.NP_EINVAL
    assert b"exceeds the maximum" in L.nested_poisson_last_error(None)
