"""The allocation-free loss (ngd_l2_loss_noalloc) against ngd_l2_loss,
through the C-ABI: identical loss and gradient bits on two calls in a row,
the second with a smaller input, so the second reuses the static scratch
the first left filled.  Also checked against the float64 mean squared
error."""

import ctypes

import numpy as np
import pytest

from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    return torch


def _call(L, name, f, t, loss, grad, stream):
    q = f.numel() // 3
    rc = getattr(L, name)(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(t.data_ptr()), q,
                          ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                          stream)
    assert rc == 0, L.ngd_last_error()


def test_noalloc_loss_matches_allocating_loss(torch_cuda):
    torch = torch_cuda
    from paper_2405_20067_amd import ngd
    L = ngd.lib()
    rng = np.random.default_rng(2024)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for q in (700001, 4099, 1, 0):
        print(f"noalloc loss: q={q}", flush=True)
        f = dev(rng.standard_normal((q, 3)).astype(np.float32))
        t = dev(rng.standard_normal((q, 3)).astype(np.float32))
        loss_a = torch.full((1,), float("nan"), device="cuda")
        loss_b = torch.full((1,), float("nan"), device="cuda")
        grad_a = torch.full((q, 3), float("nan"), device="cuda")
        grad_b = torch.full((q, 3), float("nan"), device="cuda")
        _call(L, "ngd_l2_loss", f, t, loss_a, grad_a, stream)
        _call(L, "ngd_l2_loss_noalloc", f, t, loss_b, grad_b, stream)
        torch.cuda.synchronize()
        la, lb = host(loss_a), host(loss_b)
        assert la.tobytes() == lb.tobytes(), (q, la, lb)
        assert host(grad_a).tobytes() == host(grad_b).tobytes(), q
        d = host(f).astype(np.float64) - host(t)
        want = float(np.mean(d * d)) if q else 0.0
        assert float(lb[0]) == pytest.approx(want, rel=1e-6, abs=1e-30)


def test_noalloc_loss_binding(torch_cuda):
    torch = torch_cuda
    from paper_2405_20067_amd import ngd
    f = dev(np.arange(12, dtype=np.float32).reshape(4, 3))
    t = torch.zeros_like(f)
    loss, grad = ngd.l2_loss_noalloc(f, t, torch.empty(1, device="cuda"), torch.empty_like(f))
    torch.cuda.synchronize()
    v = np.arange(12, dtype=np.float64)
    assert float(host(loss)[0]) == pytest.approx(np.mean(v * v), rel=1e-6)
    np.testing.assert_allclose(host(grad).ravel(), 2 * v / 12, rtol=1e-6)
