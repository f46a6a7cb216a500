"""rsl_mlp_backward_noalloc (partial gradients in the library's scratch array)
against rsl_mlp_backward (partial gradients in a caller workspace), through
the C ABI, on two calls in a row, the second with fewer samples: the same
kernels in the same partition give bitwise equal gradients."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _sig(lib):
    f = lib.rsl_mlp_backward_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    return f


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_backward_noalloc_matches_workspace_call():
    from paper_1612_01287_amd import rsl
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    noalloc = _sig(rsl.lib())
    rng = np.random.default_rng(31)
    net = rsl.MLP(rng.standard_normal(rsl.RSL_MLP_NPARAM) * 0.1)
    stream = torch.cuda.current_stream()
    for n in (20000, 777):                      # 256 workgroups of partials, then 13
        x = torch.as_tensor(rng.standard_normal((n, 81)), dtype=torch.float32, device="cuda")
        t = torch.as_tensor(rng.standard_normal((n, 3)), dtype=torch.float32, device="cuda")
        y, h1, h2 = net.forward(x, keep=True)
        want = net.backward(x, h1, h2, y, t).clone()
        got = torch.full_like(want, float("nan"))
        rc = noalloc(_p(net.pb), _p(x), _p(h1), _p(h2), _p(y), _p(t), n, _p(got),
                     ctypes.c_void_p(stream.cuda_stream))
        assert rc == 0, rsl.lib().rsl_last_error()
        torch.cuda.synchronize()
        assert torch.isfinite(want).all()
        assert torch.equal(got, want), n
    x = torch.zeros((1, 81), device="cuda")
    assert noalloc(_p(net.pb), _p(x), _p(h1), _p(h2), _p(y), _p(t), 0, _p(got),
                   ctypes.c_void_p(stream.cuda_stream)) == rsl.RSL_EINVAL
