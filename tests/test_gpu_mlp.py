"""GPU parity of the learned-correction kernels against the oracle's FP64
reference, on identical bf16-rounded weights and inputs: forward within 1e-2
relative, gradients within 2e-2 relative in the 2-norm of each parameter
block (bf16 operands and bf16-stored back-propagated signals, fp32 accumulation);
features within 1e-6 (fp32 output of FP64 moments); Adam within fp32 rounding."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rsl():
    from paper_1612_01287_amd import rsl as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mod


def bf16_round(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_features_match_oracle(rsl):
    vs = oracle.VelocitySet(3, 8, 3)
    quad = rsl.Quadrature(3, 8, 3)
    for dtype in ("f64", "f32"):
        p = rsl.make_problem(nz=700, dtype=dtype, tau_r=0.05)
        inst = rsl.Instance(quad, p)
        inst.init()
        inst.step(0.5 / 700, 30)
        f = inst.f().double().cpu().numpy()
        got = rsl.features(quad, p, inst.f_buf, np.log(0.05)).cpu().numpy()
        ref = mlp.features(vs, f, np.log(0.05))
        assert np.max(np.abs(got - ref) / (np.abs(ref) + 1e-3)) < 2e-6


def test_standardised_features(rsl):
    """(x - shift) / scale in fp32, as the training data are prepared."""
    quad = rsl.Quadrature(3, 16, 4)
    p = rsl.make_problem(nz=300, dtype="f64", tau_r=0.05)
    inst = rsl.Instance(quad, p)
    inst.init()
    inst.step(0.5 / 300, 20)
    raw = rsl.features(quad, p, inst.f_buf, np.log(0.05))
    shift = raw.mean(dim=0).contiguous()
    scale = raw.std(dim=0).clamp_min(1e-4).contiguous()
    got = rsl.features(quad, p, inst.f_buf, np.log(0.05), shift, scale)
    assert torch.equal(got, (raw - shift) / scale)
    with pytest.raises(RuntimeError):
        rsl.features(quad, p, inst.f_buf, np.log(0.05), shift, None)


@pytest.mark.parametrize("n", [1, 63, 64, 1000])
def test_forward_backward_match_oracle(rsl, n):
    rng = np.random.default_rng(n)
    P = mlp.init_params(3)
    for k in P:
        P[k] = P[k] + 0.02 * rng.standard_normal(P[k].shape)
    net = rsl.MLP(rsl.MLP.pack(P))
    Pb = {k: bf16_round(v) for k, v in P.items()}           # what the kernels compute with
    X = rng.standard_normal((n, 81)).astype(np.float32)
    T = rng.standard_normal((n, 3)).astype(np.float32) * 0.1
    Xd = torch.tensor(X, device="cuda")
    Td = torch.tensor(T, device="cuda")
    y, h1, h2 = net.forward(Xd, keep=True)
    yref, cache = mlp.forward(Pb, bf16_round(X))
    assert _rel(y.cpu().numpy(), yref) < 1e-2
    G = net.backward(Xd, h1, h2, y, Td).cpu().numpy()
    Gref = mlp.backward(Pb, cache, yref, T.astype(np.float64))
    flat = rsl.MLP.pack(Gref)
    off = 0
    for name, shp in rsl.MLP_SHAPES:
        k = int(np.prod(shp))
        a, b = G[off:off + k], flat[off:off + k]
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 2e-2, name
        assert _rel(a, b) < 5e-2, name
        off += k


def test_adam_matches_oracle(rsl):
    rng = np.random.default_rng(9)
    P = mlp.init_params(4)
    net = rsl.MLP(rsl.MLP.pack(P))
    state = {}
    Pc = {k: v.copy() for k, v in P.items()}
    for t in range(1, 4):
        G = {k: rng.standard_normal(v.shape) for k, v in P.items()}
        net.grad.copy_(torch.tensor(rsl.MLP.pack(G), dtype=torch.float32))
        net.adam(lr=1e-2)
        mlp.adam_step(Pc, G, state, t, lr=1e-2)
    got = net.params.cpu().numpy()
    ref = rsl.MLP.pack(Pc)
    assert np.max(np.abs(got - ref)) < 1e-5


def test_training_reduces_loss(rsl):
    """A few hundred Adam steps on a smooth synthetic target fall well below
    the initial loss (the training loop runs entirely in the kernels)."""
    rng = np.random.default_rng(1)
    n = 4096
    X = rng.uniform(-1, 1, (n, 81)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]) * 0.3, X[:, 1] * X[:, 2] * 0.2, 0.1 * X[:, 3]], axis=1).astype(np.float32)
    net = rsl.MLP(rsl.MLP.pack(mlp.init_params(0)))
    Xd, Td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    losses = []
    for it in range(300):
        y, h1, h2 = net.forward(Xd, keep=True)
        losses.append(float(((y - Td) ** 2).mean()))
        net.backward(Xd, h1, h2, y, Td)
        net.adam(lr=3e-3)
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])
