"""GPU parity of the velocity sets with azimuthal nodes (rsl_make_quadrature3,
rsl_feq3, rsl_moments3) against the oracle (oracle/vel3d.py): the equilibrium
at every node for fluid velocities in any direction, and the moments with the
Landau frame of off-equilibrium populations.  Sec. III D (eq. leg_product and
the azimuthal rule), eqs. feq_trunc, fjk, macro_jk; Sec. II E.

Bar: max |gpu - oracle| / max |oracle| <= 1e-12 for binary64 populations and
derived fields, 1e-6 for binary32 populations (one rounding of each value)."""
import numpy as np
import pytest
import torch

from oracle import vel3d
from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rsl():
    from paper_1612_01287_amd import rsl as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mod


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _states(ncell, seed, beta_max=0.9):
    """(ncell, 5) rows (n, T, u^x, u^y, u^z): directions uniform on the sphere,
    |beta| uniform in [0, beta_max], with a few special rows (rest, +-z, +-x,
    |beta| at beta_max)."""
    rng = inputs.rng(seed)
    n = rng.uniform(0.3, 2.0, ncell)
    T = rng.uniform(0.4, 2.0, ncell)
    d = rng.normal(size=(ncell, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    beta = rng.uniform(0.0, beta_max, ncell)
    special = [np.zeros(3), [0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0], [-0.6, 0.8, 0.0]]
    for i, e in enumerate(special[:ncell]):
        d[i] = e
        beta[i] = 0.0 if i == 0 else (0.5 if i < 4 else beta_max)
    u = d * (beta / np.sqrt(1.0 - beta * beta))[:, None]
    return np.column_stack([n, T, u])


CASES = [(3, 16, 8, 4), (2, 8, 5, 2), (3, 12, 1, 3), (3, 10, 9, 6), (4, 20, 7, 5)]


@pytest.mark.parametrize("QL,Q,Qphi,NOm", CASES)
def test_feq3_matches_oracle(rsl, QL, Q, Qphi, NOm):
    ncell = 203                                   # ragged: not a multiple of 64 or 256
    S = _states(ncell, 17 + Q)
    q3 = rsl.Quadrature3(QL, Q, Qphi, NOm)
    vs = vel3d.VelocitySet3(QL, Q, Qphi, NOm)
    assert q3.V == vs.V
    st = torch.tensor(S, device="cuda")
    f64 = rsl.feq3(q3, st, "f64", pitch=256).cpu().numpy()
    f32 = rsl.feq3(q3, st, "f32", pitch=256).cpu().numpy()
    want = np.stack([vel3d.feq3(vs, *S[c, :2], S[c, 2:]) for c in range(ncell)], axis=1)
    assert _rel(f64[:, :ncell], want) < 1e-12
    assert _rel(f32[:, :ncell], want) < 1e-6
    assert np.all(f64[:, ncell:] == 0.0)          # cells past ncell untouched


@pytest.mark.parametrize("QL,Q,Qphi,NOm", CASES[:3])
def test_moments3_and_landau_match_oracle(rsl, QL, Q, Qphi, NOm):
    """Off-equilibrium populations (the equilibrium of random states times
    1 + 0.2 x noise) uploaded in both precisions: raw moments and the frame
    against the oracle's sums and its 4x4 eigen-solution.  Noise this strong
    on a fast cell can leave T^{mu nu} without a timelike eigenvector (a
    complex pair): there the library must report NaN."""
    ncell = 150
    S = _states(ncell, 5 + Qphi, beta_max=0.85)
    vs = vel3d.VelocitySet3(QL, Q, Qphi, NOm)
    rng = inputs.rng(77)
    F = np.stack([vel3d.feq3(vs, *S[c, :2], S[c, 2:]) for c in range(ncell)], axis=1)
    F *= 1.0 + 0.2 * rng.uniform(-1.0, 1.0, F.shape)
    q3 = rsl.Quadrature3(QL, Q, Qphi, NOm)
    for dt, F_up in (("f64", F), ("f32", F.astype(np.float32))):
        ft = torch.tensor(F_up, device="cuda")
        got = rsl.moments3(q3, ft, ncell).cpu().numpy()
        Fd = np.asarray(F_up, dtype=np.float64)
        N, Tm = vel3d.moments3(vs, Fd)
        iu = np.triu_indices(4)
        raw = np.concatenate([N, Tm[iu[0], iu[1], :]], axis=0).T       # (ncell, 14) in the header's order
        assert _rel(got[:, :14], raw) < 1e-12
        framed = 0
        for c in range(ncell):
            L = vel3d.landau3(N[:, c], Tm[:, :, c])
            if L is None:      # complex eigenvalues: no Landau frame, the library says NaN
                assert np.all(np.isnan(got[c, 14:])), (dt, c)
                continue
            framed += 1
            want = np.array([L["n"], L["E"], L["P"], L["T"], *L["u"]])
            assert _rel(got[c, 14:], want) < 1e-11, (dt, c)
        assert framed >= (ncell - 5 if Qphi >= NOm + 3 else ncell // 2)   # Q_phi = 1 cannot carry u^y


def test_feq3_moments_round_trip_at_full_size(rsl):
    """The bench configuration (2^20 cells, Q_L = 3, Q_xi = 16, Q_phi = 8,
    N_Omega = 4, binary32): every cell's frame recovered from its own
    equilibrium (a property at any size; N_Omega >= 2 and Q_phi >= N_Omega + 3
    keep N^mu and T^{mu nu} exact), and sampled cells against the oracle."""
    ncell = 1 << 20
    S = _states(ncell, 2024, beta_max=0.9)
    q3 = rsl.Quadrature3(3, 16, 8, 4)
    st = torch.tensor(S, device="cuda")
    f = rsl.feq3(q3, st, "f32")
    m = rsl.moments3(q3, f, ncell).cpu().numpy()
    assert np.all(np.isfinite(m))
    assert _rel(m[:, 14], S[:, 0]) < 2e-6
    assert _rel(m[:, 17], S[:, 1]) < 2e-6
    assert np.max(np.abs(m[:, 19:22] - S[:, 2:5])) < 2e-5 * np.max(np.abs(S[:, 2:5]))
    vs = vel3d.VelocitySet3(3, 16, 8, 4)
    fh = f.cpu().numpy()
    for c in inputs.rng(3).choice(ncell, 16, replace=False):
        want = vel3d.feq3(vs, *S[c, :2], S[c, 2:])
        assert _rel(fh[:, c], want) < 1e-6


def test_moments3_flags_states_without_a_frame(rsl):
    q3 = rsl.Quadrature3(3, 8, 5, 2)
    vs = vel3d.VelocitySet3(3, 8, 5, 2)
    F = np.zeros((vs.V, 3))
    F[:, 0] = vel3d.feq3(vs, 1.0, 1.0, np.array([0.1, 0.0, 0.2]))
    # all particles along one direction: T^{mu nu} has no timelike eigenvector
    F[np.argmax(vs.Om[:, 0] * (vs.k == 0)), 1] = 1.0
    F[:, 2] = -F[:, 0]                                                  # negative energy
    got = rsl.moments3(q3, torch.tensor(F, device="cuda"), 3).cpu().numpy()
    assert np.all(np.isfinite(got[0]))
    assert np.all(np.isnan(got[1, 14:])) and np.all(np.isnan(got[2, 14:]))
    assert np.all(np.isfinite(got[1:, :14]))


def test_vel3d_argument_errors(rsl):
    import ctypes
    lib = rsl.lib()
    h = ctypes.c_void_p()
    assert lib.rsl_make_quadrature3(3, 8, 0, 2, 1.0, ctypes.byref(h)) == rsl.RSL_EINVAL
    assert not h.value
    assert lib.rsl_make_quadrature3(3, 8, 4, 7, 1.0, ctypes.byref(h)) == rsl.RSL_EUNSUPPORTED
    q3 = rsl.Quadrature3(3, 8, 4, 3)
    st = torch.zeros((4, 5), dtype=torch.float64, device="cuda")
    f = torch.zeros((q3.V, 4), dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert lib.rsl_feq3(q3.handle, p(st), 4, 0, p(f), 3, s) == rsl.RSL_EINVAL          # pitch < ncell
    assert lib.rsl_feq3(q3.handle, p(st), 4, 7, p(f), 4, s) == rsl.RSL_EINVAL          # dtype
    assert lib.rsl_feq3(q3.handle, None, 4, 0, p(f), 4, s) == rsl.RSL_EINVAL           # null state
    assert lib.rsl_feq3(q3.handle, None, 0, 0, None, 0, s) == rsl.RSL_OK               # empty
    assert lib.rsl_moments3(q3.handle, None, 0, 0, 0, None, s) == rsl.RSL_OK
    assert lib.rsl_moments3(None, p(f), 0, 4, 4, p(st), s) == rsl.RSL_EINVAL
