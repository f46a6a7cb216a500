"""End-to-end learned correction on the GPU: paired low/high-order Sod data from
the solver, training with the library's own forward/backward/Adam kernels, and
the gain over the uncorrected low-order set on unseen instances (scaled-down
version of the 8192-cell, 512-instance evaluation)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_learned_correction_gain():
    from paper_1612_01287_amd import learned
    X, T = learned.generate(n_runs=16, nz=512, t_snaps=(0.1, 0.175, 0.25), seed=5, q_lo=8, q_hi=64)
    assert X.shape == (16 * 512 * 3, 81) and torch.isfinite(X).all() and torch.isfinite(T).all()
    corr, hist = learned.train(X, T, epochs=40, batch=2048, lr=3e-3, seed=1, margin=0.25)
    assert hist[-1] < 0.3 * hist[0]
    # unseen instances drawn from inside the training distribution
    res = learned.evaluate(corr, n_inst=4, nz=512, t_end=0.25, seed=6, tau_range=(0.03, 0.3), q_lo=8, q_hi=64)
    print(res)
    if res["fallback"]:
        pytest.skip("evaluation features left the training range: fallback to the high-order solve (%s)" % res)
    assert res["err_corrected"] < 0.7 * res["err_lo"], res


def test_guard_triggers_fallback():
    from paper_1612_01287_amd import learned, rsl
    X = torch.zeros((10, 81), device="cuda")
    lo = torch.full((81,), -1.0, device="cuda")
    hi = torch.full((81,), 1.0, device="cuda")
    assert not rsl.guard(X, lo, hi)
    X[3, 7] = 5.0
    assert rsl.guard(X, lo, hi)
    corr = learned.Correction(rsl.MLP(), lo, hi, torch.zeros(81, device="cuda"), torch.ones(81, device="cuda"))
    assert corr.apply(X, torch.zeros((10, 13), dtype=torch.float64, device="cuda")) is None
