"""Convergence harness of the paper's quadrature-order studies, on the batched
solver and the device diagnostics.

* Sod (Sec. IV E, eqs. eps_def, eps_th; Table III): for one eta/s, every
  R-SLB(N_Omega; Q_xi) of a list and the reference model run together in one
  batch (same grid, time step and initial state) to t_end; the error
  eps = max over n, T, gamma of max_z |d - d_ref| / (max d - min d) per model
  (rsl_sod_eps), and the smallest Q_xi from which every larger model of the
  list stays below the threshold.
* Bjorken (Sec. V E, eq. bjork_L2; Table IV): the models and the reference run
  together from tau = 1 to tau_f; the moments of every instance are sampled on
  the device every `sample_every` steps, and the L2 norm of n, T, P, Pi against
  the reference follows from rsl_bjorken_l2.

Orchestration only: stepping, moments and error measures run in librsl.
"""
import math

import torch

from . import rsl

HBARC = 0.1973269804          # GeV fm
PAPER_SOD = dict(nL=1.0, TL=1.0, nR=0.125, TR=0.5)     # eq. Sod:right_adim


def sod_convergence(eta_s, qxis, ref=(500, 6), QL=2, nz=1000, t_end=0.5, dt=5e-4, nom=lambda Q: min(Q - 1, 5),
                    eps_th=0.01, T_ref_GeV=0.4, L_ref_fm=6.4, states=PAPER_SOD, stream=None):
    """eps of each R-SLB(nom(Q); Q) in qxis against R-SLB(ref[1]; ref[0]) at
    t_end, with tau_AW from eq. Sod:tau (lambda_ref = 1).  The common time
    step is dt, or smaller when the stiffness guard of the reference problem
    asks for it.  Returns (dict Q -> eps tuple, Q_conv or None, dt used)."""
    taw0 = 5 * HBARC * eta_s / (T_ref_GeV * L_ref_fm)
    models = [(Q, nom(Q)) for Q in qxis] + [(ref[0], ref[1])]
    quads = [rsl.Quadrature(QL, Q, no) for Q, no in models]
    probs = [rsl.make_problem(nz=nz, bc="eq", tau_mode="etas", tau_aw0=taw0, **states) for _ in models]
    cfl, stiff = rsl.max_dt(quads[-1], probs[-1])
    dt = min(dt, stiff, 0.999 * cfl)
    nsteps = int(math.ceil(t_end / dt - 1e-9))
    dt = t_end / nsteps
    B = rsl.Batch(quads, probs, [dt] * len(models))
    B.init(stream=stream)
    B.step(nsteps, stream=stream)
    M = B.moments(stream=stream)
    ref_rows = M[len(qxis) * nz:]
    eps = {}
    for i, (Q, _) in enumerate(models[:-1]):
        eps[Q] = tuple(rsl.sod_eps(M[i * nz:(i + 1) * nz], ref_rows, stream=stream).tolist())
    qconv = None
    for Q in sorted(qxis, reverse=True):
        if eps[Q][3] < eps_th:
            qconv = Q
        else:
            break
    return eps, qconv, dt


def bjorken_convergence(eta_s, qxis, T0_GeV=0.3, gas="parton", ref=(100, 5), QL=2, tau_f=40.0, dtau=1e-3,
                        sample_every=100, nom=lambda Q: min(Q - 1, 5), stream=None):
    """L2 norms (eq. bjork_L2) of each R-SLB(nom(Q); Q) in qxis against the
    reference R-SLB(ref[1]; ref[0]) from tau = 1 to tau_f; tau_AW from eq.
    bjorken_tauAW (tau0 = 0.25 fm).  Returns dict Q -> (L2(n), L2(T), L2(P),
    L2(Pi), max)."""
    taw0 = 5 * HBARC * eta_s / (0.25 * T0_GeV)
    models = [(Q, nom(Q)) for Q in qxis] + [(ref[0], ref[1])]
    quads = [rsl.Quadrature(QL, Q, no) for Q, no in models]
    probs = [rsl.make_problem(kind="bjorken", gas=gas, tau_mode="etas", tau_aw0=taw0) for _ in models]
    B = rsl.Batch(quads, probs, [dtau] * len(models))
    nsteps = int(round((tau_f - 1.0) / dtau))
    nsamp = nsteps // sample_every + 1
    hist = torch.empty((len(models), nsamp, rsl.RSL_MOM_ALL), dtype=torch.float64, device=B.f_buf.device)
    B.init(stream=stream)
    hist[:, 0] = B.moments(stream=stream)
    for s in range(1, nsamp):
        B.step(sample_every, stream=stream)
        hist[:, s] = B.moments(stream=stream)
    out = {}
    for i, (Q, _) in enumerate(models[:-1]):
        out[Q] = tuple(rsl.bjorken_l2(hist[i].contiguous(), hist[-1].contiguous(), dtau * sample_every,
                                      stream=stream).tolist())
    return out, hist
