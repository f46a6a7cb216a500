"""Learned T^{mu nu} correction for a low-order velocity set: data generation
with the high-order solver, training with the library's own forward/backward/
Adam kernels, evaluation against the plain high-order solve.

Orchestration only: every solver step, feature, network pass, gradient,
optimiser update and correction runs in librsl's kernels (rsl.py binding).

The workload: Sod tubes with (T, n)_L = (1, 1), T_R = T_L / r (r uniform in
[1.1, 3]), n_R = T_R^3, at rest, zero-gradient ghosts, tau_r log-uniform in
[tau_min, tau_max]; the low-order set is R-SLB(min(Q_lo - 1, 4); Q_lo) with
Q_L = 3, the high-order one R-SLB(4; Q_hi).  Targets are
(T_hi - T_lo) / T^00_lo for (T^00, T^0z, T^zz) in every cell of snapshots.
"""
import math
import time

import numpy as np
import torch

from . import rsl

QL = 3


def _states(rng, n, tau_lo, tau_hi):
    out = []
    for _ in range(n):
        r = rng.uniform(1.1, 3.0)
        TR = 1.0 / r
        tau = math.exp(rng.uniform(math.log(tau_lo), math.log(tau_hi)))
        out.append((TR, TR ** 3, tau))
    return out


class PairedEnsemble:
    """Two batches (low- and high-order velocity sets) on identical initial states."""

    def __init__(self, states, nz, q_lo=8, q_hi=128, dtype="f32"):
        self.nz, self.states = nz, states
        self.quads = {Q: rsl.Quadrature(QL, Q, min(Q - 1, 4)) for Q in (q_lo, q_hi)}
        self.q_lo, self.q_hi = q_lo, q_hi
        self.dt = 0.5 / nz
        self.batches = {}
        for Q in (q_lo, q_hi):
            probs = [rsl.make_problem(nz=nz, dtype=dtype, bc="outflow", tau_r=tau, nL=1.0, TL=1.0, nR=nR, TR=TR,
                                      kappa=1e9) for (TR, nR, tau) in states]
            B = rsl.Batch([self.quads[Q]] * len(states), probs, [self.dt] * len(states))
            B.init()
            self.batches[Q] = B

    def advance(self, nsteps, which=None, stream=None):
        for Q in ((self.q_lo, self.q_hi) if which is None else (which,)):
            self.batches[Q].step(nsteps, stream=stream)

    def features(self):
        B = self.batches[self.q_lo]
        feats = [rsl.features(self.quads[self.q_lo], B.problems[i], B.f(i), math.log(self.states[i][2]))
                 for i in range(B.n)]
        return torch.cat(feats, dim=0)

    def moments(self, Q):
        return self.batches[Q].moments()


def generate(n_runs, nz, t_snaps, seed, tau_range=(0.01, 1.0), q_lo=8, q_hi=128, dtype="f32"):
    """Features X [N, 81] and targets T [N, 3] from paired runs (on the GPU)."""
    rng = np.random.default_rng(seed)
    ens = PairedEnsemble(_states(rng, n_runs, *tau_range), nz, q_lo, q_hi, dtype)
    X, T = [], []
    done = 0
    for ts in t_snaps:
        k = int(round(ts / ens.dt)) - done
        ens.advance(k)
        done += k
        X.append(ens.features())
        T.append(rsl.tmunu_targets(ens.moments(q_lo), ens.moments(q_hi)))
    return torch.cat(X), torch.cat(T)


class Correction:
    """A trained network plus the feature range it was trained on (the guard)."""

    def __init__(self, net, lo, hi):
        self.net, self.lo, self.hi = net, lo, hi

    def apply(self, X, m_lo):
        """Corrected (T^00, T^0z, T^zz) [N, 3] (fp64), or None when a feature
        lies outside the training range (caller falls back to the high-order solve)."""
        if rsl.guard(X, self.lo, self.hi):
            return None
        y = self.net.forward(X)
        return rsl.tmunu_correct(m_lo, y)


def train(X, T, epochs=20, batch=8192, lr=2e-3, seed=0, margin=0.05, init=None):
    """Adam on shuffled minibatches with a cosine learning-rate decay; returns
    the Correction (network + feature range for the guard) and the per-epoch
    mean loss."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    net = rsl.MLP(init if init is not None else _he_init(seed))
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        tot, cnt = 0.0, 0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            xb, tb = X[idx].contiguous(), T[idx].contiguous()
            y, h1, h2 = net.forward(xb, keep=True)
            net.backward(xb, h1, h2, y, tb)
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * step / max(1, epochs * ((n + batch - 1) // batch))))
            net.adam(lr=lr_t)
            step += 1
            tot += float(((y - tb) ** 2).mean()) * xb.shape[0]
            cnt += xb.shape[0]
        hist.append(tot / cnt)
    span = X.max(dim=0).values - X.min(dim=0).values
    lo = (X.min(dim=0).values - margin * span - 1e-6).contiguous()
    hi = (X.max(dim=0).values + margin * span + 1e-6).contiguous()
    return Correction(net, lo, hi), hist


def _he_init(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in rsl.MLP_SHAPES:
        if name.startswith("W"):
            w = rng.standard_normal(shp) * math.sqrt(2.0 / shp[0])
            if name == "W3":
                w *= 0.1
            parts.append(w.ravel())
        else:
            parts.append(np.zeros(shp).ravel())
    return np.concatenate(parts)


def evaluate(corr, n_inst, nz, t_end, seed, tau_range=(0.01, 1.0), q_lo=8, q_hi=128, dtype="f32"):
    """Errors of T_lo and of the corrected T_lo against T_hi, and wall times of
    (low-order solve + features + network + correction) vs the high-order solve."""
    rng = np.random.default_rng(seed)
    ens = PairedEnsemble(_states(rng, n_inst, *tau_range), nz, q_lo, q_hi, dtype)
    nsteps = int(round(t_end / ens.dt))
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.advance(nsteps, which=q_lo, stream=stream)
    X = ens.features()
    m_lo = ens.moments(q_lo)
    Tc = corr.apply(X, m_lo)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    t0 = time.perf_counter()
    ens.advance(nsteps, which=q_hi, stream=stream)
    m_hi = ens.moments(q_hi)
    torch.cuda.synchronize()
    t_hi = time.perf_counter() - t0
    Thi = m_hi[:, 2:5]
    Tlo = m_lo[:, 2:5]
    def rel(a):
        return float(torch.linalg.norm(a - Thi) / torch.linalg.norm(Thi))
    out = {"err_lo": rel(Tlo), "t_learned_s": t_learned, "t_high_order_s": t_hi,
           "fallback": Tc is None, "cells": int(Thi.shape[0])}
    out["err_corrected"] = rel(Tc) if Tc is not None else None
    return out
