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
        for Q in dict.fromkeys((q_lo, q_hi)):
            probs = [rsl.make_problem(nz=nz, dtype=dtype, bc="outflow", tau_r=tau, nL=1.0, TL=1.0, nR=nR, TR=TR)
                     for (TR, nR, tau) in states]
            B = rsl.Batch([self.quads[Q]] * len(states), probs, [self.dt] * len(states))
            B.init()
            self.batches[Q] = B

    def advance(self, nsteps, which=None, stream=None):
        for Q in ((self.q_lo, self.q_hi) if which is None else (which,)):
            self.batches[Q].step(nsteps, stream=stream)

    def features(self, shift=None, scale=None):
        B = self.batches[self.q_lo]
        feats = [rsl.features(self.quads[self.q_lo], B.problems[i], B.f(i), math.log(self.states[i][2]),
                              shift, scale) for i in range(B.n)]
        return torch.cat(feats, dim=0)

    def moments(self, Q):
        return self.batches[Q].moments()


def generate(n_runs, nz, t_snaps, seed, tau_range=(0.01, 1.0), q_lo=8, q_hi=128, dtype="f32", progress=None,
             chunk=None):
    """Features X [N, 81] and targets T [N, 3] from paired runs (on the GPU).
    With `chunk`, the runs are generated `chunk` at a time (bounded memory);
    `progress(msg)` is called after every snapshot."""
    rng = np.random.default_rng(seed)
    states = _states(rng, n_runs, *tau_range)
    chunk = chunk or n_runs
    X, T = [], []
    for c0 in range(0, n_runs, chunk):
        ens = PairedEnsemble(states[c0:c0 + chunk], nz, q_lo, q_hi, dtype)
        done = 0
        for ts in t_snaps:
            k = int(round(ts / ens.dt)) - done
            ens.advance(k)
            done += k
            X.append(ens.features())
            T.append(rsl.tmunu_targets(ens.moments(q_lo), ens.moments(q_hi)))
            if progress:
                torch.cuda.synchronize()
                progress("runs %d-%d: snapshot t = %.3g" % (c0, min(n_runs, c0 + chunk) - 1, ts))
        del ens
    return torch.cat(X), torch.cat(T)


class Correction:
    """A trained network, the feature standardisation it expects and the range
    of standardised features it was trained on (the guard)."""

    def __init__(self, net, lo, hi, shift, scale):
        self.net, self.lo, self.hi = net, lo, hi
        self.shift, self.scale = shift, scale

    def features(self, ens):
        """Standardised features of an ensemble's low-order states (one kernel per instance)."""
        return ens.features(self.shift, self.scale)

    def apply(self, X, m_lo):
        """Corrected (T^00, T^0z, T^zz) [N, 3] (fp64) from standardised features,
        or None when a feature lies outside the training range (caller falls
        back to the high-order solve)."""
        if rsl.guard(X, self.lo, self.hi):
            return None
        y = self.net.forward(X)
        return rsl.tmunu_correct(m_lo, y)

    def outside(self, X):
        """Indices of the features that leave the training range somewhere in X."""
        out = ((X < self.lo) | (X > self.hi)).any(dim=0)
        return [int(i) for i in torch.nonzero(out).flatten().tolist()]


def train(X, T, epochs=20, batch=8192, lr=2e-3, seed=0, margin=0.05, init=None, min_scale=1e-4, progress=None):
    """Adam on shuffled minibatches with a cosine learning-rate decay.

    Inputs are standardised per feature (mean, standard deviation floored at
    min_scale; the features kernel applies the same map at inference) and the
    targets are divided by their root mean square per output during training;
    that factor is folded into the last layer afterwards, so the returned
    network maps standardised features to the unscaled targets.  Returns the
    Correction and the per-epoch mean loss in the scaled units."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    shift = X.mean(dim=0).contiguous()
    scale = X.std(dim=0).clamp_min(min_scale).contiguous()
    Xs = ((X - shift) / scale).contiguous()
    tsc = T.pow(2).mean(dim=0).sqrt().clamp_min(1e-30)
    Ts = (T / tsc).contiguous()
    net = rsl.MLP(init if init is not None else _he_init(seed))
    hist = []
    step = 0
    nb = (n + batch - 1) // batch
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        tot = torch.zeros((), dtype=torch.float64, device=X.device)   # summed on the device: no sync per batch
        cnt = 0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            xb, tb = Xs[idx].contiguous(), Ts[idx].contiguous()
            y, h1, h2 = net.forward(xb, keep=True)
            net.backward(xb, h1, h2, y, tb)
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * step / max(1, epochs * nb)))
            net.adam(lr=lr_t)
            step += 1
            tot += ((y - tb) ** 2).mean().double() * xb.shape[0]
            cnt += xb.shape[0]
        hist.append(float(tot) / cnt)
        if progress and (ep % 10 == 9 or ep == epochs - 1):
            progress("epoch %d: loss %.4g" % (ep + 1, hist[-1]))
    _fold_output_scale(net, tsc)
    span = Xs.max(dim=0).values - Xs.min(dim=0).values
    lo = (Xs.min(dim=0).values - margin * span - 1e-6).contiguous()
    hi = (Xs.max(dim=0).values + margin * span + 1e-6).contiguous()
    return Correction(net, lo, hi, shift, scale), hist


def _fold_output_scale(net, tsc):
    """W3 <- W3 diag(tsc), b3 <- b3 tsc on the fp32 master copy, then a fresh bf16 copy."""
    o = 0
    for name, shp in rsl.MLP_SHAPES:
        k = int(np.prod(shp))
        if name == "W3":
            net.params[o:o + k].view(shp).mul_(tsc.to(net.params.dtype))
        elif name == "b3":
            net.params[o:o + k].mul_(tsc.to(net.params.dtype))
        o += k
    net.refresh()


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


def evaluate(corr, n_inst, nz, t_end, seed, tau_range=(0.01, 1.0), q_lo=8, q_hi=128, dtype="f32", tune=True,
             progress=None):
    """Errors of T_lo and of the corrected T_lo against T_hi, and wall times of
    (low-order solve + features + network + correction) vs the high-order solve.
    When the guard rejects the features, the corrected path's answer is the
    high-order solve, and its wall time includes that solve.
    With `tune`, both batches first pick their stage-kernel shapes with the
    autotuner (which restores the state it times on), so that neither solve
    runs on untuned defaults."""
    rng = np.random.default_rng(seed)
    ens = PairedEnsemble(_states(rng, n_inst, *tau_range), nz, q_lo, q_hi, dtype)
    nsteps = int(round(t_end / ens.dt))
    stream = torch.cuda.current_stream()
    if tune:
        for Q in (q_lo, q_hi):
            ens.batches[Q].autotune(reps=2, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.advance(nsteps, which=q_lo, stream=stream)
    X = corr.features(ens)
    m_lo = ens.moments(q_lo)
    Tc = corr.apply(X, m_lo)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    if progress:
        progress("low-order solve and correction: %.2f s" % t_learned)
    t0 = time.perf_counter()
    ens.advance(nsteps, which=q_hi, stream=stream)
    m_hi = ens.moments(q_hi)
    torch.cuda.synchronize()
    t_hi = time.perf_counter() - t0
    Thi = m_hi[:, 2:5]
    Tlo = m_lo[:, 2:5]
    def rel(a):
        return float(torch.linalg.norm(a - Thi) / torch.linalg.norm(Thi))
    if Tc is None:
        t_learned += t_hi              # the fallback is the plain high-order solve
    out = {"err_lo": rel(Tlo), "t_learned_s": t_learned, "t_high_order_s": t_hi,
           "fallback": Tc is None, "cells": int(Thi.shape[0])}
    if Tc is None:
        out["features_outside"] = corr.outside(X)
    out["err_corrected"] = rel(Tc) if Tc is not None else None
    return out


# ------------------------------------------------------------ in-loop feedback
#
# The correction fed back through f instead of applied to the output: every
# `interval` of time the low-order state's features give the network's
# (T_hi - T_lo) / T^00_lo, and rsl_mlp_inject moves the state's T^00, T^0z,
# T^zz by that much (N^mu unchanged).  Training pairs come from the same loop
# with the true defect in place of the network's (teacher forcing): both sets
# advance one interval, the pair is (features of the low-order state, the
# high-order minus low-order T^{mu nu}), and that defect is injected into the
# low-order state before the next interval, so the training states are the
# corrected low-order states inference meets.

def _inject_all(ens, y, stream=None):
    Bl, ql = ens.batches[ens.q_lo], ens.quads[ens.q_lo]
    nz = ens.nz
    for i in range(Bl.n):
        rsl.inject(ql, Bl.problems[i], Bl.f(i), y[i * nz:(i + 1) * nz].contiguous(), stream=stream)


def generate_inloop(n_runs, nz, interval, n_intervals, seed, tau_range=(0.01, 1.0), q_lo=8, q_hi=128, dtype="f32",
                    progress=None, chunk=None):
    """Features X [N, 81] of the teacher-forced low-order states at the end of
    each interval and the defects T [N, 3] there."""
    rng = np.random.default_rng(seed)
    states = _states(rng, n_runs, *tau_range)
    chunk = chunk or n_runs
    X, T = [], []
    for c0 in range(0, n_runs, chunk):
        ens = PairedEnsemble(states[c0:c0 + chunk], nz, q_lo, q_hi, dtype)
        k = int(round(interval / ens.dt))
        for it in range(n_intervals):
            ens.advance(k)
            X.append(ens.features())
            T.append(rsl.tmunu_targets(ens.moments(q_lo), ens.moments(q_hi)))
            if it + 1 < n_intervals:
                _inject_all(ens, T[-1])
            if progress:
                torch.cuda.synchronize()
                progress("runs %d-%d: interval %d of %d" % (c0, min(n_runs, c0 + chunk) - 1, it + 1, n_intervals))
        del ens
    return torch.cat(X), torch.cat(T)


def evaluate_inloop(corr, n_inst, nz, interval, n_intervals, seed, tau_range=(0.01, 1.0), q_lo=8, q_hi=128,
                    dtype="f32", tune=True, progress=None):
    """Relative T^{mu nu} errors at t_end = n_intervals * interval of the plain
    low-order solve and of the low-order solve with the correction injected
    after every interval, against the high-order solve; wall times of the
    corrected low-order path and of the high-order solve.  If the guard rejects
    the features at some interval, the corrected path falls back to the
    high-order solve (its time included)."""
    rng = np.random.default_rng(seed)
    states = _states(rng, n_inst, *tau_range)
    ens = PairedEnsemble(states, nz, q_lo, q_hi, dtype)
    plain = PairedEnsemble(states, nz, q_lo, q_lo, dtype)        # a second low-order copy, never corrected
    k = int(round(interval / ens.dt))
    stream = torch.cuda.current_stream()
    if tune:
        for Q in (q_lo, q_hi):
            ens.batches[Q].autotune(reps=2, stream=stream)
        plain.batches[q_lo].autotune(reps=2, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fallback = False
    for it in range(n_intervals):
        ens.advance(k, which=q_lo, stream=stream)
        X = corr.features(ens)
        if rsl.guard(X, corr.lo, corr.hi):
            fallback = True
            break
        _inject_all(ens, corr.net.forward(X), stream=stream)
    m_lo = ens.moments(q_lo)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    if progress:
        progress("in-loop corrected low-order solve: %.2f s" % t_learned)
    t0 = time.perf_counter()
    ens.advance(k * n_intervals, which=q_hi, stream=stream)
    m_hi = ens.moments(q_hi)
    torch.cuda.synchronize()
    t_hi = time.perf_counter() - t0
    plain.advance(k * n_intervals, which=q_lo, stream=stream)
    m_plain = plain.moments(q_lo)
    Thi = m_hi[:, 2:5]

    def rel(a):
        return float(torch.linalg.norm(a - Thi) / torch.linalg.norm(Thi))
    if fallback:
        t_learned += t_hi
    return {"err_lo": rel(m_plain[:, 2:5]), "err_inloop": None if fallback else rel(m_lo[:, 2:5]),
            "t_learned_s": t_learned, "t_high_order_s": t_hi, "fallback": fallback, "cells": int(Thi.shape[0])}
