"""Seeded synthetic inputs shared by the oracle and the HIP path in the tests.

Holds no arithmetic of the method: only parameter sets and random arrays drawn
from numpy's PCG64 generator with fixed seeds."""
import numpy as np

# Sod states used throughout: the C1/C2 shock tube ((T, n)_L = (1, 1),
# (T, n)_R = (0.8, 0.4)) and the paper's own right state (T = 0.5, n = 0.125).
SOD_C1 = dict(nL=1.0, TL=1.0, nR=0.4, TR=0.8)
SOD_PAPER = dict(nL=1.0, TL=1.0, nR=0.125, TR=0.5)


def positive_populations(V, nz, seed, weights=None, lo=0.2, hi=1.0):
    """Random positive populations [V, nz], optionally scaled per velocity by
    `weights` (e.g. w_j w_k) so that they resemble a distribution."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(lo, hi, size=(V, nz))
    if weights is not None:
        f = f * np.asarray(weights, dtype=np.float64)[:, None]
    return f


def smooth_perturbation(V, nz, seed, amp=0.05):
    """1 + amp * (random Fourier modes along z), per velocity, shape [V, nz]."""
    rng = np.random.default_rng(seed)
    z = (np.arange(nz) + 0.5) / nz
    out = np.ones((V, nz))
    for m in range(1, 4):
        a = rng.uniform(-1, 1, size=(V, 1))
        ph = rng.uniform(0, 2 * np.pi, size=(V, 1))
        out += amp * a * np.sin(2 * np.pi * m * z[None, :] + ph) / m
    return out


def rng(seed):
    """The seeded generator every synthetic input of the tests draws from."""
    return np.random.default_rng(seed)
