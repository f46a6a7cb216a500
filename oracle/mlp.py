"""FP64 reference of the learned T^{mu nu} correction (features, MLP, loss,
gradients, Adam) -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The correction is not part of the paper: it maps the local moments of a
low-order velocity set to the difference between the high-order and the
low-order T^{mu nu}.  Its pieces, written out plainly:

* features of cell s: the moments M_{a,r} = sum_jk f_jk p_k^a xi_j^r
  (Sec. III E, eq. momsr in discrete form) for a in {0, 1}, r in 0..7, of the
  cells s-2 .. s+2 (zero-gradient ghosts), the a = 0 ones divided by the centre
  cell's N^0 = M_{0,0}, the a = 1 ones by its T^00 = M_{1,0}; then log tau_r:
  5 * 16 + 1 = 81 inputs;
* network 81 -> 128 -> 128 -> 3, ReLU, linear output;
* target (T_hi - T_lo) / T^00_lo for (T^00, T^0z, T^zz);
* loss: mean over samples and outputs of the squared error;
* Adam (Kingma & Ba) with bias correction.
"""
import numpy as np

N_IN, N_H, N_OUT = 81, 128, 3
R_MAX = 7


def moments_ar(vs, f):
    """M[a, r, s] for a in {0,1}, r in 0..7 of populations f [V, nz] (v = k Q + j)."""
    V, nz = f.shape
    xi = np.tile(vs.xi, vs.QL)
    p = np.repeat(vs.pb * vs.T0, vs.Q)
    M = np.zeros((2, R_MAX + 1, nz))
    for a in range(2):
        for r in range(R_MAX + 1):
            wgt = (p ** a) * (xi ** r)
            M[a, r] = wgt @ f
    return M


def features(vs, f, log_tau):
    """[nz, 81] features of every cell (zero-gradient ghosts at both ends)."""
    M = moments_ar(vs, f)
    nz = f.shape[1]
    idx = np.arange(nz)
    out = np.zeros((nz, N_IN))
    n0 = M[0, 0]
    e0 = M[1, 0]
    col = 0
    for o in range(-2, 3):
        src = np.clip(idx + o, 0, nz - 1)
        for a in range(2):
            norm = n0 if a == 0 else e0
            for r in range(R_MAX + 1):
                out[:, col] = M[a, r, src] / norm
                col += 1
    out[:, col] = log_tau
    return out


def targets(M_lo, M_hi):
    """(T_hi - T_lo)/T^00_lo for (T^00, T^0z, T^zz); M_* are [nz, 13] moment rows."""
    d = M_hi[:, 2:5] - M_lo[:, 2:5]
    return d / M_lo[:, 2:3]


def init_params(seed):
    rng = np.random.default_rng(seed)
    def he(n_in, n_out):
        return rng.standard_normal((n_in, n_out)) * np.sqrt(2.0 / n_in)
    return {"W1": he(N_IN, N_H), "b1": np.zeros(N_H), "W2": he(N_H, N_H), "b2": np.zeros(N_H),
            "W3": he(N_H, N_OUT) * 0.1, "b3": np.zeros(N_OUT)}


def forward(P, X):
    """Returns y and the cache of pre-activations (z1, z2) and activations (h1, h2)."""
    z1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"] + P["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(y, T):
    return float(np.mean((y - T) ** 2))


def backward(P, cache, y, T):
    """Gradients of loss() with respect to every parameter."""
    X, z1, h1, z2, h2 = cache
    n = y.shape[0]
    dy = 2.0 * (y - T) / (n * y.shape[1])
    g = {"W3": h2.T @ dy, "b3": dy.sum(axis=0)}
    dh2 = dy @ P["W3"].T
    dz2 = dh2 * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ P["W2"].T
    dz1 = dh1 * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(P, G, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) in place."""
    for k in P:
        m, v = state.setdefault(k, (np.zeros_like(P[k]), np.zeros_like(P[k])))
        m = b1 * m + (1 - b1) * G[k]
        v = b2 * v + (1 - b2) * G[k] ** 2
        state[k] = (m, v)
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P


# ---------------------------------------------------------------- in-loop feedback
#
# Feeding a correction of the moments back into the populations.  A change of
# (T^00, T^0z, T^zz) is taken in the span of the three population vectors
#     b_c[v] = w_j w_k L^(2)_1(pbar_k) xi_j^c,      c = 0, 1, 2  (v = k Q + j)
# (no N^0, N^z: the Laguerre rule gives sum_k w_k (3 - pbar_k) = 0), a change
# of (N^0, N^z) in the span of
#     b'_c[v] = w_j w_k (4 - pbar_k) xi_j^c,        c = 0, 1
# (no T^{mu nu}: sum_k w_k pbar_k (4 - pbar_k) = 0).  The coefficients solve
# the moment equations written out as a 5 x 5 system (rows N^0, N^z, T^00,
# T^0z, T^zz of each vector) by least squares.

def _basis(vs):
    xi = np.tile(vs.xi, vs.QL)
    w = np.outer(vs.wL, vs.wxi).ravel()
    L1 = np.repeat(3.0 - vs.pb, vs.Q)
    G0 = np.repeat(4.0 - vs.pb, vs.Q)
    return np.stack([w * L1 * xi ** c for c in range(3)] + [w * G0 * xi ** c for c in range(2)], axis=1)


def _moment_rows(vs):
    """(5, V): N^0, N^z, T^00, T^0z, T^zz weights of each population."""
    xi = np.tile(vs.xi, vs.QL)
    p = np.repeat(vs.pb * vs.T0, vs.Q)
    return np.stack([np.ones_like(xi), xi, p, p * xi, p * xi * xi])


def inject(vs, f, dT, dN=None):
    """f + df with moments(df) = (dN, dT) per cell (dN = 0 if None); f [V, nz],
    dT [nz, 3], dN [nz, 2]."""
    nz = dT.shape[0]
    B = _basis(vs)
    A = _moment_rows(vs) @ B                                                # (5, 5)
    dN = np.zeros((nz, 2)) if dN is None else np.asarray(dN, dtype=np.float64)
    rhs = np.concatenate([dN.T, np.asarray(dT, dtype=np.float64).T])
    coef, *_ = np.linalg.lstsq(A, rhs, rcond=None)                          # (5, nz)
    return np.asarray(f, dtype=np.float64) + B @ coef


def project(vs_hi, f_hi, vs_lo):
    """Low-order populations with the N^mu and T^{mu nu} of f_hi [V_hi, nz]:
    the low-order equilibrium of f_hi's Landau frame plus the change that
    carries the rest of both."""
    from . import feq, landau
    R_hi, R_lo = _moment_rows(vs_hi), _moment_rows(vs_lo)
    M = R_hi @ np.asarray(f_hi, dtype=np.float64)                           # (5, nz)
    nz = M.shape[1]
    out = np.zeros((vs_lo.V, nz))
    for s in range(nz):
        L = landau(M[:, s])
        out[:, s] = feq(vs_lo, L["n"], L["T"], L["beta"])
    D = M - R_lo @ out
    return inject(vs_lo, out, D[2:].T, D[:2].T)
