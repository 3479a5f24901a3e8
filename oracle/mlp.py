"""FP64 reference of the learned interface closure (test infrastructure).

A 10 -> 64 -> 64 -> 8 perceptron (tanh after the two hidden layers, linear
output), its loss, analytic backward pass and Adam update, and the
features / targets it is trained on.  Only tests and the benchmark's CPU leg
use this module.

Closure (the lift of Sec. 2.2 in moment form): when low-order populations
are lifted to the high-order set, the non-equilibrium Hermite coefficients
the low set cannot carry are unknown; the network predicts the six of total
order 3 and 4 that a tensor-product D2Q9 lacks -- (3,0), (0,3), (3,1), (1,3),
(4,0), (0,4) -- and two logits of a region flag (does the node's
non-equilibrium indicator exceed the threshold).

Inputs (node-local, from the low-order populations): rho - 1, ux, uy,
log Kn_loc and the non-equilibrium coefficients a_km - rho ux^k uy^m
(k + m <= 2; the 2nd-order equilibrium has no higher components) for
(2,0), (1,1), (0,2), (2,1), (1,2), (2,2), each divided by rho.  Inputs and
regression targets are standardised with dataset means and deviations.

Parameter vector layout (5384 values): W1[64][10], b1[64], W2[64][64],
b2[64], W3[8][64], b3[8].
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 10, 64, 8
NREG = 6
MISSING = ((3, 0), (0, 3), (3, 1), (1, 3), (4, 0), (0, 4))
FEATURE_NEQ = ((2, 0), (1, 1), (0, 2), (2, 1), (1, 2), (2, 2))
SIZES = [(NH, NIN), (NH,), (NH, NH), (NH,), (NOUT, NH), (NOUT,)]
NPARAM = sum(int(np.prod(s)) for s in SIZES)


def unpack(p):
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def init(uniforms):
    """Xavier-uniform weights from given U(-1, 1) draws (len NPARAM); zero biases."""
    u = np.asarray(uniforms, dtype=np.float64)
    p = np.zeros(NPARAM)
    o = 0
    for s in SIZES:
        n = int(np.prod(s))
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            p[o:o + n] = lim * u[o:o + n]
        o += n
    return p


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64))
    H1 = np.tanh(X @ W1.T + b1)
    H2 = np.tanh(H1 @ W2.T + b2)
    return H2 @ W3.T + b3, (H1, H2)


def loss_grad(p, X, T, flag):
    """Mean over the batch of: mean squared error of the 6 regression outputs
    + cross-entropy of the 2 flag logits.  Returns (loss, gradient)."""
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, dtype=np.float64))
    Y, (H1, H2) = forward(p, X)
    r = Y[:, :NREG] - T
    z = Y[:, NREG:]
    zm = z - z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(zm).sum(axis=1))
    logp = zm - lse[:, None]
    onehot = np.zeros_like(z)
    onehot[np.arange(B), flag] = 1.0
    loss = np.mean(np.sum(r * r, axis=1) / NREG - np.sum(onehot * logp, axis=1))
    dY = np.zeros_like(Y)
    dY[:, :NREG] = 2.0 * r / NREG / B
    dY[:, NREG:] = (np.exp(logp) - onehot) / B
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * (1.0 - H2 * H2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (1.0 - H1 * H1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return loss, g


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(oracle, f9, kn_loc):
    """Raw (unstandardised) inputs of one D2Q9 node (absolute populations)."""
    a = oracle.hermite_coeffs(3, f9)
    rho = a[0, 0]
    ux, uy = a[1, 0] / rho, a[0, 1] / rho
    x = [rho - 1.0, ux, uy, np.log(kn_loc)]
    for k, m in FEATURE_NEQ:
        eq = rho * ux ** k * uy ** m if k + m <= 2 else 0.0
        x.append((a[k, m] - eq) / rho)
    return np.array(x)


def targets(oracle, f36, eq_order=4):
    """Raw regression targets of one D2Q36 node: the missing non-equilibrium
    coefficients (a_km - rho ux^k uy^m) / rho."""
    a = oracle.hermite_coeffs(6, f36)
    rho = a[0, 0]
    ux, uy = a[1, 0] / rho, a[0, 1] / rho
    out = []
    for k, m in MISSING:
        eq = rho * ux ** k * uy ** m if k + m <= eq_order else 0.0
        out.append((a[k, m] - eq) / rho)
    return np.array(out)


def closure_coeffs(y_reg, t_mean, t_std, rho, nd=6):
    """Closure coefficients (nd*nd, row k*nd + m) from the standardised
    regression outputs of one node: C_km = rho (mean + std * y)."""
    c = np.zeros(nd * nd)
    for idx, (k, m) in enumerate(MISSING):
        c[k * nd + m] = rho * (t_mean[idx] + t_std[idx] * y_reg[idx])
    return c
