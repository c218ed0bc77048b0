"""Translation-symmetric single-layer network with ELU activation, in float64:
the ground-state ansatz of the paper's example (Sec. 5.1, eq:gs_nqs).

Test infrastructure only: this module checks the HIP library and is never
called by it.

For a ring of L sites with spins sigma_l = 2 s_l - 1 and alpha filters,
    theta_{a,w} = b_a + sum_l W_{a,l} sigma_{(l + w) mod L},   w = 0 .. L-1,
    log psi(s)  = sum_a sum_w ELU(theta_{a,w}),
    ELU(x) = x (x > 0),  e^x - 1 (x <= 0).
Real parameters in the order [W (alpha x L, row-major), b (alpha)],
K = alpha (L + 1).  Readings: sigma in {-1, +1} from the bit encoding (bit 1 =
+1); the translation omega(l) = (l + w) mod L.
Log-derivatives: with g_{a,w} = ELU'(theta_{a,w}) = 1 (theta > 0) or e^theta,
    d/dW_{a,l} = sum_w g_{a,w} sigma_{(l + w) mod L},   d/db_a = sum_w g_{a,w}.
"""
from __future__ import annotations

import numpy as np


def elu(x):
    return np.where(x > 0, x, np.expm1(np.minimum(x, 0.0)))


def split(theta, L, alpha):
    p = np.asarray(theta).real.astype(np.float64)
    return p[: alpha * L].reshape(alpha, L), p[alpha * L:]


def pre_activations(theta, x, L, alpha):
    """(B, alpha, L) theta_{a,w} for the (B, L) 0/1 rows of x."""
    W, b = split(theta, L, alpha)
    sig = 2.0 * np.atleast_2d(x).astype(np.float64) - 1.0
    out = np.empty((sig.shape[0], alpha, L))
    for w in range(L):
        shifted = np.roll(sig, -w, axis=1)        # shifted[:, l] = sigma[(l + w) mod L]
        out[:, :, w] = shifted @ W.T + b
    return out


def log_psi(theta, x, L, alpha):
    return elu(pre_activations(theta, x, L, alpha)).sum(axis=(1, 2))


def grad_log_psi(theta, x, L, alpha):
    """(B, K) log-derivatives in parameter order."""
    t = pre_activations(theta, x, L, alpha)
    g = np.where(t > 0, 1.0, np.exp(np.minimum(t, 0.0)))   # ELU'
    sig = 2.0 * np.atleast_2d(x).astype(np.float64) - 1.0
    B = sig.shape[0]
    dW = np.zeros((B, alpha, L))
    for w in range(L):
        shifted = np.roll(sig, -w, axis=1)
        dW += g[:, :, w][:, :, None] * shifted[:, None, :]
    db = g.sum(axis=2)
    return np.concatenate([dW.reshape(B, -1), db], axis=1)
