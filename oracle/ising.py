"""Exact results for the square-lattice Ising model on a periodic torus, used
to pin the learned-proposal state.

Test infrastructure only: this module checks the HIP library and is never
called by it.

The bond-RBM state (one hidden unit per bond, W_bi = W_bj = w, all other
parameters 0) has |psi(s)|^2 proportional to prod_b exp(K s_i s_j) with
K = ln cosh(2 w), the Boltzmann weight of the classical Ising model.  The
finite-torus partition function is Kaufman's (B. Kaufman, Phys. Rev. 76, 1232
(1949)): for m rows and n columns,
    Z = (1/2) (2 sinh 2K)^(mn/2) (Z1 + Z2 + Z3 + Z4),
    Z1 = prod_r 2 cosh(m g_(2r+1) / 2),   Z2 = prod_r 2 sinh(m g_(2r+1) / 2),
    Z3 = prod_r 2 cosh(m g_(2r) / 2),     Z4 = prod_r 2 sinh(m g_(2r) / 2),
r = 0 .. n-1, with cosh g_k = cosh 2K coth 2K - cos(pi k / n) (g_k > 0) for
k != 0 and g_0 = 2K + ln tanh K (of either sign).  It is evaluated here in
log form with signs; ``log_z_enumerated`` is the plain sum over all 2^(mn)
configurations that pins it on small tori.
"""
from __future__ import annotations

import numpy as np


def _gamma(k, n, K):
    if k == 0:
        return 2.0 * K + np.log(np.tanh(K))
    c = np.cosh(2.0 * K) / np.tanh(2.0 * K) - np.cos(np.pi * k / n)
    return np.arccosh(c)


def _log2cosh(x):
    x = abs(x)
    return x + np.log1p(np.exp(-2.0 * x))


def _log2sinh(x):
    """(sign, log|2 sinh x|)"""
    if x == 0.0:
        return 0.0, -np.inf
    ax = abs(x)
    return np.sign(x), ax + np.log1p(-np.exp(-2.0 * ax))


def log_z_kaufman(m, n, K):
    """ln Z of the m x n periodic Ising model with coupling K (closed form)."""
    terms = []  # (sign, log)
    for odd, hyper in [(1, "c"), (1, "s"), (0, "c"), (0, "s")]:
        sign, lg = 1.0, 0.0
        for r in range(n):
            g = _gamma(2 * r + odd, n, K)
            if hyper == "c":
                lg += _log2cosh(0.5 * m * g)
            else:
                sg, l2 = _log2sinh(0.5 * m * g)
                sign *= sg
                lg += l2
        terms.append((sign, lg))
    top = max(t[1] for t in terms if t[0] != 0.0)
    acc = sum(sg * np.exp(lg - top) for sg, lg in terms if sg != 0.0)
    return np.log(0.5) + 0.5 * m * n * np.log(2.0 * np.sinh(2.0 * K)) + top + np.log(acc)


def bonds(m, n):
    """Nearest-neighbour bonds of the periodic m x n torus (rows of length n)."""
    out = []
    for y in range(m):
        for x in range(n):
            i = y * n + x
            out.append((i, y * n + (x + 1) % n))
            out.append((i, ((y + 1) % m) * n + x))
    return out


def log_z_enumerated(m, n, K):
    """ln Z by the plain sum over all 2^(mn) configurations (small tori only)."""
    N = m * n
    codes = np.arange(2 ** N, dtype=np.int64)
    s = 2 * ((codes[:, None] >> np.arange(N)[None, :]) & 1) - 1
    e = np.zeros(2 ** N)
    for i, j in bonds(m, n):
        e += s[:, i] * s[:, j]
    top = K * e.max()
    return top + np.log(np.sum(np.exp(K * e - top)))


def nn_correlation(m, n, K, h=1e-5):
    """<s_i s_j> over nearest-neighbour pairs: (1 / 2mn) d ln Z / dK (central difference)."""
    return (log_z_kaufman(m, n, K + h) - log_z_kaufman(m, n, K - h)) / (2.0 * h) / (2.0 * m * n)


K_CRITICAL = 0.5 * np.log(1.0 + np.sqrt(2.0))
