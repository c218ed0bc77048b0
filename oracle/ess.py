"""Integrated autocorrelation time and effective sample size of chain series.

Not part of the paper; needed to compare Metropolis proposals at equal
statistical error.  Reading (Sokal, "Monte Carlo methods in statistical
mechanics", 1997 lecture notes, Sec. 3):
  rho(t)   autocorrelation of the series at lag t, averaged over chains, each
           chain centred on the grand mean;
  tau(W)   = 1/2 + sum_{t=1}^{W} rho(t);
  window   the smallest W with W >= c * tau(W), c = 5;
  ESS      = N_total / (2 tau);  sigma_mean = sqrt(Var / ESS).
A batch-means estimate is provided as an independent cross-check.
"""
from __future__ import annotations

import numpy as np


def autocorrelation(x):
    """x: (T, n_chains) real series -> rho(t), t = 0..T-1 (chain-averaged)."""
    x = np.asarray(x, dtype=np.float64)
    T, C = x.shape
    xc = x - x.mean()
    var = np.mean(xc * xc)
    rho = np.empty(T)
    for t in range(T):
        rho[t] = np.mean(xc[: T - t] * xc[t:]) / var if var > 0 else 0.0
    return rho


def tau_int(x, c=5.0):
    rho = autocorrelation(x)
    tau = 0.5
    for W in range(1, len(rho)):
        tau += rho[W]
        if W >= c * tau:
            return tau, W
    return tau, len(rho) - 1


def ess(x, c=5.0):
    x = np.asarray(x, dtype=np.float64)
    tau, _ = tau_int(x, c)
    return x.size / (2.0 * tau), tau


def batch_means_tau(x, n_batches=16):
    """tau from the variance of batch means (each chain cut into batches)."""
    x = np.asarray(x, dtype=np.float64)
    T, C = x.shape
    bl = T // n_batches
    means = x[: bl * n_batches].reshape(n_batches, bl, C).mean(axis=1)
    var_b = means.var(ddof=1)
    return 0.5 * bl * var_b / x.var()
