"""Host-side statistics of chain series: integrated autocorrelation time and
effective sample size (ESS), used to compare Metropolis proposals at equal
statistical error.

tau_int = 1/2 + sum_{t=1}^{W} rho(t) with Sokal's self-consistent window, the
smallest W >= c tau_int(W) (c = 5); rho is the chain-averaged autocorrelation
of the series centred on the grand mean, each lag averaged over its T - t
pairs, computed by FFT (zero-padded, so the lag sums are the same finite sums
as the direct definition).
ESS = (number of values) / (2 tau_int).
"""
from __future__ import annotations

import numpy as np


def autocorrelation_fft(x: np.ndarray) -> np.ndarray:
    """x: (T, n_chains) -> rho(t) for t = 0..T-1, averaged over chains."""
    x = np.asarray(x, dtype=np.float64)
    T, C = x.shape
    xc = x - x.mean()
    n = 1 << int(np.ceil(np.log2(2 * T)))
    f = np.fft.rfft(xc, n=n, axis=0)
    acf = np.fft.irfft(f * np.conj(f), n=n, axis=0)[:T]   # sum_i x_i x_{i+t}, per chain
    acf = acf.sum(axis=1) / (C * (T - np.arange(T)))     # mean over the T - t pairs at lag t
    return acf / acf[0] if acf[0] > 0 else np.zeros(T)


def tau_int(x: np.ndarray, c: float = 5.0):
    rho = autocorrelation_fft(x)
    tau = 0.5
    for W in range(1, len(rho)):
        tau += rho[W]
        if W >= c * tau:
            return tau, W
    return tau, len(rho) - 1


def ess(x: np.ndarray, c: float = 5.0):
    """(ESS, tau_int) of a (T, n_chains) series."""
    x = np.asarray(x, dtype=np.float64)
    tau, _ = tau_int(x, c)
    return x.size / (2.0 * max(tau, 0.5)), tau
