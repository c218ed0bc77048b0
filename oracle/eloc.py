"""Local estimator and exact-enumeration expectation values.

Paper: Sec. 2.1, eq:Oloc
    O_loc(s) = sum_s' <s|O|s'> psi(s') / psi(s),
evaluated with psi(s')/psi(s) = exp(log psi(s') - log psi(s)); eq:expectation_value
    <O> = sum_s p(s) O_loc(s),  p(s) = |psi(s)|^2 / <psi|psi>;
and eq:Oloc_mean, the empirical mean over samples.  The exact "sampler" of
Sec. 4.2 ("Sampler") evaluates the network on all 2^N configurations.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def local_energy(logpsi_fn, kind, bits, Lx, Ly, periodic, J, h=0.0):
    """E_loc for each row of the (B, N) 0/1 array ``bits``.

    ``logpsi_fn`` maps a (M, N) 0/1 array to complex128 (M,) log-amplitudes.
    Every connected configuration is evaluated by the network (the paper's
    evaluation of psi on the off-diagonal configurations)."""
    bits = np.atleast_2d(bits)
    out = np.zeros(len(bits), dtype=np.complex128)
    for n, s in enumerate(bits):
        sp, mel, cnt = lattice.connected(kind, s, Lx, Ly, periodic, J, h)
        lp_s = logpsi_fn(s[None, :])[0]
        lp_sp = logpsi_fn(sp[:cnt])
        out[n] = np.sum(mel[:cnt] * np.exp(lp_sp - lp_s))
    return out


def all_states(n: int) -> np.ndarray:
    """All 2^n configurations as a (2^n, n) 0/1 array; row k has bit i of k at site i."""
    k = np.arange(2 ** n, dtype=np.int64)
    return ((k[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)


def exact_probabilities(logpsi_fn, n: int, states=None):
    """p(s) = |psi(s)|^2 / Z over ``states`` (default all 2^n), with log psi."""
    if states is None:
        states = all_states(n)
    lp = logpsi_fn(states)
    w = np.exp(2.0 * (lp.real - lp.real.max()))
    return states, w / w.sum(), lp


def exact_expectation(logpsi_fn, kind, n, Lx, Ly, periodic, J, h=0.0, states=None):
    """<H> = sum_s p(s) E_loc(s) by enumeration; returns (E, p, E_loc, states)."""
    states, p, _ = exact_probabilities(logpsi_fn, n, states)
    el = local_energy(logpsi_fn, kind, states, Lx, Ly, periodic, J, h)
    return np.sum(p * el), p, el, states
