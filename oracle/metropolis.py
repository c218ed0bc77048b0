"""Metropolis sampling of p(s) = |psi(s)|^2 / <psi|psi> with many chains in sync.

Paper: Sec. 2.1 (samples from the Metropolis-Hastings algorithm) and Sec. 4.2
"Sampler" (MCSampler: an update proposer, proposals per sweep, thermalisation
sweeps, many chains run in a vectorised manner, sample count rounded up to
fill all chains).  The acceptance rule is Metropolis' for a symmetric proposal:
accept s -> s' with probability min(1, |psi(s')|^2 / |psi(s)|^2).

Readings (the paper fixes none of these; the library documents the same):
  * randomness: Philox4x32-10, key = (seed_lo, seed_hi);
      proposal t of chain c:      counter (c, t_lo, t_hi, 0)
      initial state of chain c:   counter (c, w, 0, 2) (random words) or
                                   (c, i, 1, 2) (Fisher-Yates step i)
  * flip proposal: site l = idx(x0, N); exchange proposal: bond b = idx(x0,
    n_bonds), the two spins of the bond swapped (equal spins: identity move);
  * u = unif(x1, x2); r = 2 Re(log psi(s') - log psi(s)); accept iff r >= 0 or
    u < exp(r);
  * initial state: uniformly random bits (flip), or the configuration with
    sites 0..N/2-1 up shuffled by Fisher-Yates with j = idx(x0, i + 1) for
    i = N-1 .. 1 (exchange, Sz = 0);
  * one sweep = sweep_steps proposals; therm_sweeps sweeps before the first
    recorded sample; one recorded sample per chain per sweep; sample-major
    output (index = k * n_chains + c).
"""
from __future__ import annotations

import numpy as np

from . import philox, lattice


def initial_states(n_chains, n_sites, key, sz0, chain_ids=None):
    """Initial 0/1 configurations (n_chains, N) as described in the module doc."""
    cids = np.arange(n_chains) if chain_ids is None else np.asarray(chain_ids)
    out = np.zeros((len(cids), n_sites), dtype=np.uint8)
    for r, c in enumerate(cids):
        if not sz0:
            n_words = (n_sites + 63) // 64
            for w in range(n_words):
                x = philox.philox4x32_10([c, w // 2, 0, 2], key)
                lo, hi = (x[0], x[1]) if w % 2 == 0 else (x[2], x[3])
                word = int(lo) | (int(hi) << 32)
                for b in range(64):
                    i = 64 * w + b
                    if i < n_sites:
                        out[r, i] = (word >> b) & 1
        else:
            s = np.zeros(n_sites, dtype=np.uint8)
            s[: n_sites // 2] = 1
            for i in range(n_sites - 1, 0, -1):
                x = philox.philox4x32_10([c, i, 1, 2], key)
                j = int(philox.to_index(x[0], i + 1))
                s[i], s[j] = s[j], s[i]
            out[r] = s
    return out


def propose(kind_prop, states, t, key, chain_ids, bond_list):
    """Proposals of step t for every chain; returns (s', u)."""
    cids = np.asarray(chain_ids, dtype=np.uint64)
    ctr = np.zeros((len(cids), 4), dtype=np.uint32)
    ctr[:, 0] = cids.astype(np.uint32)
    ctr[:, 1] = np.uint32(t & 0xFFFFFFFF)
    ctr[:, 2] = np.uint32(t >> 32)
    x = philox.philox4x32_10(ctr, key)
    sp = states.copy()
    N = states.shape[1]
    if kind_prop == "flip":
        l = philox.to_index(x[:, 0], N)
        sp[np.arange(len(sp)), l] ^= 1
    elif kind_prop == "exchange":
        b = philox.to_index(x[:, 0], len(bond_list))
        bl = np.asarray(bond_list)
        i, j = bl[b, 0], bl[b, 1]
        rows = np.arange(len(sp))
        sp[rows, i], sp[rows, j] = states[rows, j], states[rows, i]
    else:
        raise ValueError(kind_prop)
    u = philox.to_uniform(x[:, 1], x[:, 2])
    return sp, u


def accept(r, u):
    """Metropolis decision for r = 2 Re(log psi(s') - log psi(s))."""
    return (r >= 0.0) | (u < np.exp(np.minimum(r, 0.0)))


class Chains:
    """A set of Metropolis chains (possibly a subset of a larger ensemble,
    given by ``chain_ids``) that replays the library's random stream.

    proposal "made_mix" (not in the paper): every sweep (thermalisation
    sweeps included) starts with ``global_steps`` global proposals made by all
    chains together, then ``sweep_steps`` single-spin flips as for "flip".
    Global proposal g (counted from 0 over the chains' life, apart from the
    flip counter t) of chain c draws s' ~ q with oracle.made.sample at (row,
    counter) = (c, g) and u = unif(x1, x2) of x = Philox((c, g_lo, g_hi, 3)),
    and is accepted with the Metropolis-Hastings rule for the independent
    proposal q: r = 2 Re(log psi(s') - log psi(s)) + log q(s) - log q(s'),
    accept iff r >= 0 or u < exp(r).  Each global step and each flip leaves
    |psi|^2 invariant, so their composition does too."""

    def __init__(self, logpsi_fn, n_sites, proposal, seed, chain_ids,
                 bond_list=None, sweep_steps=None, therm_sweeps=20, made=None, global_steps=0):
        self.f = logpsi_fn
        self.key = philox.seed_key(seed)
        self.proposal = proposal
        self.cids = np.asarray(chain_ids)
        self.bonds = bond_list
        self.sweep = n_sites if sweep_steps is None else sweep_steps
        self.therm = therm_sweeps
        self.seed = seed
        self.made = made            # (params, N, H) of the frozen proposal network
        self.global_steps = global_steps
        self.g = 0                  # global proposals made so far (per chain)
        self.n_global = 0
        self.acc_global = 0
        self.states = initial_states(len(self.cids), n_sites, self.key,
                                     proposal == "exchange", self.cids)
        self.logpsi = self.f(self.states)
        self.t = 0
        self.thermalized = False
        self.accepted = 0
        self.proposed = 0
        self.near_ties = 0

    def step(self):
        kind = "flip" if self.proposal == "made_mix" else self.proposal
        sp, u = propose(kind, self.states, self.t, self.key, self.cids, self.bonds)
        lp = self.f(sp)
        r = 2.0 * (lp.real - self.logpsi.real)
        with np.errstate(divide="ignore"):
            self.near_ties += int(np.sum(np.abs(r - np.log(u)) < 1e-12))
        acc = accept(r, u)
        self.states[acc] = sp[acc]
        self.logpsi[acc] = lp[acc]
        self.accepted += int(acc.sum())
        self.proposed += len(acc)
        self.t += 1

    def global_step(self):
        """One MADE proposal for every chain, Metropolis-Hastings acceptance."""
        from . import made as omade

        mp, N, H = self.made
        g = self.g
        sp, lq_new = omade.sample(mp, len(self.cids), N, H, self.seed, g & 0xFFFFFFFF, g >> 32, rows=self.cids)
        lq_old = omade.log_q(mp, self.states, N, H)
        lp_new = self.f(sp)
        ctr = np.zeros((len(self.cids), 4), dtype=np.uint32)
        ctr[:, 0] = self.cids.astype(np.uint32)
        ctr[:, 1] = np.uint32(g & 0xFFFFFFFF)
        ctr[:, 2] = np.uint32(g >> 32)
        ctr[:, 3] = 3
        x = philox.philox4x32_10(ctr, self.key)
        u = philox.to_uniform(x[:, 1], x[:, 2])
        r = 2.0 * (lp_new.real - self.logpsi.real) + lq_old - lq_new
        with np.errstate(divide="ignore"):
            self.near_ties += int(np.sum(np.abs(r - np.log(u)) < 1e-12))
        acc = accept(r, u)
        self.states[acc] = sp[acc]
        self.logpsi[acc] = lp_new[acc]
        self.accepted += int(acc.sum())
        self.acc_global += int(acc.sum())
        self.n_global += len(acc)
        self.proposed += len(acc)
        self.g += 1

    def _sweep(self):
        if self.proposal == "made_mix":
            for _ in range(self.global_steps):
                self.global_step()
        for _ in range(self.sweep):
            self.step()

    def sample(self, n_per_chain):
        """Returns (configs (n_per_chain, n_chains, N), logpsi (n_per_chain, n_chains))."""
        if not self.thermalized:
            for _ in range(self.therm):
                self._sweep()
            self.thermalized = True
        out_s, out_l = [], []
        for _ in range(n_per_chain):
            self._sweep()
            out_s.append(self.states.copy())
            out_l.append(self.logpsi.copy())
        return np.stack(out_s), np.stack(out_l)


def transition_matrix(logpsi_fn, kind_prop, n_sites, bond_list=None, states=None):
    """Exact one-proposal transition matrix P[s, s'] over ``states`` (default all
    2^N), for the flip or exchange proposal with Metropolis acceptance."""
    from .eloc import all_states

    if states is None:
        states = all_states(n_sites)
    codes = (states.astype(np.int64) << np.arange(n_sites)).sum(1)
    index = {int(c): k for k, c in enumerate(codes)}
    lp = logpsi_fn(states)
    n = len(states)
    P = np.zeros((n, n))
    for k, s in enumerate(states):
        moves = []
        if kind_prop == "flip":
            for l in range(n_sites):
                sp = s.copy()
                sp[l] ^= 1
                moves.append(sp)
        else:
            for (i, j) in bond_list:
                sp = s.copy()
                sp[i], sp[j] = s[j], s[i]
                moves.append(sp)
        q = 1.0 / len(moves)
        for sp in moves:
            kk = index[int((sp.astype(np.int64) << np.arange(n_sites)).sum())]
            if kk == k:
                continue
            ratio = np.exp(2.0 * (lp[kk].real - lp[k].real))
            P[k, kk] += q * min(1.0, ratio)
        P[k, k] = 1.0 - P[k].sum()
    return P, states, lp
