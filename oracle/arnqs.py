"""Autoregressive neural quantum state with direct sampling, in float64.

Test infrastructure only: this module checks the HIP library and is never
called by it.

Paper: Sec. 2.4 (autoregressive NQS).  A distribution written as a product of
conditionals, q(s) = prod_i q_i(s_i | s_1 .. s_{i-1}), is sampled exactly one
site after the other, with no Markov chain.  The state used here is
psi(s) = sqrt(q(s)) with q the masked network of ``oracle.made`` (MADE, one
ReLU hidden layer), so

    log psi(s) = (1/2) log q(s) = (1/2) sum_i [s_i l_i - softplus(l_i)],

real and normalised over all 2^N configurations.

Only the weights the masks leave live are parameters, in the order
    W1 entries (k ascending, then d = 0 .. m(k)-1)
    b1 (H)
    W2 entries (i ascending, then k ascending with m(k) <= i)
    b2 (N)
so K = N H + H + N (every hidden unit k reaches m(k) inputs and N - m(k)
outputs).  Samples come from ``oracle.made.sample`` on the dense parameters
with the counter pair (lo, hi) of the 64-bit call counter.

Pins: normalisation sum_s q(s) = 1 over all configurations (fails for any
mask that lets a logit see its own or a later site); the first conditional is
sigmoid(b2_0) by marginalisation; O_k against central finite differences of
log psi; the live layout against the masks; <H> from the local energies
against psi^T H psi with the Kronecker-product Hamiltonian.
"""
from __future__ import annotations

import numpy as np

from . import made


def live_entries(N, H):
    """[(block, r, c)] in parameter order; block 0 = W1 (k, d), 1 = b1 (k),
    2 = W2 (i, k), 3 = b2 (i)."""
    m = made.degrees(N, H)
    out = []
    for k in range(H):
        for d in range(m[k]):
            out.append((0, k, d))
    for k in range(H):
        out.append((1, k, 0))
    for i in range(N):
        for k in range(H):
            if m[k] <= i:
                out.append((2, i, k))
    for i in range(N):
        out.append((3, i, 0))
    return out


def num_params(N, H):
    return N * H + H + N


def dense_params(theta, N, H):
    """Dense MADE vector [W1 (H x N), b1, W2 (N x H), b2] with zeros at masked weights."""
    theta = np.asarray(theta).real.astype(np.float64)
    W1 = np.zeros((H, N))
    b1 = np.zeros(H)
    W2 = np.zeros((N, H))
    b2 = np.zeros(N)
    for v, (blk, r, c) in zip(theta, live_entries(N, H)):
        if blk == 0:
            W1[r, c] = v
        elif blk == 1:
            b1[r] = v
        elif blk == 2:
            W2[r, c] = v
        else:
            b2[r] = v
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2])


def log_psi(theta, x, N, H):
    """(B,) float64 log psi for the (B, N) 0/1 rows of x."""
    return 0.5 * made.log_q(dense_params(theta, N, H), np.atleast_2d(x), N, H)


def grad_log_psi(theta, x, N, H):
    """(B, K) O_k = d log psi / d theta_k: per row, minus one half of the gradient
    of that row's negative log-likelihood, taken at the live entries."""
    p = dense_params(theta, N, H)
    ent = live_entries(N, H)
    HN = H * N
    pos = []
    for blk, r, c in ent:
        pos.append([r * N + c, HN + r, HN + H + r * H + c, 2 * HN + H + r][blk])
    pos = np.array(pos)
    x = np.atleast_2d(x)
    out = np.zeros((len(x), len(ent)))
    for n in range(len(x)):
        _, g = made.nll_and_grad(p, x[n:n + 1], N, H)
        out[n] = -0.5 * g[pos]
    return out


def sample(theta, B, N, H, seed, counter):
    """Direct samples of the call with 64-bit counter ``counter``: ((B, N) uint8, log psi (B,))."""
    x, lq = made.sample(dense_params(theta, N, H), B, N, H, seed, counter & 0xFFFFFFFF, counter >> 32)
    return x, 0.5 * lq
