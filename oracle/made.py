"""Masked autoregressive network (MADE) used as a global Metropolis-Hastings
proposal, in float64.

Not part of the paper: the paper's autoregressive networks sample directly
(Sec. 2.4: p(s) = prod_i p_i(s_i | s_<i), one network pass per sample instead
of O(N) Metropolis evaluations).  Here such a network q is trained on the
chain's own samples and used as an independent proposal inside Metropolis-
Hastings (Hastings 1970), so the chain keeps |psi|^2 as its exact target.

Network (Germain, Gregor, Murray, Larochelle, "MADE", ICML 2015), inputs x = s
in {0, 1}^N in site order, one ReLU hidden layer of H units:
  hidden degree   m(k) = (k mod (N - 1)) + 1,   input/output degree of site d: d + 1
  masks           M1[k, d] = [m(k) >= d + 1],   M2[d, k] = [d + 1 > m(k)]
  logits          l = (W2 * M2) relu((W1 * M1) x + b1) + b2,   p = sigmoid(l)
  log q(s)        = sum_d s_d log p_d + (1 - s_d) log(1 - p_d) = sum_d s_d l_d - softplus(l_d)
Flat parameter order: [W1 (H x N), b1 (H), W2 (N x H), b2 (N)].

Readings: loss = mean negative log-likelihood over a minibatch; Adam (Kingma &
Ba 2015) with beta1 0.9, beta2 0.999, eps 1e-8; minibatches are consecutive
rows in order.  Autoregressive sampling of row c with a counter pair (lo, hi):
site d draws x = Philox4x32-10((c, lo, hi, 1 + 256 * (d // 4)), key) and is up
iff x[d % 4] * 2^-32 < p_d.
"""
from __future__ import annotations

import numpy as np

from . import philox


def degrees(N, H):
    return (np.arange(H) % (N - 1)) + 1


def masks(N, H):
    m = degrees(N, H)
    d = np.arange(N) + 1
    M1 = (m[:, None] >= d[None, :]).astype(np.float64)   # H x N
    M2 = (d[:, None] > m[None, :]).astype(np.float64)    # N x H
    return M1, M2


def split(params, N, H):
    p = np.asarray(params, dtype=np.float64)
    W1 = p[: H * N].reshape(H, N)
    b1 = p[H * N: H * N + H]
    W2 = p[H * N + H: H * N + H + N * H].reshape(N, H)
    b2 = p[H * N + H + N * H:]
    return W1, b1, W2, b2


def softplus(x):
    return np.logaddexp(0.0, x)


def forward(params, x, N, H):
    """Returns (pre-activations a (B,H), hidden h (B,H), logits l (B,N))."""
    W1, b1, W2, b2 = split(params, N, H)
    M1, M2 = masks(N, H)
    x = np.atleast_2d(x).astype(np.float64)
    a = x @ (W1 * M1).T + b1
    h = np.maximum(a, 0.0)
    l = h @ (W2 * M2).T + b2
    return a, h, l


def log_q(params, x, N, H):
    x = np.atleast_2d(x).astype(np.float64)
    _, _, l = forward(params, x, N, H)
    return np.sum(x * l - softplus(l), axis=1)


def nll_and_grad(params, x, N, H):
    """Mean negative log-likelihood over the rows of x and its gradient (flat order)."""
    x = np.atleast_2d(x).astype(np.float64)
    B = len(x)
    W1, b1, W2, b2 = split(params, N, H)
    M1, M2 = masks(N, H)
    a, h, l = forward(params, x, N, H)
    nll = -np.mean(np.sum(x * l - softplus(l), axis=1))
    g_l = (1.0 / (1.0 + np.exp(-l)) - x) / B          # d nll / d logits
    gW2 = (g_l.T @ h) * M2
    gb2 = g_l.sum(0)
    g_h = g_l @ (W2 * M2)
    g_a = g_h * (a > 0.0)
    gW1 = (g_a.T @ x) * M1
    gb1 = g_a.sum(0)
    return nll, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


class Adam:
    def __init__(self, n, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, params, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return params - self.lr * mh / (np.sqrt(vh) + self.eps)


def train(params, x, N, H, epochs, batch, lr):
    """Adam on consecutive minibatches; returns (params, mean nll of the last epoch)."""
    opt = Adam(len(params), lr)
    p = np.array(params, dtype=np.float64)
    last = 0.0
    for _ in range(epochs):
        tot, nb = 0.0, 0
        for b0 in range(0, len(x), batch):
            nll, g = nll_and_grad(p, x[b0: b0 + batch], N, H)
            p = opt.step(p, g)
            tot += nll
            nb += 1
        last = tot / nb
    return p, last


def sample(params, B, N, H, seed, lo, hi, rows=None):
    """Autoregressive samples for rows (default 0..B-1); returns (x (B,N) uint8, log q (B,))."""
    W1, b1, W2, b2 = split(params, N, H)
    M1, M2 = masks(N, H)
    W1m, W2m = W1 * M1, W2 * M2
    key = philox.seed_key(seed)
    rows = np.arange(B) if rows is None else np.asarray(rows)
    x = np.zeros((len(rows), N), dtype=np.uint8)
    lq = np.zeros(len(rows))
    for d in range(N):
        ctr = np.zeros((len(rows), 4), dtype=np.uint32)
        ctr[:, 0] = rows.astype(np.uint32)
        ctr[:, 1] = np.uint32(lo)
        ctr[:, 2] = np.uint32(hi)
        ctr[:, 3] = np.uint32(1 + 256 * (d // 4))
        u = philox.philox4x32_10(ctr, key)[:, d % 4].astype(np.float64) * 2.0 ** -32
        h = np.maximum(x.astype(np.float64) @ W1m.T + b1, 0.0)
        ld = h @ W2m[d] + b2[d]
        p = 1.0 / (1.0 + np.exp(-ld))
        xd = (u < p).astype(np.uint8)
        x[:, d] = xd
        lq += xd * ld - softplus(ld)
    return x, lq


def global_transition_matrix(logpsi_fn, params, N, H, states=None):
    """Exact kernel of one global proposal over all 2^N states (the independent
    Metropolis-Hastings kernel of q): P(s -> s') = q(s') min(1, pi(s') q(s) /
    (pi(s) q(s'))) for s' != s, the diagonal takes the remainder."""
    from .eloc import all_states

    if states is None:
        states = all_states(N)
    lp = logpsi_fn(states)
    lq = log_q(params, states, N, H)
    q = np.exp(lq)
    lpi = 2.0 * lp.real
    n = len(states)
    P = np.zeros((n, n))
    for k in range(n):
        r = (lpi - lpi[k]) + (lq[k] - lq)
        P[k] = q * np.minimum(1.0, np.exp(np.minimum(r, 0.0)))
        P[k, k] = 0.0
        P[k, k] = 1.0 - P[k].sum()
    return P, states, lp, lq


def sweep_transition_matrix(logpsi_fn, params, N, H, global_steps, flip_steps, states=None):
    """Kernel of one sweep of the mixed sampler: global_steps global proposals,
    then flip_steps single-spin flips (matrix product in that order)."""
    from .metropolis import transition_matrix

    Pg, states, lp, lq = global_transition_matrix(logpsi_fn, params, N, H, states)
    Pf, _, _ = transition_matrix(logpsi_fn, "flip", N, None, states)
    P = np.linalg.matrix_power(Pg, global_steps) @ np.linalg.matrix_power(Pf, flip_steps)
    return P, states, lp, lq
