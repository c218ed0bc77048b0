"""Two-layer periodic convolutional NQS: log-amplitude and log-derivatives.

Paper: the convolutional network class of Sec. 4.2 ("nets"; ANN layers as in
eq:affine-linear with a non-linearity), holomorphic complex parameters
(Sec. 2.3), sum-pooled output so that log psi is translation invariant (the
symmetrisation the paper obtains with periodic CNNs, Sec. 5.1).  The
architecture of the benchmark workload (reading; the paper's CNNs differ in
depth): on an Lx x Ly torus with C channels and k x k kernels,
  z1[c,y,x] = b1_c + sum_{dy,dx} W1[c,dy,dx] sigma[(y+dy) % Ly, (x+dx) % Lx]
  a1        = log cosh(z1)
  z2[c,y,x] = b2_c + sum_{c',dy,dx} W2[c,c',dy,dx] a1[c', (y+dy) % Ly, (x+dx) % Lx]
  log psi   = sum_{c,y,x} log cosh(z2[c,y,x])
(cross-correlation, stride 1, circular padding, sigma = 2 s - 1, site index
i = y Lx + x).  Flat parameter order [W1 (C,k,k), b1 (C), W2 (C,C,k,k), b2 (C)].
"""
from __future__ import annotations

import numpy as np


def num_params(C, k):
    return C * k * k + C + C * C * k * k + C


def split(params, C, k):
    p = np.asarray(params, dtype=np.complex128)
    n1 = C * k * k
    W1 = p[:n1].reshape(C, k, k)
    b1 = p[n1:n1 + C]
    W2 = p[n1 + C:n1 + C + C * C * k * k].reshape(C, C, k, k)
    b2 = p[n1 + C + C * C * k * k:]
    return W1, b1, W2, b2


def _shift(a, dy, dx):
    """out[..., y, x] = a[..., (y + dy) % Ly, (x + dx) % Lx]."""
    return np.roll(a, shift=(-dy, -dx), axis=(-2, -1))


def layers(params, bits, Lx, Ly, C, k):
    """Returns (sigma (B,Ly,Lx), z1 (B,C,Ly,Lx), a1, z2 (B,C,Ly,Lx))."""
    W1, b1, W2, b2 = split(params, C, k)
    bits = np.atleast_2d(bits)
    sigma = (2.0 * bits.astype(np.float64) - 1.0).reshape(-1, Ly, Lx)
    B = len(sigma)
    z1 = np.broadcast_to(b1[None, :, None, None], (B, C, Ly, Lx)).astype(np.complex128).copy()
    for dy in range(k):
        for dx in range(k):
            z1 += W1[None, :, dy, dx, None, None] * _shift(sigma, dy, dx)[:, None]
    a1 = np.log(np.cosh(z1))
    z2 = np.broadcast_to(b2[None, :, None, None], (B, C, Ly, Lx)).astype(np.complex128).copy()
    for dy in range(k):
        for dx in range(k):
            sh = _shift(a1, dy, dx)                      # (B, C', Ly, Lx)
            z2 += np.einsum("oi,biyx->boyx", W2[:, :, dy, dx], sh)
    return sigma, z1, a1, z2


def log_psi(params, bits, Lx, Ly, C, k):
    _, _, _, z2 = layers(params, bits, Lx, Ly, C, k)
    return np.sum(np.log(np.cosh(z2)), axis=(1, 2, 3))


def grad_log_psi(params, bits, Lx, Ly, C, k):
    """O_k(s) by the chain rule (complex derivative); (B, K) in flat order."""
    W1, b1, W2, b2 = split(params, C, k)
    sigma, z1, a1, z2 = layers(params, bits, Lx, Ly, C, k)
    B = len(sigma)
    g2 = np.tanh(z2)                                      # d log psi / d z2
    gW2 = np.zeros((B, C, C, k, k), dtype=np.complex128)
    ga1 = np.zeros_like(a1)                               # d log psi / d a1
    for dy in range(k):
        for dx in range(k):
            gW2[:, :, :, dy, dx] = np.einsum("boyx,biyx->boi", g2, _shift(a1, dy, dx))
            # z2[o,y,x] uses a1[i,(y+dy),(x+dx)]: scatter back with the opposite shift
            ga1 += np.einsum("oi,boyx->biyx", W2[:, :, dy, dx], _shift(g2, -dy, -dx))
    gb2 = g2.sum(axis=(2, 3))
    g1 = ga1 * np.tanh(z1)                                # d log psi / d z1
    gW1 = np.zeros((B, C, k, k), dtype=np.complex128)
    for dy in range(k):
        for dx in range(k):
            gW1[:, :, dy, dx] = np.einsum("bcyx,byx->bc", g1, _shift(sigma, dy, dx))
    gb1 = g1.sum(axis=(2, 3))
    return np.concatenate([gW1.reshape(B, -1), gb1, gW2.reshape(B, -1), gb2], axis=1)
