"""Restricted Boltzmann machine log-amplitude and log-derivatives.

Paper: Sec. 4.2 "Variational wave functions", eq:rbm_ex:
    log psi(s) = sum_i a_i sigma_i + sum_j log cosh( sum_i W_ji sigma_i + b_j ),
with sigma = 2 s - 1 (the 0/1 -> -1/+1 map of the accompanying network
definition) and one hidden bias per hidden unit (the equation places b inside
the visible sum; the dense layer it describes has one bias per output).

Log-derivatives O_k = d log psi / d theta_k (Sec. 2.2; complex derivative for
holomorphic nets, Sec. 2.3):
    O_{a_i} = sigma_i,   O_{b_j} = tanh(theta_j),   O_{W_ji} = sigma_i tanh(theta_j).

Flat parameter order (reading): [a (N), b (N_h), W (N_h x N, row-major)].
"""
from __future__ import annotations

import numpy as np


def unpack(words: np.ndarray, n: int) -> np.ndarray:
    """(B, W) uint64 packed configurations -> (B, n) 0/1 int array."""
    words = np.atleast_2d(np.asarray(words, dtype=np.uint64))
    i = np.arange(n)
    return ((words[:, i // 64] >> (i % 64).astype(np.uint64)) & np.uint64(1)).astype(np.int64)


def split(params: np.ndarray, n: int, n_hidden: int):
    p = np.asarray(params)
    a = p[:n]
    b = p[n:n + n_hidden]
    W = p[n + n_hidden:].reshape(n_hidden, n)
    return a, b, W


def log_psi(params: np.ndarray, bits: np.ndarray, n_hidden: int) -> np.ndarray:
    """log psi for each row of the (B, N) 0/1 array ``bits``; complex128 (B,)."""
    bits = np.atleast_2d(bits)
    n = bits.shape[1]
    a, b, W = split(np.asarray(params, dtype=np.complex128), n, n_hidden)
    sigma = 2.0 * bits.astype(np.float64) - 1.0
    theta = sigma @ W.T + b[None, :]
    return sigma @ a + np.sum(np.log(np.cosh(theta)), axis=1)


def grad_log_psi(params: np.ndarray, bits: np.ndarray, n_hidden: int) -> np.ndarray:
    """O_k(s) for each row of ``bits``; complex128 (B, K) in flat parameter order."""
    bits = np.atleast_2d(bits)
    n = bits.shape[1]
    a, b, W = split(np.asarray(params, dtype=np.complex128), n, n_hidden)
    sigma = 2.0 * bits.astype(np.float64) - 1.0
    t = np.tanh(sigma @ W.T + b[None, :])
    Ow = t[:, :, None] * sigma[:, None, :]
    return np.concatenate([sigma.astype(np.complex128), t, Ow.reshape(len(bits), -1)], axis=1)
