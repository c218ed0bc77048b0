"""Pins of oracle.made: normalisation of q by enumeration, the autoregressive
property (masks), finite-difference gradients, Adam against its definition on
a quadratic, sample frequencies against q, and exact stationarity of the mixed
Metropolis-Hastings kernel."""
import numpy as np
import pytest
from scipy import stats

from oracle import made, eloc, rbm
import synth_inputs as si


def test_q_is_normalised():
    N, H = 8, 24
    p = si.made_params(N, H, seed=1) * 3.0
    states = eloc.all_states(N)
    assert abs(np.exp(made.log_q(p, states, N, H)).sum() - 1.0) < 1e-12


def test_autoregressive_property():
    # p_d depends only on x_<d: perturbing x_j for j >= d leaves logits l_d unchanged
    N, H = 9, 40
    p = si.made_params(N, H, seed=2) * 2.0
    x = si.random_bits(20, N, seed=3)
    _, _, l = made.forward(p, x, N, H)
    for j in range(N):
        x2 = x.copy()
        x2[:, j] ^= 1
        _, _, l2 = made.forward(p, x2, N, H)
        assert np.array_equal(l[:, : j + 1], l2[:, : j + 1])
        if j < N - 1:
            assert np.any(l[:, j + 1:] != l2[:, j + 1:])


def test_masks_structure():
    N, H = 6, 12
    M1, M2 = made.masks(N, H)
    assert M2[0].sum() == 0                      # first site is unconditional
    assert np.all(M1[:, N - 1] == 0)             # last input feeds nothing
    assert M1.shape == (H, N) and M2.shape == (N, H)


def test_nll_gradient_matches_finite_differences():
    N, H = 5, 12
    p = si.made_params(N, H, seed=4) * 1.5
    p[H * N: H * N + H] = np.random.default_rng(0).normal(0, 0.3, H)  # hidden biases
    x = si.random_bits(16, N, seed=5)
    nll, g = made.nll_and_grad(p, x, N, H)
    eps = 1e-6
    fd = np.zeros_like(p)
    for k in range(len(p)):
        d = np.zeros_like(p)
        d[k] = eps
        fd[k] = (made.nll_and_grad(p + d, x, N, H)[0] - made.nll_and_grad(p - d, x, N, H)[0]) / (2 * eps)
    assert np.max(np.abs(fd - g)) < 1e-8


def test_adam_definition_on_quadratic():
    # first step of Adam moves every coordinate by exactly lr (bias-corrected m/sqrt(v) = sign(g))
    opt = made.Adam(3, lr=0.1)
    x = np.array([1.0, -2.0, 3.0])
    x1 = opt.step(x, 2 * x)
    assert np.allclose(x1, x - 0.1 * np.sign(x), atol=1e-8)
    for _ in range(3000):
        x1 = opt.step(x1, 2 * x1)
    assert np.max(np.abs(x1)) < 1e-2


def test_sample_frequencies_match_q():
    N, H = 6, 16
    p = si.made_params(N, H, seed=6) * 4.0
    x, lq = made.sample(p, 20000, N, H, seed=9, lo=3, hi=0)
    assert np.allclose(lq, made.log_q(p, x, N, H), atol=1e-12)
    codes = (x.astype(np.int64) << np.arange(N)).sum(1)
    counts = np.bincount(codes, minlength=2 ** N)
    q = np.exp(made.log_q(p, eloc.all_states(N), N, H))
    assert stats.chisquare(counts, q * counts.sum()).pvalue > 1e-4


def test_training_lowers_nll():
    N, H = 8, 32
    p0 = si.made_params(N, H, seed=7)
    # data from a strongly correlated distribution: all-up or all-down plus noise
    rng = np.random.default_rng(1)
    base = rng.integers(0, 2, size=(2048, 1)).repeat(N, 1)
    flip = rng.random((2048, N)) < 0.05
    x = (base ^ flip).astype(np.uint8)
    nll0, _ = made.nll_and_grad(p0, x, N, H)
    p1, nll1 = made.train(p0, x, N, H, epochs=5, batch=128, lr=1e-2)
    assert nll1 < nll0 - 1.0


def test_global_kernel_detailed_balance_and_sweep_stationarity():
    # the independent MH kernel of q satisfies detailed balance with pi = |psi|^2;
    # a sweep (global proposals, then flips) is a product of pi-invariant kernels
    N, H = 6, 16
    pr = si.rbm_params(N, N, std=0.5, seed=3)
    f = lambda b: rbm.log_psi(pr, b, N)
    pm = si.made_params(N, H, seed=8) * 2.0
    Pg, states, lp, lq = made.global_transition_matrix(f, pm, N, H)
    pi = np.exp(2 * (lp.real - lp.real.max()))
    pi /= pi.sum()
    assert np.all(Pg >= -1e-15) and np.allclose(Pg.sum(1), 1.0, atol=1e-13)
    assert np.max(np.abs(pi @ Pg - pi)) < 1e-14
    D = pi[:, None] * Pg
    assert np.max(np.abs(D - D.T)) < 1e-15
    for G, L in [(1, 3), (4, 6), (2, 0)]:
        P, *_ = made.sweep_transition_matrix(f, pm, N, H, G, L)
        assert np.allclose(P.sum(1), 1.0, atol=1e-12)
        assert np.max(np.abs(pi @ P - pi)) < 1e-13


def test_mixed_oracle_chains_sample_psi_squared():
    # the oracle's mixed chains (global MADE steps + flips) histogram against
    # |psi|^2 on all 2^6 states (chi-square, samples thinned to every 4th sweep)
    from scipy import stats
    from oracle import metropolis as omet, eloc as oeloc
    N, H = 6, 16
    pr = si.rbm_params(N, N, std=0.5, seed=3)
    f = lambda b: rbm.log_psi(pr, b, N)
    pm = si.made_params(N, H, seed=8) * 2.0
    ch = omet.Chains(f, N, "made_mix", seed=5, chain_ids=np.arange(256), sweep_steps=2, therm_sweeps=10,
                     made=(pm, N, H), global_steps=1)
    s, _ = ch.sample(80)
    assert 0 < ch.acc_global < ch.n_global
    codes = (s[::4].reshape(-1, N).astype(np.int64) << np.arange(N)).sum(1)
    cnt = np.bincount(codes, minlength=2 ** N)
    _, prob, _ = oeloc.exact_probabilities(f, N)
    assert stats.chisquare(cnt, prob * cnt.sum()).pvalue > 1e-4
