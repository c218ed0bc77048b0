"""Pins of oracle.symelu (the translation-symmetric ELU network of the paper's
ground-state example): translation invariance, the W = 0 closed form, the ELU
branches, finite-difference log-derivatives, and a brute-force double loop."""
import numpy as np

from oracle import symelu
import synth_inputs as si


def test_translation_invariance():
    L, al = 9, 3
    th = si.symelu_params(L, al, seed=1, std=0.4)
    x = si.random_bits(20, L, seed=2)
    lp = symelu.log_psi(th, x, L, al)
    for k in range(1, L):
        assert np.allclose(symelu.log_psi(th, np.roll(x, k, axis=1), L, al), lp, atol=1e-12)


def test_zero_weights_closed_form():
    L, al = 7, 2
    th = np.zeros(al * (L + 1))
    th[al * L:] = [0.3, -0.8]
    x = si.random_bits(5, L, seed=3)
    want = L * (0.3 + np.expm1(-0.8))
    assert np.allclose(symelu.log_psi(th, x, L, al), want, atol=1e-14)


def test_brute_force_double_loop():
    L, al = 6, 2
    th = si.symelu_params(L, al, seed=4, std=0.6)
    W, b = th[: al * L].reshape(al, L), th[al * L:]
    x = si.random_bits(4, L, seed=5)
    for r, s in enumerate(x):
        sig = 2.0 * s - 1.0
        tot = 0.0
        for a in range(al):
            for w in range(L):
                t = b[a] + sum(W[a, l] * sig[(l + w) % L] for l in range(L))
                tot += t if t > 0 else np.exp(t) - 1.0
        assert abs(symelu.log_psi(th, s[None], L, al)[0] - tot) < 1e-12


def test_grad_against_finite_differences():
    L, al = 8, 2
    th = si.symelu_params(L, al, seed=6, std=0.5)
    x = si.random_bits(6, L, seed=7)
    O = symelu.grad_log_psi(th, x, L, al)
    eps = 1e-6
    for k in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (symelu.log_psi(tp, x, L, al) - symelu.log_psi(tm, x, L, al)) / (2 * eps)
        assert np.max(np.abs(O[:, k] - fd)) < 1e-7
