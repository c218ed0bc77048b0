"""Pins of oracle.rbm and oracle.eloc: hidden units summed out by brute force,
finite differences, Cauchy-Riemann, closed-form local energies, an exact
eigenstate and two independent routes to <H>."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import rbm, eloc, lattice
import kron_ref
import synth_inputs as si


def brute_force_log_psi(params, bits, n_hidden):
    """The RBM as a Boltzmann machine with +-1 hidden units summed out:
    psi(s) = 2^-N_h sum_h exp(sum_i a_i sigma_i + sum_j h_j (sum_i W_ji sigma_i + b_j))."""
    n = bits.shape[1]
    p = np.asarray(params, dtype=np.complex128)
    a, b, W = p[:n], p[n:n + n_hidden], p[n + n_hidden:].reshape(n_hidden, n)
    out = []
    for s in bits:
        sig = 2.0 * s - 1.0
        tot = 0.0
        for h in itertools.product([-1.0, 1.0], repeat=n_hidden):
            h = np.array(h)
            energy = np.dot(a, sig) + np.dot(h, W @ sig + b)
            tot = tot + np.exp(energy)
        out.append(np.log(tot / 2.0 ** n_hidden))
    return np.array(out)


def wrap(d):
    return (d + np.pi) % (2 * np.pi) - np.pi


def test_log_psi_equals_hidden_sum():
    n, nh = 5, 4
    p = si.rbm_params(n, nh, std=0.4, seed=11)
    bits = si.random_bits(6, n, seed=3)
    lp = rbm.log_psi(p, bits, nh)
    bf = brute_force_log_psi(p, bits, nh)
    assert np.allclose(lp.real, bf.real, atol=1e-13)
    assert np.allclose(wrap(lp.imag - bf.imag), 0.0, atol=1e-13)


def test_zero_parameters_give_zero():
    p = np.zeros(si.rbm_num_params(7, 3), dtype=np.complex128)
    assert np.all(rbm.log_psi(p, si.random_bits(9, 7, 1), 3) == 0)


def test_grad_finite_differences_and_cauchy_riemann():
    n, nh = 6, 5
    p = si.rbm_params(n, nh, std=0.3, seed=5)
    bits = si.random_bits(4, n, seed=8)
    O = rbm.grad_log_psi(p, bits, nh)
    eps = 1e-5
    for k in range(len(p)):
        dp = np.zeros_like(p)
        dp[k] = eps
        fd_re = (rbm.log_psi(p + dp, bits, nh) - rbm.log_psi(p - dp, bits, nh)) / (2 * eps)
        fd_im = (rbm.log_psi(p + 1j * dp, bits, nh) - rbm.log_psi(p - 1j * dp, bits, nh)) / (2 * eps)
        assert np.allclose(fd_re, O[:, k], atol=1e-9)
        # holomorphic: d/dIm = i d/dRe
        assert np.allclose(fd_im, 1j * O[:, k], atol=1e-9)


def _zz(s, bl):
    z = 2 * s.astype(int) - 1
    return sum(z[i] * z[j] for i, j in bl)


@pytest.mark.parametrize("kind,Lx,Ly,J,h", [("tfim", 8, 1, 1.0, 0.9), ("tfim", 3, 3, 0.7, 3.0),
                                            ("heisenberg", 8, 1, 1.0, 0.0), ("heisenberg", 4, 4, 1.3, 0.0)])
def test_constant_psi_local_energy(kind, Lx, Ly, J, h):
    n = Lx * Ly
    p = np.zeros(si.rbm_num_params(n, n), dtype=np.complex128)
    bits = si.random_bits(10, n, seed=4)
    el = eloc.local_energy(lambda x: rbm.log_psi(p, x, n), kind, bits, Lx, Ly, True, J, h)
    bl = lattice.bonds(Lx, Ly, True)
    for s, e in zip(bits, el):
        zz = _zz(s, bl)
        if kind == "tfim":
            exp = -J * zz - h * n
        else:
            n_anti = sum(1 for i, j in bl if s[i] != s[j])
            exp = J * zz + 2 * J * n_anti
        assert abs(e - exp) < 1e-12


def table_logpsi(vec, n):
    """log psi from a table indexed by the library's state code (bit i = site i)."""
    lv = np.log(vec.astype(np.complex128))

    def f(bits):
        codes = (np.atleast_2d(bits).astype(np.int64) << np.arange(n)).sum(1)
        return lv[codes]
    return f


def test_eigenstate_has_constant_local_energy():
    # Sec. 5.1: the energy variance vanishes in an exact eigenstate.
    L, h = 8, 0.7
    Hk = kron_ref.tfim(L, 1, True, 1.0, h)
    w, v = sla.eigsh(Hk, k=1, which="SA", tol=1e-14)
    codes = np.arange(2 ** L)
    vec = v[kron_ref.code_to_kron(codes, L), 0]
    vec = vec * np.sign(vec[np.argmax(np.abs(vec))])
    assert np.all(vec > 0)  # Perron-Frobenius for the stoquastic TFIM
    f = table_logpsi(vec, L)
    el = eloc.local_energy(f, "tfim", eloc.all_states(L), L, 1, True, 1.0, h)
    assert np.max(np.abs(el - w[0])) < 1e-10
    assert abs(w[0] - kron_ref.pfeuty_e0(L, h)) < 1e-10


@pytest.mark.parametrize("kind,Lx,Ly,h,cplx", [("tfim", 10, 1, 1.0, False), ("tfim", 3, 3, 3.0, True),
                                               ("heisenberg", 8, 1, 0.0, True)])
def test_exact_energy_two_routes(kind, Lx, Ly, h, cplx):
    n = Lx * Ly
    p = si.rbm_params(n, n, std=0.2, is_complex=cplx, seed=9)
    f = lambda x: rbm.log_psi(p, x, n)
    E, prob, el, states = eloc.exact_expectation(f, kind, n, Lx, Ly, True, 1.0, h)
    codes = (states.astype(np.int64) << np.arange(n)).sum(1)
    v = np.zeros(2 ** n, dtype=np.complex128)
    v[kron_ref.code_to_kron(codes, n)] = np.exp(f(states) - f(states).real.max())
    Hk = kron_ref.tfim(Lx, Ly, True, 1.0, h) if kind == "tfim" else kron_ref.heisenberg(Lx, Ly, True, 1.0)
    E2 = np.vdot(v, Hk @ v) / np.vdot(v, v)
    assert abs(E - E2) < 1e-11 * max(1, abs(E2))
