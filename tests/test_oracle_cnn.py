"""Pins of oracle.cnn: the convolution as an explicit circulant matrix built
from index arithmetic, translation invariance, the W2 = 0 and single-tap
special cases, finite differences and Cauchy-Riemann, and local energies of
the constant-amplitude limit."""
import numpy as np
import pytest

from oracle import cnn, eloc, lattice
import synth_inputs as si


def circulant_log_psi(params, bits, Lx, Ly, C, k):
    """The same network written as dense matrix products: layer-1 matrix
    M1[(c,y,x),(Y,X)] = W1[c,(Y-y)%Ly,(X-x)%Lx] when both offsets are < k."""
    W1, b1, W2, b2 = cnn.split(params, C, k)
    n = Lx * Ly
    M1 = np.zeros((C * n, n), dtype=np.complex128)
    M2 = np.zeros((C * n, C * n), dtype=np.complex128)
    for c in range(C):
        for y in range(Ly):
            for x in range(Lx):
                row = c * n + y * Lx + x
                for Y in range(Ly):
                    for X in range(Lx):
                        dy, dx = (Y - y) % Ly, (X - x) % Lx
                        if dy < k and dx < k:
                            M1[row, Y * Lx + X] += W1[c, dy, dx]
                            for ci in range(C):
                                M2[row, ci * n + Y * Lx + X] += W2[c, ci, dy, dx]
    sig = 2.0 * np.atleast_2d(bits).astype(np.float64) - 1.0
    z1 = sig @ M1.T + np.repeat(b1, n)
    a1 = np.log(np.cosh(z1))
    z2 = a1 @ M2.T + np.repeat(b2, n)
    return np.log(np.cosh(z2)).sum(1)


@pytest.mark.parametrize("Lx,Ly,C,k", [(5, 5, 2, 3), (6, 4, 3, 2), (4, 4, 2, 4)])
def test_matches_circulant_form(Lx, Ly, C, k):
    p = si._normal_params(cnn.num_params(C, k), 0.3, True, seed=Lx * Ly + C)
    bits = si.random_bits(7, Lx * Ly, seed=2)
    a = cnn.log_psi(p, bits, Lx, Ly, C, k)
    b = circulant_log_psi(p, bits, Lx, Ly, C, k)
    assert np.allclose(a.real, b.real, atol=1e-12)
    assert np.allclose((a.imag - b.imag + np.pi) % (2 * np.pi) - np.pi, 0, atol=1e-12)


def test_translation_invariance():
    Lx = Ly = 6
    C, k = 3, 4
    p = si._normal_params(cnn.num_params(C, k), 0.2, True, seed=1)
    bits = si.random_bits(3, Lx * Ly, seed=4).reshape(3, Ly, Lx)
    ref = cnn.log_psi(p, bits.reshape(3, -1), Lx, Ly, C, k)
    for ty in range(Ly):
        for tx in range(Lx):
            t = np.roll(bits, (ty, tx), axis=(1, 2)).reshape(3, -1)
            assert np.allclose(cnn.log_psi(p, t, Lx, Ly, C, k), ref, atol=1e-12)


def test_special_cases():
    Lx, Ly, C, k = 4, 4, 3, 4
    p = si._normal_params(cnn.num_params(C, k), 0.3, True, seed=5)
    W1, b1, W2, b2 = cnn.split(p, C, k)
    q = p.copy()
    q[C * k * k + C: C * k * k + C + C * C * k * k] = 0.0   # W2 = 0
    bits = si.random_bits(4, 16, seed=6)
    assert np.allclose(cnn.log_psi(q, bits, Lx, Ly, C, k), Lx * Ly * np.sum(np.log(np.cosh(b2))), atol=1e-12)
    # one channel, 1x1 kernels: log psi = sum_i logcosh(b2 + w2 logcosh(b1 + w1 sigma_i))
    w1, c1, w2, c2 = 0.3 + 0.1j, -0.2 + 0.05j, 0.7 - 0.2j, 0.1 + 0.3j
    p1 = np.array([w1, c1, w2, c2])
    sig = 2.0 * bits - 1.0
    exp = np.log(np.cosh(c2 + w2 * np.log(np.cosh(c1 + w1 * sig)))).sum(1)
    assert np.allclose(cnn.log_psi(p1, bits, Lx, Ly, 1, 1), exp, atol=1e-13)


def test_grad_finite_differences_and_cauchy_riemann():
    Lx, Ly, C, k = 4, 3, 2, 2
    K = cnn.num_params(C, k)
    p = si._normal_params(K, 0.3, True, seed=7)
    bits = si.random_bits(3, Lx * Ly, seed=8)
    O = cnn.grad_log_psi(p, bits, Lx, Ly, C, k)
    eps = 1e-6
    for j in range(K):
        d = np.zeros(K, dtype=np.complex128)
        d[j] = eps
        fr = (cnn.log_psi(p + d, bits, Lx, Ly, C, k) - cnn.log_psi(p - d, bits, Lx, Ly, C, k)) / (2 * eps)
        fi = (cnn.log_psi(p + 1j * d, bits, Lx, Ly, C, k) - cnn.log_psi(p - 1j * d, bits, Lx, Ly, C, k)) / (2 * eps)
        assert np.allclose(fr, O[:, j], atol=1e-8)
        assert np.allclose(fi, 1j * O[:, j], atol=1e-8)


def test_constant_psi_local_energy():
    # W2 = 0: log psi constant -> E_loc = -J sum zz - h N for the TFIM
    Lx = Ly = 4
    C, k = 2, 4
    p = si._normal_params(cnn.num_params(C, k), 0.3, True, seed=9)
    p[C * k * k + C: C * k * k + C + C * C * k * k] = 0.0
    bits = si.random_bits(6, 16, seed=10)
    el = eloc.local_energy(lambda b: cnn.log_psi(p, b, Lx, Ly, C, k), "tfim", bits, Lx, Ly, True, 1.0, 3.0)
    bl = lattice.bonds(Lx, Ly, True)
    z = 2 * bits.astype(int) - 1
    zz = np.array([sum(zi[i] * zi[j] for i, j in bl) for zi in z])
    assert np.allclose(el, -zz - 3.0 * 16, atol=1e-11)
