"""Pins of oracle.ising and of the bond-RBM state it describes: Kaufman's
finite-torus partition function against enumeration of all configurations,
the bond-RBM |psi|^2 against the Ising Boltzmann weight, and the critical
nearest-neighbour correlation against the infinite-lattice value."""
import numpy as np
import pytest

from oracle import ising, rbm, eloc
import synth_inputs as si


@pytest.mark.parametrize("m,n", [(4, 4), (3, 4), (4, 3), (2, 6), (4, 5)])
@pytest.mark.parametrize("K", [0.1, 0.3, ising.K_CRITICAL, 0.6, 1.2])
def test_kaufman_matches_enumeration(m, n, K):
    assert abs(ising.log_z_kaufman(m, n, K) - ising.log_z_enumerated(m, n, K)) < 1e-11 * abs(
        ising.log_z_enumerated(m, n, K))


def test_bond_rbm_weight_is_the_ising_weight():
    # |psi(s)|^2 / prod_b exp(K s_i s_j) is the same for every configuration, K = ln cosh 2w
    Lx = Ly = 4
    w = si.W_CRITICAL
    p = si.bond_rbm_params(Lx, Ly, w)
    states = eloc.all_states(Lx * Ly)
    lp = rbm.log_psi(p, states, 2 * Lx * Ly)
    s = 2.0 * states - 1.0
    K = np.log(np.cosh(2.0 * w))
    e = sum(s[:, i] * s[:, j] for i, j in ising.bonds(Ly, Lx))
    d = 2.0 * lp.real - K * e
    assert np.ptp(d) < 1e-10
    assert abs(K - ising.K_CRITICAL) < 1e-14


def test_critical_correlation_approaches_the_infinite_lattice():
    # at K_c the nearest-neighbour correlation of the infinite lattice is sqrt(2)/2;
    # finite tori approach it with corrections of order 1/L
    vals = [ising.nn_correlation(L, L, ising.K_CRITICAL) for L in (8, 16, 32, 64)]
    diffs = [abs(v - np.sqrt(0.5)) for v in vals]
    assert diffs[-1] < 0.01
    assert all(diffs[i + 1] < diffs[i] for i in range(3))
