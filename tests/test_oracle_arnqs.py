"""Pins of oracle.arnqs (autoregressive state psi = sqrt(q), Sec. 2.4):
normalisation over all configurations, the unconditional first site, the live
parameter layout against the masks, O_k against finite differences, <H> from
local energies against the Kronecker-product Hamiltonian, and direct-sample
frequencies against q."""
import numpy as np
import pytest
from scipy import stats

from oracle import arnqs, eloc, made
import kron_ref
import synth_inputs as si


def test_live_layout_matches_masks():
    N, H = 7, 15
    K = arnqs.num_params(N, H)
    ent = arnqs.live_entries(N, H)
    assert len(ent) == K == N * H + H + N
    dense = arnqs.dense_params(np.ones(K), N, H)
    M1, M2 = made.masks(N, H)
    want = np.concatenate([M1.ravel(), np.ones(H), M2.ravel(), np.ones(N)])
    assert np.array_equal(dense, want)
    # order: W1 rows by hidden unit, then b1, then W2 rows by output site, then b2
    assert ent[0] == (0, 0, 0) and ent[-1] == (3, N - 1, 0)
    blocks = [e[0] for e in ent]
    assert blocks == sorted(blocks)


@pytest.mark.parametrize("N,H", [(6, 9), (9, 20)])
def test_normalised_over_all_states(N, H):
    th = si.ar_params(N, H, seed=3, std=1.0)
    states = eloc.all_states(N)
    assert abs(np.exp(2.0 * arnqs.log_psi(th, states, N, H)).sum() - 1.0) < 1e-12


def test_first_site_marginal_is_sigmoid_of_its_bias():
    N, H = 7, 11
    th = si.ar_params(N, H, seed=4, std=1.0)
    states = eloc.all_states(N)
    q = np.exp(2.0 * arnqs.log_psi(th, states, N, H))
    b2_0 = th[arnqs.num_params(N, H) - N]
    assert abs(q[states[:, 0] == 1].sum() - 1.0 / (1.0 + np.exp(-b2_0))) < 1e-12


def test_grad_against_finite_differences():
    N, H = 6, 10
    th = si.ar_params(N, H, seed=5, std=0.8)
    x = si.random_bits(5, N, seed=6)
    O = arnqs.grad_log_psi(th, x, N, H)
    eps = 1e-6
    fd = np.zeros_like(O)
    for k in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        fd[:, k] = (arnqs.log_psi(tp, x, N, H) - arnqs.log_psi(tm, x, N, H)) / (2 * eps)
    # ReLU kinks are measure-zero at these random parameters
    assert np.max(np.abs(O - fd)) < 1e-7


@pytest.mark.parametrize("kind,Lx,Ly", [("tfim", 8, 1), ("tfim", 3, 3), ("heisenberg", 3, 3)])
def test_energy_from_local_energies_matches_kronecker(kind, Lx, Ly):
    N = Lx * Ly
    H = 12
    th = si.ar_params(N, H, seed=7, std=0.7)
    f = lambda X: arnqs.log_psi(th, X, N, H).astype(np.complex128)
    E, p, el, states = eloc.exact_expectation(f, kind, N, Lx, Ly, True, 1.0, h=0.9)
    codes = (states.astype(np.int64) << np.arange(N)).sum(1)
    v = np.zeros(2 ** N)
    v[kron_ref.code_to_kron(codes, N)] = np.exp(arnqs.log_psi(th, states, N, H))
    Hk = kron_ref.tfim(Lx, Ly, True, 1.0, 0.9) if kind == "tfim" else kron_ref.heisenberg(Lx, Ly, True, 1.0)
    assert abs(v @ v - 1.0) < 1e-12
    assert abs(E - np.vdot(v, Hk @ v)) < 1e-10


def test_direct_samples_follow_q():
    N, H = 4, 6
    th = si.ar_params(N, H, seed=8, std=1.0)
    x, lp = arnqs.sample(th, 20000, N, H, seed=9, counter=0)
    assert np.allclose(lp, arnqs.log_psi(th, x, N, H), atol=1e-12)
    codes = (x.astype(np.int64) << np.arange(N)).sum(1)
    obs = np.bincount(codes, minlength=2 ** N)
    q = np.exp(2.0 * arnqs.log_psi(th, eloc.all_states(N), N, H))
    chi2 = np.sum((obs - 20000 * q) ** 2 / (20000 * q))
    assert stats.chi2.sf(chi2, 2 ** N - 1) > 1e-3
    x2, _ = arnqs.sample(th, 64, N, H, seed=9, counter=1)
    assert not np.array_equal(x2, x[:64])
