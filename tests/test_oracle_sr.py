"""Pins of oracle.sr and oracle.ess: exact-energy gradient identity, the
Fubini-Study (fidelity) form of the Fisher diagonal, LAPACK solves and
factorisations, limits of the diagonal shift, and the AR(1) autocorrelation."""
import numpy as np
import pytest

from oracle import sr, rbm, eloc, ess
import synth_inputs as si


def _exact_energy(p, n, nh, kind="tfim", h=1.0):
    f = lambda x: rbm.log_psi(p, x, nh)
    E, prob, el, states = eloc.exact_expectation(f, kind, n, n, 1, True, 1.0, h)
    return E.real, prob, el, states


def test_force_is_half_the_exact_energy_gradient():
    # eq:energy_gradient: dE/dRe theta_k = 2 Re F_k; holomorphy adds dE/dIm theta_k = 2 Im F_k
    n, nh = 6, 3
    p = si.rbm_params(n, nh, std=0.3, seed=21)
    E, prob, el, states = _exact_energy(p, n, nh)
    O = rbm.grad_log_psi(p, states, nh)
    S, F = sr.fisher_and_force(O, el, prob)
    eps = 1e-6
    for k in range(len(p)):
        d = np.zeros_like(p)
        d[k] = eps
        gr = (_exact_energy(p + d, n, nh)[0] - _exact_energy(p - d, n, nh)[0]) / (2 * eps)
        gi = (_exact_energy(p + 1j * d, n, nh)[0] - _exact_energy(p - 1j * d, n, nh)[0]) / (2 * eps)
        assert abs(gr - 2 * F[k].real) < 1e-7
        assert abs(gi - 2 * F[k].imag) < 1e-7


def test_fisher_diagonal_is_fidelity_curvature():
    # S is the Fubini-Study metric: 1 - |<psi|psi_eps>|^2/(|psi|^2 |psi_eps|^2) = eps^2 S_kk + O(eps^4)
    n, nh = 6, 4
    p = si.rbm_params(n, nh, std=0.4, seed=22)
    states = eloc.all_states(n)
    E, prob, el, _ = _exact_energy(p, n, nh)
    O = rbm.grad_log_psi(p, states, nh)
    S, _ = sr.fisher_and_force(O, el, prob)
    eps = 1e-4
    v0 = np.exp(rbm.log_psi(p, states, nh))
    def one_minus_fid(v1):
        # |a|^2 |b|^2 - |<a,b>|^2 = 1/2 sum_ij |a_i b_j - a_j b_i|^2 (Lagrange; no cancellation)
        cross = v0[:, None] * v1[None, :] - v0[None, :] * v1[:, None]
        return 0.5 * np.sum(np.abs(cross) ** 2) / (np.vdot(v0, v0).real * np.vdot(v1, v1).real)

    for k in range(0, len(p), 3):
        d = np.zeros_like(p)
        d[k] = eps
        # the eps^3 term is odd in eps: average +eps and -eps
        curv = (one_minus_fid(np.exp(rbm.log_psi(p + d, states, nh)))
                + one_minus_fid(np.exp(rbm.log_psi(p - d, states, nh)))) / (2 * eps ** 2)
        assert abs(curv - S[k, k].real) < 1e-6 * max(1.0, S[k, k].real)


def test_S_hermitian_psd_and_rank():
    n, nh, ns = 8, 8, 40
    p = si.rbm_params(n, nh, std=0.3, seed=23)
    bits = si.random_bits(ns, n, seed=1)
    O = rbm.grad_log_psi(p, bits, nh)
    el = np.random.default_rng(0).normal(size=ns) + 0j
    S, F = sr.fisher_and_force(O, el)
    assert np.allclose(S, S.conj().T, atol=1e-15)
    lam = np.linalg.eigvalsh(S)
    assert lam.min() >= -1e-12 * np.abs(lam).max()
    assert np.linalg.matrix_rank(S, tol=1e-10 * lam.max()) <= ns - 1
    # the connected correlator equals the covariance of explicitly centred data
    Oc = O - O.mean(0)
    assert np.allclose(S, Oc.conj().T @ Oc / ns, atol=1e-14)


def test_cholesky_and_solve_match_lapack():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(30, 30)) + 1j * rng.normal(size=(30, 30))
    A = A @ A.conj().T + 30 * np.eye(30)
    L, fail, piv = sr.cholesky(A)
    assert fail == -1
    assert np.allclose(L, np.linalg.cholesky(A), atol=1e-12)
    b = rng.normal(size=30) + 1j * rng.normal(size=30)
    x = sr.back_sub_h(L, sr.forward_sub(L, b))
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-12)


@pytest.mark.parametrize("mode,gamma", [("complex", 1.0), ("complex", 1j), ("real", 1.0)])
def test_sr_solve_vs_lapack(mode, gamma):
    n, nh, ns = 6, 6, 200
    p = si.rbm_params(n, nh, std=0.3, seed=24)
    bits = si.random_bits(ns, n, seed=2)
    O = rbm.grad_log_psi(p, bits, nh)
    el = eloc.local_energy(lambda x: rbm.log_psi(p, x, nh), "tfim", bits, n, 1, True, 1.0, 1.0)
    x, info = sr.sr_solve(O, el, nu_rel=1e-2, mode=mode, gamma=gamma)
    S, F = sr.fisher_and_force(O, el)
    S = sr.project(S, mode)
    rhs = -sr.project(gamma * F, mode)
    St = S + 1e-2 * np.diag(np.diag(S))
    ref = np.linalg.solve(St, rhs)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref) * max(1.0, np.linalg.cond(St) * 1e-5)
    assert info["residual"] < 1e-12
    assert abs(info["e_mean"] - el.mean()) < 1e-12


def test_shift_limits_and_not_pd():
    n, nh, ns = 6, 6, 20
    p = si.rbm_params(n, nh, std=0.3, seed=25)
    bits = si.random_bits(ns, n, seed=3)
    O = rbm.grad_log_psi(p, bits, nh)
    el = np.random.default_rng(1).normal(size=ns) + 0.1j
    S, F = sr.fisher_and_force(O, el)
    # large shift: nu * x -> -F_k / S_kk (diagonal preconditioning)
    nu = 1e9
    x, _ = sr.sr_solve(O, el, nu_rel=nu)
    assert np.allclose(nu * x, -F / np.diag(S).real, rtol=1e-6, atol=1e-9)
    # nu = 0 with fewer samples than parameters: S is singular -> reported, not repaired
    x, info = sr.sr_solve(O, el, nu_rel=0.0)
    assert x is None and info["fail_index"] >= 0
    # additive shift alone makes it solvable
    x, info = sr.sr_solve(O, el, nu_rel=0.0, eps_abs=1e-3)
    assert x is not None and info["residual"] < 1e-10


def test_ar1_integrated_autocorrelation_time():
    rho, T, C = 0.8, 20000, 16
    rng = np.random.default_rng(5)
    x = np.zeros((T, C))
    e = rng.normal(size=(T, C))
    x[0] = e[0] / np.sqrt(1 - rho ** 2)
    for t in range(1, T):
        x[t] = rho * x[t - 1] + e[t]
    tau, W = ess.tau_int(x)
    exact = (1 + rho) / (2 * (1 - rho))
    assert abs(tau - exact) < 0.05 * exact
    assert abs(ess.batch_means_tau(x) - exact) < 0.15 * exact
    n_eff, _ = ess.ess(x)
    assert abs(n_eff - x.size / (2 * exact)) < 0.06 * x.size / (2 * exact)


def test_package_ess_matches_oracle_and_ar1():
    from paper_2108_03409_amd import stats as pstats
    rho, T, C = 0.9, 4000, 8
    rng = np.random.default_rng(6)
    x = np.zeros((T, C))
    e = rng.normal(size=(T, C))
    for t in range(1, T):
        x[t] = rho * x[t - 1] + e[t]
    assert np.allclose(pstats.autocorrelation_fft(x), ess.autocorrelation(x), atol=1e-10)
    t1, _ = pstats.tau_int(x)
    t2, _ = ess.tau_int(x)
    assert abs(t1 - t2) < 1e-8
    exact = (1 + rho) / (2 * (1 - rho))
    assert abs(t1 - exact) < 0.15 * exact


# ---- eigen-decomposition regularisations (Sec. 3.3) ----

def _eig_problem(ns=400, K=12, seed=3, cplx=True):
    rng = np.random.default_rng(seed)
    O = rng.normal(size=(ns, K)) + (1j * rng.normal(size=(ns, K)) if cplx else 0.0)
    O = O * np.logspace(0, -3, K)            # spread the spectrum of S
    e = rng.normal(size=ns) + 1j * rng.normal(size=ns) * 0.3 + O[:, 0].real
    return O, e


def test_eigen_solve_without_cutoff_is_the_cholesky_solve():
    O, e = _eig_problem()
    for mode, gamma in [("complex", 1.0), ("real", 1.0), ("complex", 1j)]:
        x_e, _ = sr.eigen_solve(O, e, nu_rel=1e-3, mode=mode, gamma=gamma)
        x_c, _ = sr.sr_solve(O, e, nu_rel=1e-3, mode=mode, gamma=gamma)
        assert np.linalg.norm(x_e - x_c) <= 1e-10 * np.linalg.norm(x_c)


def test_hard_cutoff_equals_library_pseudo_inverse():
    # numpy's pinv (singular values of the Hermitian matrix, relative cutoff) is an
    # independent route to the truncated inverse of eq:pinv_cutoff
    O, e = _eig_problem(seed=4)
    S, F = sr.fisher_and_force(O, e)
    lam = np.linalg.eigvalsh(S)
    r = np.abs(lam) / np.abs(lam).max()
    eps = np.sqrt(r[3] * r[4])                 # strictly between two eigenvalue ratios
    x, info = sr.eigen_solve(O, e, eps_pinv=eps)
    x_ref = np.linalg.pinv(S, rcond=eps, hermitian=True) @ (-F)
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert info["residual"] > 1e-6             # components were dropped


def test_soft_cutoff_values():
    # one eigen-direction at |lambda / lambda_1| = eps / 2: weight 1 / (1 + 2^6) of 1/lambda
    rng = np.random.default_rng(5)
    K = 6
    Q, _ = np.linalg.qr(rng.normal(size=(K, K)) + 1j * rng.normal(size=(K, K)))
    d = np.array([1.0, 0.5, 0.1, 1e-2, 1e-3, 1e-4])
    S = (Q * d) @ Q.conj().T
    # samples with exactly this S: rows sqrt(K) * sqrt(d_j) q_j^dagger with signs, mean zero
    O = np.concatenate([np.sqrt(K) * (Q * np.sqrt(d)).conj().T, -np.sqrt(K) * (Q * np.sqrt(d)).conj().T])
    e = np.concatenate([np.ones(K), -np.ones(K)])
    S_o, F_o = sr.fisher_and_force(O, e)
    assert np.allclose(S_o, S, atol=1e-13)
    eps = 2e-2                                  # lambda_4 / lambda_1 = 1e-2 = eps / 2
    x, info = sr.eigen_solve(O, e, eps_pinv=eps, soft=True)
    lam, V = np.linalg.eigh(S_o)
    rho = V.conj().T @ (-F_o)
    y = V.conj().T @ x
    for j in range(K):
        want = 1.0 / (lam[j] * (1.0 + (eps / (abs(lam[j]) / lam.max())) ** 6))
        assert abs(y[j] - want * rho[j]) <= 1e-9 * abs(rho[j] / lam[j]) + 1e-14
    j4 = np.argmin(np.abs(lam - 1e-2))
    assert abs(y[j4] / (rho[j4] / lam[j4]) - 1.0 / 65.0) < 1e-9
    assert abs(abs(y[np.argmin(np.abs(lam - 0.1))] / (rho[np.argmin(np.abs(lam - 0.1))] / 0.1)) - 1.0) < 1e-4


def test_snr_estimate_and_zero_signal():
    O, e = _eig_problem(ns=3000, K=5, seed=6)
    x, info = sr.eigen_solve(O, e, eps_snr=1.0)
    # the variance is the plain (ddof 0) variance of the per-sample eigen components
    S, F = sr.fisher_and_force(O, e)
    lam, V = np.linalg.eigh(S)
    Ob = O - O.mean(0)
    f = (e - e.mean())[:, None] * Ob.conj()
    P = f @ V.conj()
    assert np.allclose(info["var"], np.var(P, axis=0), rtol=1e-10)
    assert np.allclose(np.abs(info["rho"]), np.abs(P.mean(0)), rtol=1e-10)
    # replicas (K = 1, so the eigen-basis is fixed): the standard error predicts
    # the spread of rho over independent sample sets
    rng = np.random.default_rng(7)
    rhos, sigs = [], []
    for _ in range(400):
        Orep = rng.normal(size=(300, 1)) + 1j * rng.normal(size=(300, 1))
        erep = 0.5 * Orep[:, 0].real + rng.normal(size=300)
        _, inf = sr.eigen_solve(Orep, erep)
        rhos.append(inf["rho"][0])
        sigs.append(np.abs(inf["rho"][0]) / inf["snr"][0])
    spread = np.std(np.array(rhos))
    assert abs(np.mean(sigs) / spread - 1.0) < 0.12
    # a component with exactly zero signal has SNR 0 and is dropped
    O2 = np.zeros((4, 2), dtype=complex)
    O2[:, 0] = [1, -1, 1, -1]
    O2[:, 1] = [1, 1, -1, -1]
    e2 = np.array([1.0, -1.0, 1.0, -1.0])       # correlated with column 0 only
    x2, inf2 = sr.eigen_solve(O2, e2, eps_snr=0.5)
    assert np.min(inf2["snr"]) == 0.0
    y2 = np.linalg.eigh(sr.fisher_and_force(O2, e2)[0])[1].conj().T @ x2
    assert abs(y2[np.argmin(inf2["snr"])]) == 0.0


# ---- Im projection (eq:tdvp_im): real parameters, antisymmetric Im S ----

def test_imag_mode_hard_cutoff_equals_svd_pseudo_inverse():
    # numpy's SVD-based pinv of the real antisymmetric Im S (singular values =
    # |eigenvalues of i Im S|) is an independent route to the truncated inverse
    O, e = _eig_problem(ns=500, K=11, seed=21)        # odd K: Im S has a zero eigenvalue
    for gamma in (1j, 1.0, 0.3 - 0.7j):
        S, F = sr.fisher_and_force(O, e)
        A = S.imag
        assert np.allclose(A, -A.T, atol=1e-15) and np.max(np.abs(np.diag(A))) <= 1e-15
        sv = np.sort(np.linalg.svd(A, compute_uv=False))[::-1]
        eps = np.sqrt(sv[5] * sv[6]) / sv[0]          # strictly between two singular-value pairs
        x, info = sr.eigen_solve(O, e, mode="imag", gamma=gamma, eps_pinv=eps)
        x_ref = np.linalg.pinv(A, rcond=eps) @ (-(gamma * F).imag)
        assert np.max(np.abs(x.imag)) == 0.0
        assert np.linalg.norm(x.real - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
        # eigenvalues of i Im S come in +- pairs
        lam = info["evals"]
        assert np.allclose(np.sort(lam), np.sort(-lam), atol=1e-12 * np.abs(lam).max())


def test_imag_mode_on_real_parametrisation_equals_holomorphic_solve():
    # A holomorphic network written with real parameters (Re p, Im p) has the
    # log-derivatives O' = [O, i O].  Its Im-projected equation Im[S'] q = Im[-i F']
    # reads  Im S u + Re S v = -Re F  and  -Re S u + Im S v = -Im F, the real and
    # imaginary parts of S (u + i v) = -i F: the holomorphic real-time equation.
    O, e = _eig_problem(ns=600, K=9, seed=22)
    Op = np.concatenate([O, 1j * O], axis=1)
    q, info = sr.eigen_solve(Op, e, mode="imag", gamma=1j, eps_pinv=1e-12)
    x_c, _ = sr.eigen_solve(O, e, mode="complex", gamma=1j, eps_pinv=1e-12)
    K = O.shape[1]
    z = q[:K].real + 1j * q[K:].real
    assert np.linalg.norm(z - x_c) <= 1e-9 * np.linalg.norm(x_c)
    # the spectrum of i Im S' is +- that of S
    lam_s = np.linalg.eigvalsh(sr.fisher_and_force(O, e)[0])
    assert np.allclose(np.sort(np.abs(info["evals"])), np.sort(np.concatenate([lam_s, lam_s])),
                       rtol=1e-9, atol=1e-14)


def test_imag_mode_conserves_energy_to_first_order():
    # dE/dt = sum_k dE/dtheta_k x_k = 2 Re F . x with real parameters
    # (eq:energy_gradient); with gamma = i the Im equation gives
    # x = -A^+ Re F, A^+ antisymmetric, so Re F . x = 0 for every cutoff
    # (pairs +-lambda share their cutoff and SNR factors)
    rng = np.random.default_rng(23)
    ns, K = 800, 10
    O = rng.normal(size=(ns, K)) + 1j * rng.normal(size=(ns, K))   # non-holomorphic: arbitrary complex O
    e = rng.normal(size=ns) + 0.5j * rng.normal(size=ns) + 0.3 * O[:, 2] + 0.2j * O[:, 5].real
    S, F = sr.fisher_and_force(O, e)
    for kw in (dict(eps_pinv=1e-10), dict(eps_pinv=0.05, soft=True), dict(eps_pinv=1e-8, eps_snr=2.0)):
        x, _ = sr.eigen_solve(O, e, mode="imag", gamma=1j, **kw)
        assert abs(np.dot(F.real, x.real)) <= 1e-12 * np.linalg.norm(F.real) * np.linalg.norm(x.real)
        # the Re projection does not conserve it
    x_re, _ = sr.eigen_solve(O, e, mode="real", gamma=1j, eps_pinv=1e-10)
    assert abs(np.dot(F.real, x_re.real)) > 1e-3 * np.linalg.norm(F.real) * np.linalg.norm(x_re.real)


def test_imag_mode_refuses_additive_shift():
    O, e = _eig_problem(ns=50, K=4, seed=24)
    with pytest.raises(ValueError):
        sr.eigen_solve(O, e, mode="imag", eps_abs=1e-3, eps_pinv=1e-8)


# ---- per-row S and F alone (the large-K parity path) ----

def test_fisher_rows_and_force_equal_the_full_matrices():
    # the row-at-a-time S and the S-free F are the same connected correlators
    # as fisher_and_force (itself pinned by the energy gradient and the
    # Fubini-Study curvature above), with and without weights
    rng = np.random.default_rng(31)
    ns, K = 257, 40
    O = rng.normal(size=(ns, K)) + 1j * rng.normal(size=(ns, K)) + 0.3
    e = rng.normal(size=ns) + 1j * rng.normal(size=ns)
    for w in (None, rng.uniform(0.1, 2.0, size=ns)):
        S, F = sr.fisher_and_force(O, e, w)
        rows = [0, 7, 39, 13]
        assert np.allclose(sr.fisher_rows(O, rows, w), S[rows], rtol=0, atol=1e-13)
        assert np.allclose(sr.force(O, e, w), F, rtol=0, atol=1e-13)
