"""Quantum Fisher matrix, force vector and the regularised TDVP / SR solve.

Paper:
  * eq:qfm            S_kk' = <O_k^* O_k'>^c  (connected: <AB> - <A><B>)
  * eq:force_vector   F_k   = <E_loc O_k^*>^c
  * eq:energy_gradient  dE/dtheta_k = 2 Re F_k  (SR step eq:stochastic_reconfiguration)
  * eq:tdvp_util      [[S]] theta_dot = -[[gamma F]],  gamma in {1, i},
                      [[.]] = identity (holomorphic nets), Re or Im
  * Sec. 3.1 "Diagonal shift": S~_kk' = (1 + nu delta_kk') S_kk'.

Readings:
  * expectation values are plain empirical means (1/N_s) over the samples
    (eq:Oloc_mean), or sum_n w_n (.) with normalised weights w (the exact
    enumeration path, where w = p(s));
  * an optional additive shift eps_abs * I is applied after the relative one;
  * the solve is a textbook Cholesky factorisation S~ = L L^H (Golub & Van
    Loan, "Matrix Computations", Alg. 4.2.1, column form) followed by forward
    and back substitution; a non-positive pivot is reported, never repaired;
  * the factor 2 of the SR gradient is absorbed into the step size: the
    solve returns x with [[S~]] x = -[[gamma F]].

Eigen-decomposition regularisations (Sec. 3.3, ``eigen_solve``): with
S~ = V diag(lambda) V^dagger (numpy's Hermitian eigensolver as the library
step), rho = V^dagger (-[[gamma F]]) and x = V diag(lambda^+) rho, where
lambda^+ follows the hard cutoff (eq:pinv_cutoff), the soft cutoff, and the
signal-to-noise factor of the "eliminating noisy contributions" subsection.
Readings: lambda_1 is the eigenvalue of largest modulus; the cutoffs combine
as a product of the pinv inverse and the SNR factor; a zero eigenvalue gets
lambda^+ = 0; the SNR of rho_j is |rho_j| over the standard error of a mean of
N_s samples, sqrt(var_j / N_s), with var_j the weighted variance of the
eigen-basis components of the per-sample terms
f_n = [[gamma (E_n - <E>) conj(O_n - <O>)]] whose weighted sum is [[gamma F]].

The Im projection (eq:tdvp_im, real parameters of a non-holomorphic network)
gives Im[S~] x = -Im[gamma F] with A = Im S~ real and antisymmetric (zero
diagonal, so the relative shift does nothing and an additive one would break
the antisymmetry: it is refused).  A has no real eigendecomposition; the
Hermitian matrix H = i A does (eigenvalues in +- pairs), and A x = b is
H x = i b.  The cutoffs of Sec. 3.3 act on the eigenvalues of H, i.e. on the
singular values of A (pairs are kept or dropped together, so x stays real).
"""
from __future__ import annotations

import numpy as np


def _weights(n, weights):
    if weights is None:
        return np.full(n, 1.0 / n)
    w = np.asarray(weights, dtype=np.float64)
    return w / w.sum()


def energy_stats(eloc, weights=None):
    """Mean and variance of E_loc: (<E>, <|E - <E>|^2>)."""
    e = np.asarray(eloc, dtype=np.complex128)
    w = _weights(len(e), weights)
    mean = np.sum(w * e)
    var = np.sum(w * np.abs(e - mean) ** 2)
    return mean, var


def fisher_and_force(O, eloc, weights=None):
    """S (K x K) and F (K) from per-sample log-derivatives O (N_s x K)."""
    O = np.asarray(O, dtype=np.complex128)
    e = np.asarray(eloc, dtype=np.complex128)
    w = _weights(O.shape[0], weights)
    mean_O = w @ O                                   # <O_k>
    mean_E = np.sum(w * e)                           # <E_loc>
    S = (O.conj().T * w[None, :]) @ O - np.outer(mean_O.conj(), mean_O)
    F = (O.conj().T * w[None, :]) @ e - mean_O.conj() * mean_E
    return S, F


def force(O, eloc, weights=None):
    """F alone (eq:force_vector), F_k = <conj(O_k) E> - <conj(O_k)><E>, for
    sample counts where forming S would not fit."""
    O = np.asarray(O, dtype=np.complex128)
    e = np.asarray(eloc, dtype=np.complex128)
    w = _weights(O.shape[0], weights)
    mean_O = w @ O
    return (w * e) @ O.conj() - mean_O.conj() * np.sum(w * e)


def fisher_rows(O, rows, weights=None):
    """Selected rows of S (eq:qfm), S_rk' = <conj(O_r) O_k'> - <conj(O_r)><O_k'>,
    one row at a time: (len(rows), K)."""
    O = np.asarray(O, dtype=np.complex128)
    w = _weights(O.shape[0], weights)
    mean_O = w @ O
    out = np.empty((len(rows), O.shape[1]), dtype=np.complex128)
    for i, r in enumerate(rows):
        out[i] = (w * O[:, r].conj()) @ O - mean_O[r].conj() * mean_O
    return out


def project(A, mode):
    if mode == "complex":
        return A
    if mode == "real":
        return A.real.astype(np.complex128)
    if mode == "imag":
        return A.imag.astype(np.complex128)
    raise ValueError(mode)


def shifted(S, nu_rel, eps_abs=0.0):
    """S~ = S + nu_rel * diag(S) + eps_abs * I (the paper's (1 + nu delta) S)."""
    St = np.array(S, dtype=np.complex128, copy=True)
    d = np.arange(St.shape[0])
    St[d, d] = St[d, d] * (1.0 + nu_rel) + eps_abs
    return St


def cholesky(A):
    """Lower-triangular L with A = L L^H, column by column.

    Returns (L, fail_index, min_pivot); fail_index is -1 on success, else the
    first column whose pivot A_jj - sum_k |L_jk|^2 is not positive (and L is
    then only valid in its first fail_index columns)."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    L = np.zeros_like(A)
    min_pivot = np.inf
    for j in range(n):
        d = A[j, j].real - np.sum(np.abs(L[j, :j]) ** 2)
        min_pivot = min(min_pivot, d)
        if not d > 0.0:
            return L, j, min_pivot
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j].conj()) / L[j, j]
    return L, -1, min_pivot


def forward_sub(L, b):
    """Solve L y = b for lower-triangular L."""
    n = L.shape[0]
    y = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        y[i] = (b[i] - L[i, :i] @ y[:i]) / L[i, i]
    return y


def back_sub_h(L, y):
    """Solve L^H x = y for lower-triangular L."""
    n = L.shape[0]
    x = np.zeros(n, dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - L[i + 1:, i].conj() @ x[i + 1:]) / L[i, i].conj()
    return x


def sr_solve(O, eloc, *, nu_rel=1e-3, eps_abs=0.0, mode="complex", gamma=1.0,
             weights=None):
    """One regularised SR / TDVP solve, following the steps of Algorithm 1
    after the local energies: S and F, shift, factorisation, two triangular
    solves.  Returns (x, info) with [[S~]] x = -[[gamma F]]."""
    S, F = fisher_and_force(O, eloc, weights)
    mean, var = energy_stats(eloc, weights)
    Sm = project(S, mode)
    rhs = -project(gamma * F, mode)
    St = shifted(Sm, nu_rel, eps_abs)
    L, fail, min_piv = cholesky(St)
    info = dict(e_mean=mean, e_var=var, fail_index=fail, min_pivot=min_piv)
    if fail >= 0:
        return None, info
    x = back_sub_h(L, forward_sub(L, rhs))
    info["residual"] = np.linalg.norm(St @ x - rhs) / max(np.linalg.norm(rhs), 1e-300)
    return x, info


def eigen_solve(O, eloc, *, nu_rel=0.0, eps_abs=0.0, mode="complex", gamma=1.0, weights=None,
                eps_pinv=0.0, soft=False, eps_snr=0.0):
    """Regularised solve through the eigendecomposition of S~; returns
    (x, info) with info['evals'] (ascending) and info['snr'] (same order).
    For mode "imag" the eigenvalues are those of i Im[S~] and x is real."""
    O = np.asarray(O, dtype=np.complex128)
    e = np.asarray(eloc, dtype=np.complex128)
    N = O.shape[0]
    w = _weights(N, weights)
    S, F = fisher_and_force(O, e, weights)
    if mode == "imag" and eps_abs != 0.0:
        raise ValueError("an additive shift breaks the antisymmetry of Im S")
    St = shifted(project(S, mode), nu_rel, eps_abs)
    rhs = -project(gamma * F, mode)
    # the Hermitian matrix that is decomposed, and the right-hand side in its frame
    Hm, rhs_h = (1j * St, 1j * rhs) if mode == "imag" else (St, rhs)
    lam, V = np.linalg.eigh(Hm)
    rho = V.conj().T @ rhs_h
    # per-sample terms and their eigen-basis components (plain definition)
    Ob = O - w @ O
    dE = e - np.sum(w * e)
    f = project(gamma * dE[:, None] * Ob.conj(), mode)       # (N, K), sum_n w_n f_n = [[gamma F]]
    if mode == "imag":
        f = 1j * f
    P = f @ V.conj()                                           # P_nj = sum_k f_nk conj(V_kj)
    mean_P = w @ P
    var = w @ (np.abs(P) ** 2) - np.abs(mean_P) ** 2
    sig = np.sqrt(np.maximum(var, 0.0) / N)
    with np.errstate(divide="ignore", invalid="ignore"):
        snr = np.where(sig > 0, np.abs(rho) / sig, np.where(np.abs(rho) > 0, np.inf, 0.0))
    lam1 = np.max(np.abs(lam))
    inv = np.zeros(len(lam))
    for j, l in enumerate(lam):
        if l == 0.0:
            continue
        r = abs(l) / lam1
        if eps_pinv <= 0.0:
            inv[j] = 1.0 / l
        elif soft:
            inv[j] = 1.0 / (l * (1.0 + (eps_pinv / r) ** 6))
        else:
            inv[j] = 0.0 if r < eps_pinv else 1.0 / l
        if eps_snr > 0.0:
            if snr[j] == 0.0:
                inv[j] = 0.0
            elif np.isfinite(snr[j]):
                inv[j] /= 1.0 + (eps_snr / snr[j]) ** 6
    x = V @ (inv * rho)
    if mode == "imag":
        x = x.real.astype(np.complex128)
    mean, evar = energy_stats(e, weights)
    res = np.linalg.norm(St @ x - rhs) / max(np.linalg.norm(rhs), 1e-300)
    return x, dict(evals=lam, snr=snr, rho=rho, var=var, e_mean=mean, e_var=evar, residual=res)
