"""Device Hermitian eigensolver and the eigen-decomposition regularisations of
the TDVP equation (pseudo-inverse cutoffs, signal-to-noise filter; Sec. 3.3)
through the C ABI, against numpy's eigensolver and oracle.sr.eigen_solve."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import rbm as orbm, eloc as oeloc, sr as osr
from gpu_common import DEV, dev_c128, flush

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2108_03409_amd import nqsvmc as V  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    return V.Context(0)


def _hermitian(K, seed, spread=6.0, cplx=True):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(K + 3, K)) + (1j * rng.normal(size=(K + 3, K)) if cplx else 0.0)
    X = X * np.logspace(0, -spread / 2, K)
    return X.conj().T @ X


@pytest.mark.parametrize("K,cplx", [(1, True), (2, True), (7, True), (64, False), (333, True), (1000, True),
                                    (2048, True)])
def test_eigh_matches_numpy(ctx, K, cplx):
    flush(f"eigh K={K}")
    A = _hermitian(K, seed=K, cplx=cplx)
    ev, Vm, sweeps = V.eigh(ctx, dev_c128(A))
    ev, Vm = ev.cpu().numpy(), Vm.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    nrm = np.abs(ref).max()
    assert np.max(np.abs(np.sort(ev) - ref)) <= 1e-12 * nrm
    assert np.linalg.norm((Vm * ev) @ Vm.conj().T - A) <= 1e-12 * np.linalg.norm(A)
    assert np.linalg.norm(Vm.conj().T @ Vm - np.eye(K)) <= 1e-11
    assert sweeps <= 20


def _problem(N, Nh, ns, std, seed, cplx=True):
    p = si.rbm_params(N, Nh, std=std, is_complex=cplx, seed=seed)
    bits = si.random_bits(ns, N, seed=seed + 1)
    O = orbm.grad_log_psi(p, bits, Nh)
    el = oeloc.local_energy(lambda x: orbm.log_psi(p, x, Nh), "tfim", bits, N, 1, True, 1.0, 1.0)
    return O, el


def _cut_between(O, el, mode, nu, frac):
    """a relative cutoff halfway (geometrically) between two eigenvalue ratios"""
    S, _ = osr.fisher_and_force(O, el)
    lam = np.linalg.eigvalsh(osr.shifted(osr.project(S, mode), nu, 0.0))
    r = np.sort(np.abs(lam) / np.abs(lam).max())
    j = int(frac * len(r))
    return float(np.sqrt(r[j] * r[j + 1]))


CASES = [
    # N, Nh, ns, mode, gamma, nu, pinv (frac or 0), soft, snr, weighted
    (8, 16, 400, "complex", 1.0, 1e-3, 0.0, False, 0.0, False),   # no cutoff: the Cholesky solution
    (8, 16, 400, "complex", 1.0, 0.0, 0.3, False, 0.0, False),    # hard cutoff
    (8, 16, 400, "complex", 1j, 0.0, 0.3, True, 0.0, True),       # soft cutoff, real time, weighted
    (10, 10, 1000, "real", 1.0, 0.0, 0.2, True, 2.0, False),      # soft + SNR, real projection
    (12, 20, 3000, "complex", 1j, 0.0, 0.0, False, 1.5, False),   # SNR only (K = 272)
]


@pytest.mark.parametrize("N,Nh,ns,mode,gamma,nu,frac,soft,snr,weighted", CASES)
def test_sr_solve_eig_matches_oracle(ctx, N, Nh, ns, mode, gamma, nu, frac, soft, snr, weighted):
    flush(f"sr eig N={N} Nh={Nh} ns={ns} mode={mode} gamma={gamma} frac={frac} soft={soft} snr={snr}")
    O, el = _problem(N, Nh, ns, 0.2, seed=N * Nh + 1, cplx=(mode != "real"))
    w = np.random.default_rng(9).uniform(0.5, 1.5, ns) if weighted else None
    eps = _cut_between(O, el, mode, nu, frac) if frac > 0 else 0.0
    x_ref, info_ref = osr.eigen_solve(O, el, nu_rel=nu, mode=mode, gamma=gamma, weights=w, eps_pinv=eps, soft=soft,
                                      eps_snr=snr)
    x, info = V.sr_solve_eig(ctx, dev_c128(O), dev_c128(el), weights=None if w is None else
                             torch.from_numpy(w).to(DEV), nu_rel=nu, mode=V.SR_REAL if mode == "real" else V.SR_COMPLEX,
                             gamma=gamma, eps_pinv=eps, soft=soft, eps_snr=snr, want_snr=True)
    x = x.cpu().numpy()
    ev = np.sort(info["evals"].cpu().numpy())
    assert np.max(np.abs(ev - info_ref["evals"])) <= 1e-12 * np.abs(info_ref["evals"]).max()
    lam = info_ref["evals"]
    # conditioning of the kept part bounds the error of x
    kept = np.abs(lam) >= max(eps, 1e-300) * np.abs(lam).max()
    kappa = np.abs(lam).max() / np.abs(lam[kept]).min()
    err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    assert err <= max(1e-11, 1e-14 * kappa * 100), (err, kappa)
    s_ref = np.sort(info_ref["snr"])
    s_got = np.sort(info["snr"].cpu().numpy())
    fin = np.isfinite(s_ref)
    assert np.allclose(s_got[fin], s_ref[fin], rtol=1e-8, atol=1e-12)
    assert abs(info["e_mean"] - info_ref["e_mean"]) < 1e-12 * max(1, abs(info_ref["e_mean"]))
    assert abs(info["residual"] - info_ref["residual"]) <= 1e-8 + 1e-6 * info_ref["residual"]


@pytest.mark.parametrize("N,Nh,ns", [(12, 48, 333), (9, 21, 1001)])
def test_gram_c64_eigenvalues_within_bound(ctx, N, Nh, ns):
    # S from complex64 O on the float32 matrix cores (three real products per
    # complex term).  K = 636 (even) takes the direct-to-LDS Gram kernel, K = 219
    # (odd) the register-staged one; both sample counts are ragged.  Weyl:
    # |d lambda| <= ||dS||_2 <= ||dS||_F, with |dS_kk'| <= 2 (N_s + 8) u M_kk',
    # M = |Obar|^T |Obar| (the factor 2 covers the imaginary part of the
    # three-product form, whose terms are bounded by 2 |Obar_k| |Obar_k'|).
    flush(f"gram c64 eigenvalues N={N} Nh={Nh} ns={ns}")
    O, el = _problem(N, Nh, ns, 0.2, seed=N + Nh, cplx=True)
    O32 = O.astype(np.complex64)
    Od = O32.astype(np.complex128)
    _, info_ref = osr.eigen_solve(Od, el, nu_rel=1e-2, mode="complex", eps_pinv=1e-8)
    _, info = V.sr_solve_eig(ctx, torch.from_numpy(O32).to(DEV), dev_c128(el), nu_rel=1e-2, mode=V.SR_COMPLEX,
                             eps_pinv=1e-8)
    ev = np.sort(info["evals"].cpu().numpy())
    Ob = (Od - Od.mean(axis=0)) / np.sqrt(ns)
    M = np.abs(Ob).T @ np.abs(Ob)
    bound = 1.01 * np.linalg.norm(2.0 * (ns + 8) * 2.0 ** -24 * M)
    err = np.max(np.abs(ev - info_ref["evals"]))
    assert err <= bound, (err, bound)
    # a wrong sign or a dropped term in the three-product form moves the
    # spectrum by O(||S||), far beyond float32 rounding
    assert err <= 1e-5 * np.abs(info_ref["evals"]).max(), err


def test_sr_solve_eig_real_o_float32(ctx):
    # real log-derivatives in float32: S from the matrix cores, eigen solve in float64
    flush("sr eig real O f32")
    O, el = _problem(10, 10, 2001, 0.2, seed=31, cplx=False)
    Or = O.real.astype(np.float32)
    x_ref, info_ref = osr.eigen_solve(Or.astype(np.float64).astype(np.complex128), el, nu_rel=1e-2, mode="real",
                                      eps_pinv=1e-6, soft=True)
    x, info = V.sr_solve_eig(ctx, torch.from_numpy(Or).to(DEV), dev_c128(el), nu_rel=1e-2, mode=V.SR_REAL,
                             eps_pinv=1e-6, soft=True)
    x = x.cpu().numpy()
    lam = info_ref["evals"]
    kappa = np.abs(lam).max() / np.abs(lam).min()
    err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    assert err <= kappa * 4 * (np.sqrt(2001) * 2.0 ** -24 + 2.0 ** -24) + 1e-12


def test_pinv_tdvp_follows_exact_evolution(ctx):
    # exact TDVP (all 2^6 configurations) with the soft pseudo-inverse instead of
    # an additive shift: the cutoff only removes directions that do not change psi
    import scipy.linalg as sla
    from kron_ref import tfim as kron_tfim, code_to_kron
    from oracle.eloc import all_states
    from gpu_common import dev_bits
    from paper_2108_03409_amd.driver import TDVP
    flush("real-time TDVP with the soft pseudo-inverse, N = 6")
    N, Nh, h, T, dt = 6, 12, 1.0, 0.3, 0.005
    model = V.Model.rbm(ctx, N, Nh, True)
    ham = V.Hamiltonian.tfim(ctx, N, 1, True, 1.0, h)
    p0 = si.rbm_params(N, Nh, std=0.15, is_complex=True, seed=21)
    states = all_states(N)
    s_dev = dev_bits(si.pack_bits(states))
    tdvp = TDVP(ctx, model, ham, torch.from_numpy(p0.astype(np.complex128)).to(DEV), real_time=True, eps_abs=0.0,
                exact_states=s_dev, eps_pinv=1e-8, soft_pinv=True)
    for _ in range(int(round(T / dt))):
        tdvp.step(dt, "heun")
    codes = (states.astype(np.int64) << np.arange(N)).sum(1)
    idx = code_to_kron(codes, N)

    def vec(p):
        v = np.zeros(2 ** N, dtype=complex)
        v[idx] = np.exp(orbm.log_psi(p, states, Nh))
        return v / np.linalg.norm(v)

    Hk = kron_tfim(N, 1, True, 1.0, h).toarray()
    v_exact = sla.expm(-1j * T * Hk) @ vec(p0)
    v_t = vec(tdvp.theta.cpu().numpy())
    fid = abs(np.vdot(v_exact, v_t)) ** 2
    flush(f"  fidelity {fid:.8f}")
    assert fid > 0.9999


@pytest.mark.parametrize("dt", ["c128", "c64", "f64", "f32"])
def test_fisher_quad_matches_oracle(ctx, dt):
    flush(f"fisher quad {dt}")
    cplx = dt.startswith("c")
    O, el = _problem(9, 21, 777, 0.2, seed=41, cplx=cplx)
    w = np.random.default_rng(2).uniform(0.5, 1.5, 777)
    v = np.random.default_rng(3).normal(size=O.shape[1]) + 1j * np.random.default_rng(4).normal(size=O.shape[1])
    On = {"c128": O, "c64": O.astype(np.complex64), "f64": O.real, "f32": O.real.astype(np.float32)}[dt]
    S, _ = osr.fisher_and_force(np.asarray(On).astype(np.complex128), el, w)
    ref = float(np.real(np.vdot(v, S @ v)))
    got = V.fisher_quad(ctx, torch.from_numpy(np.ascontiguousarray(On)).to(DEV), dev_c128(v),
                        weights=torch.from_numpy(w).to(DEV))
    assert abs(got - ref) <= 1e-11 * abs(ref)


def test_adaptive_heun_tdvp_follows_exact_evolution(ctx):
    # exact TDVP with the adaptive Heun stepper and the Fisher norm: the step
    # size grows from a small start while the state tracks exp(-iHt) psi(0)
    import scipy.linalg as sla
    from kron_ref import tfim as kron_tfim, code_to_kron
    from oracle.eloc import all_states
    from gpu_common import dev_bits
    from paper_2108_03409_amd.driver import TDVP, AdaptiveHeun
    flush("adaptive Heun TDVP, N = 6")
    N, Nh, h, T = 6, 12, 1.0, 0.3
    model = V.Model.rbm(ctx, N, Nh, True)
    ham = V.Hamiltonian.tfim(ctx, N, 1, True, 1.0, h)
    p0 = si.rbm_params(N, Nh, std=0.15, is_complex=True, seed=21)
    states = all_states(N)
    tdvp = TDVP(ctx, model, ham, torch.from_numpy(p0.astype(np.complex128)).to(DEV), real_time=True,
                eps_abs=1e-8, exact_states=dev_bits(si.pack_bits(states)))
    st = AdaptiveHeun(dt=1e-4, tol=1e-6)
    dts = []
    while tdvp.t < T - 1e-12:
        st.dt = min(st.dt, T - tdvp.t)
        dts.append(tdvp.step_adaptive(st)["dt"])
    codes = (states.astype(np.int64) << np.arange(N)).sum(1)
    idx = code_to_kron(codes, N)

    def vec(p):
        v = np.zeros(2 ** N, dtype=complex)
        v[idx] = np.exp(orbm.log_psi(p, states, Nh))
        return v / np.linalg.norm(v)

    Hk = kron_tfim(N, 1, True, 1.0, h).toarray()
    v_exact = sla.expm(-1j * tdvp.t * Hk) @ vec(p0)
    fid = abs(np.vdot(v_exact, vec(tdvp.theta.cpu().numpy()))) ** 2
    flush(f"  steps {len(dts)}  dt {dts[0]:.1e} -> {max(dts):.1e}  rejected {st.n_rejected}  fidelity {fid:.8f}")
    assert fid > 0.9999
    assert max(dts) > 10 * dts[0]


# ---- the Im projection of the TDVP equation (eq:tdvp_im, Sec. 2.3) --------

def _cut_between_imag(O, el, frac, w=None):
    """a relative cutoff between two distinct moduli of the eigenvalues of i Im S
    (they come in +- pairs: a cut never separates a pair)"""
    S, _ = osr.fisher_and_force(O, el, w)
    lam = np.linalg.eigvalsh(1j * osr.project(S, "imag"))
    r = np.sort(np.abs(lam) / np.abs(lam).max())
    j = int(frac * len(r))
    while r[j + 1] <= r[j] * (1 + 1e-6):
        j += 1
    return float(np.sqrt(r[j] * r[j + 1]))


IMAG_CASES = [
    # N, Nh, ns, gamma, pinv frac, soft, snr, weighted  (O: complex log-derivatives of real parameters)
    (8, 16, 400, 1j, 0.3, False, 0.0, False),     # hard cutoff, real time: Im S x = -Re F
    (8, 16, 400, 1.0, 0.3, True, 0.0, True),      # soft cutoff, gamma = 1, weighted
    (9, 12, 1000, 1j, 0.2, True, 2.0, False),     # soft + SNR, odd K (one zero eigenvalue)
]


@pytest.mark.parametrize("N,Nh,ns,gamma,frac,soft,snr,weighted", IMAG_CASES)
def test_sr_solve_eig_imag_matches_oracle(ctx, N, Nh, ns, gamma, frac, soft, snr, weighted):
    flush(f"sr eig imag N={N} Nh={Nh} ns={ns} gamma={gamma} frac={frac} soft={soft} snr={snr}")
    O, el = _problem(N, Nh, ns, 0.2, seed=N * Nh + 3, cplx=True)
    w = np.random.default_rng(10).uniform(0.5, 1.5, ns) if weighted else None
    eps = _cut_between_imag(O, el, frac, w)
    x_ref, info_ref = osr.eigen_solve(O, el, mode="imag", gamma=gamma, weights=w, eps_pinv=eps, soft=soft,
                                      eps_snr=snr)
    x, info = V.sr_solve_eig(ctx, dev_c128(O), dev_c128(el), weights=None if w is None else
                             torch.from_numpy(w).to(DEV), mode=V.SR_IMAG, gamma=gamma, eps_pinv=eps, soft=soft,
                             eps_snr=snr, want_snr=True)
    x = x.cpu().numpy()
    assert np.all(x.imag == 0)
    ev = np.sort(info["evals"].cpu().numpy())
    lam = info_ref["evals"]
    assert np.max(np.abs(ev - lam)) <= 1e-12 * np.abs(lam).max()
    kept = np.abs(lam) >= eps * np.abs(lam).max()
    kappa = np.abs(lam).max() / np.abs(lam[kept]).min()
    err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    assert err <= max(1e-11, 1e-14 * kappa * 100), (err, kappa)
    s_ref, s_got = np.sort(info_ref["snr"]), np.sort(info["snr"].cpu().numpy())
    fin = np.isfinite(s_ref)
    assert np.allclose(s_got[fin], s_ref[fin], rtol=1e-8, atol=1e-12)
    assert abs(info["residual"] - info_ref["residual"]) <= 1e-8 + 1e-6 * info_ref["residual"]
    # energy conservation of the Im form: Re F . x = 0 (x = A^+ b with A^+ antisymmetric)
    if gamma == 1j:
        _, F = osr.fisher_and_force(O, el, w)
        assert abs(np.dot(F.real, x.real)) <= 1e-12 * np.linalg.norm(F.real) * np.linalg.norm(x)


def test_sr_solve_eig_imag_refusals(ctx):
    O, el = _problem(6, 6, 50, 0.2, seed=2, cplx=True)
    with pytest.raises(V.VMCError):
        V.sr_solve_eig(ctx, dev_c128(O), dev_c128(el), mode=V.SR_IMAG, eps_abs=1e-3, eps_pinv=1e-8)
    with pytest.raises(V.VMCError):
        V.sr_solve_eig(ctx, torch.from_numpy(O.real.copy()).to(DEV), dev_c128(el), mode=V.SR_IMAG, eps_pinv=1e-8)
    with pytest.raises(V.VMCError):
        V.sr_solve(ctx, dev_c128(O), dev_c128(el), mode=V.SR_IMAG)


@pytest.mark.parametrize("eps_pinv,soft", [(0.0, False), (1e-3, False), (1e-3, True)])
def test_imag_form_of_holomorphic_net_is_the_complex_solve(ctx, eps_pinv, soft):
    # Sec. 2.3: solving the complex equation for complex parameters equals the Im
    # form for their real and imaginary parts, O_real = [O, i O]
    flush(f"imag form of a holomorphic net eps={eps_pinv} soft={soft}")
    O, el = _problem(8, 8, 500, 0.2, seed=77, cplx=True)
    K = O.shape[1]
    Or = np.concatenate([O, 1j * O], axis=1)
    xc, _ = V.sr_solve_eig(ctx, dev_c128(O), dev_c128(el), mode=V.SR_COMPLEX, gamma=1j, eps_pinv=eps_pinv,
                           soft=soft)
    xr, _ = V.sr_solve_eig(ctx, dev_c128(Or), dev_c128(el), mode=V.SR_IMAG, gamma=1j,
                           eps_pinv=eps_pinv if eps_pinv > 0 else 1e-12, soft=soft)
    xc, xr = xc.cpu().numpy(), xr.cpu().numpy().real
    err = np.linalg.norm(xr[:K] + 1j * xr[K:] - xc) / np.linalg.norm(xc)
    assert err <= 1e-9, err


def test_imag_form_conserves_energy_in_real_time(ctx):
    # a non-holomorphic network of real parameters: modulus and phase from two
    # real RBMs, log psi = l_A(s; a) + i l_B(s; b), O = [O_A, i O_B], started from
    # a = b.  Exact weights over all 2^6 configurations, Heun steps, pseudo-
    # inverse cutoff 1e-8, t = 0.1.  The Im form (eq:tdvp_im) conserves the
    # energy up to the integrator's error (which falls as dt^2: 4.7e-5 at
    # dt = 0.005, 1.1e-5 at 0.0025 with the oracle's solve); the Re form
    # (eq:tdvp_re) drifts by a step-independent 7e-4.
    from kron_ref import tfim as kron_tfim, code_to_kron
    from oracle.eloc import all_states
    from gpu_common import dev_bits
    N, Nh, h, T = 6, 1, 1.0, 0.1
    states = all_states(N)
    s_dev = dev_bits(si.pack_bits(states))
    idx = code_to_kron((states.astype(np.int64) << np.arange(N)).sum(1), N)
    Hk = kron_tfim(N, 1, True, 1.0, h).toarray()[np.ix_(idx, idx)]   # library code order
    mA = V.Model.rbm(ctx, N, Nh, False)
    mB = V.Model.rbm(ctx, N, Nh, False)
    p0 = si.rbm_params(N, Nh, std=0.3, is_complex=False, seed=51).real
    K = len(p0)

    def rhs(th, mode):
        mA.set_params(torch.from_numpy(th[:K].copy()).to(DEV))
        mB.set_params(torch.from_numpy(th[K:].copy()).to(DEV))
        lp = mA.log_psi(s_dev).real + 1j * mB.log_psi(s_dev).real
        O = torch.cat([mA.grad_log_psi(s_dev).real.to(torch.complex128),
                       1j * mB.grad_log_psi(s_dev).real.to(torch.complex128)], dim=1).contiguous()
        lph = lp.cpu().numpy()
        psi = np.exp(lph - lph.real.max())
        el = (Hk @ psi) / psi
        w = np.abs(psi) ** 2
        x, _ = V.sr_solve_eig(ctx, O, dev_c128(el), weights=torch.from_numpy(w / w.sum()).to(DEV), mode=mode,
                              gamma=1j, eps_pinv=1e-8)
        return x.cpu().numpy().real, float(np.real(np.sum(w * el) / w.sum()))

    drift = {}
    for mode, name in [(V.SR_IMAG, "imag"), (V.SR_REAL, "real")]:
        for dt in (0.005, 0.0025):
            th = np.concatenate([p0, p0])
            _, E0 = rhs(th, mode)
            for _ in range(int(round(T / dt))):
                k1, _ = rhs(th, mode)
                k2, _ = rhs(th + dt * k1, mode)
                th = th + 0.5 * dt * (k1 + k2)
            _, E1 = rhs(th, mode)
            drift[name, dt] = E1 - E0
    flush(f"  energy drift over t = {T}: " + ", ".join(f"{k[0]} dt={k[1]}: {v:.3e}" for k, v in drift.items()))
    assert abs(drift["imag", 0.0025]) < abs(drift["imag", 0.005]) / 2.5        # integrator error, ~dt^2
    assert abs(drift["imag", 0.0025]) < 0.05 * abs(drift["real", 0.0025])
    assert abs(drift["real", 0.0025] - drift["real", 0.005]) < 0.1 * abs(drift["real", 0.005])
