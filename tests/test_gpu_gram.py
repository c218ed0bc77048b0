"""The quantum Fisher matrix S (eq:qfm) and the force F (eq:force_vector) as
the SR solve forms them on the matrix cores, compared entry by entry with the
oracle's float64 definition on the same (complex64-rounded) log-derivatives.

Per-entry bound of the float32 Gram (three real products per complex term):
with the centred, weighted values Obar_nk = sqrt(w_n) (O_nk - <O_k>) rounded
to float32 (relative 2^-24 per part), a_nk = |Re Obar_nk| + |Im Obar_nk| and
M_kk' = sum_n a_nk a_nk', every real product sum A = sum Re Re', B = sum Im Im',
C = sum (Re - Im)(Re' + Im') has terms bounded by a_nk a_nk' and float32
recursive-summation error gamma_{N_s}, plus the input roundings (2u on a
product, u more on the sums Re - Im and Re' + Im'); Re S = A + B and
Im S = C - A + B (float64) give |dS_kk'| <= 2 (N_s + 8) 2^-24 M_kk'.  A
misplaced tile, a swapped orientation (S against S^T = conj S) or a dropped
term moves an entry by O(|S_kk'|), which the tests below also check is far
outside the bound."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import sr as osr
from gpu_common import DEV, dev_c128, flush

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2108_03409_amd import nqsvmc as V  # noqa: E402

U = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    return V.Context(0)


def _random_o(ns, K, seed, cplx=True):
    """log-derivative-like columns: magnitudes spread over three decades, a
    non-zero mean (the centring matters), complex64 values."""
    rng = np.random.default_rng(seed)
    scale = np.logspace(0, -3, K)[rng.permutation(K)]
    O = rng.normal(size=(ns, K)) + (1j * rng.normal(size=(ns, K)) if cplx else 0.0)
    O = (O + 0.7 - 0.3j * cplx) * scale
    el = rng.normal(size=ns) + 1j * rng.normal(size=ns) - 5.0
    return O.astype(np.complex64 if cplx else np.float32), el


def _centred(Od, w):
    ww = np.full(Od.shape[0], 1.0 / Od.shape[0]) if w is None else w / w.sum()
    return np.sqrt(ww)[:, None] * (Od - ww @ Od)


def _bound_matrix(Od, w, rows=None):
    Ob = _centred(Od, w)
    a = np.abs(Ob.real) + np.abs(Ob.imag)
    return (a.T @ a) if rows is None else (a[:, rows].T @ a)


def _check_force(F_got, F_ref, Od, el, w):
    # float64 on both sides, different summation orders (and the oracle's
    # uncentred form): |dF_k| <= 4 (N_s + 8) 2^-53 sum_n w_n (|O_nk| + |<O_k>|)(|E_n| + |<E>|)
    ns = Od.shape[0]
    ww = np.full(ns, 1.0 / ns) if w is None else w / w.sum()
    G = (ww * (np.abs(el) + abs(np.sum(ww * el)))) @ (np.abs(Od) + np.abs(ww @ Od))
    assert np.all(np.abs(F_got - F_ref) <= 4.0 * (ns + 8) * 2.0 ** -53 * G)


def _check(S_got, S_ref, M, ns, nu, what):
    bound = 2.0 * (ns + 8) * U * M * (1.0 + nu) + 1e-300
    err = np.abs(S_got - S_ref)
    worst = np.max(err / bound)
    assert worst <= 1.0, (what, worst)
    # the bound discriminates: the transposed (conjugated) matrix and a shifted
    # tile fail it wherever S has imaginary parts / structure
    if np.abs(S_ref.imag).max() > 0:
        assert np.max(np.abs(S_got - S_ref.conj()) / bound) > 10.0, what
    return worst


@pytest.mark.parametrize("ns,K,weighted,mode", [
    (333, 636, False, "complex"),     # even K: direct-to-LDS Gram kernel, ragged samples
    (1001, 219, True, "complex"),     # odd K: register-staged Gram kernel
    (5, 320, False, "complex"),       # fewer samples than one stage; K = 64 (mod 256)
    (2000, 1088, False, "complex"),   # K = 17 x 64: single-block last panel, ragged row tiles
    (20000, 110, False, "complex"),   # few tiles, many samples: sample range split over groups
    (777, 300, True, "real"),         # Re projection of complex O (one accumulator)
    (777, 301, False, "imag"),        # i Im S (the matrix the Im-projected eigen solve takes)
])
def test_fisher_entrywise_float32_gram(ctx, ns, K, weighted, mode):
    flush(f"fisher c64 ns={ns} K={K} weighted={weighted} mode={mode}")
    O32, el = _random_o(ns, K, seed=ns + K)
    Od = O32.astype(np.complex128)
    w = np.random.default_rng(K).uniform(0.5, 1.5, ns) if weighted else None
    nu = 1e-3 if mode != "imag" else 0.0
    md = {"complex": V.SR_COMPLEX, "real": V.SR_REAL, "imag": V.SR_IMAG}[mode]
    S, F, info = V.sr_fisher(ctx, torch.from_numpy(O32).to(DEV), dev_c128(el), nu_rel=nu, mode=md,
                             weights=None if w is None else torch.from_numpy(w).to(DEV))
    S, F = S.cpu().numpy(), F.cpu().numpy()
    S_ref, F_ref = osr.fisher_and_force(Od, el, w)
    if mode == "imag":
        St_ref = 1j * osr.project(S_ref, "imag")
    else:
        St_ref = osr.shifted(osr.project(S_ref, mode), nu)
    M = _bound_matrix(Od, w)
    worst = _check(S, St_ref, M, ns, nu, (ns, K, mode))
    flush(f"  worst |dS| / bound = {worst:.3e}")
    if mode == "imag":
        assert np.all(np.diag(S) == 0) and np.all(S.real == 0)
    # F in float64 from the same float32 O
    _check_force(F, F_ref, Od, el, w)
    mean, var = osr.energy_stats(el, w)
    assert abs(info["e_mean"] - mean) <= 1e-12 * abs(mean)


@pytest.mark.parametrize("ns,K,dt", [(1001, 219, "c128"), (1000, 300, "f32"), (999, 301, "f64")])
def test_fisher_entrywise_other_inputs(ctx, ns, K, dt):
    # complex128 O: float64 Gram (tight); real O: two samples per complex row,
    # S = Re of the packed Gram (an odd count leaves a half-empty row)
    flush(f"fisher {dt} ns={ns} K={K}")
    O32, el = _random_o(ns, K, seed=7 * K, cplx=(dt == "c128"))
    if dt == "c128":
        Od = O32.astype(np.complex128) * (1 + 1e-3j)
        Og = torch.from_numpy(Od).to(DEV)
    elif dt == "f32":
        Od = O32.astype(np.float64)
        Og = torch.from_numpy(O32).to(DEV)
    else:
        Od = O32.astype(np.float64) * 1.001
        Og = torch.from_numpy(Od).to(DEV)
    S, F, _ = V.sr_fisher(ctx, Og, dev_c128(el), nu_rel=1e-3, mode=V.SR_COMPLEX)
    S = S.cpu().numpy()
    S_ref, F_ref = osr.fisher_and_force(Od.astype(np.complex128), el)
    St_ref = osr.shifted(S_ref, 1e-3)
    M = _bound_matrix(Od.astype(np.complex128), None)
    if dt == "f32":
        _check(S, St_ref, M, ns, 1e-3, dt)
    else:
        # float64 products on both sides; the oracle's uncentred form rounds
        # relative to |O| + |<O>|, not to the centred values
        Oc = Od.astype(np.complex128)
        a = (np.abs(Oc.real) + np.abs(Oc.imag) + np.abs((Oc.mean(0)).real) + np.abs((Oc.mean(0)).imag)) / np.sqrt(ns)
        Mu = a.T @ a
        assert np.max(np.abs(S - St_ref) / (4.0 * (ns + 8) * 2.0 ** -53 * Mu + 1e-300)) <= 1.0
    _check_force(F.cpu().numpy(), F_ref, Od.astype(np.complex128), el, None)


def test_fisher_entrywise_split16(ctx):
    # gram = 1: hi + lo float16 parts per value after a per-column power-of-two
    # scale (column maximum in [2^13, 2^14)); per product relative error below
    # 3 x 2^-22 (dropped lo lo', rounding of lo), plus an absolute floor from
    # float16 subnormals (spacing 2^-24 in scaled units: 2^-25 x 2^-e_k per value)
    flush("fisher split16")
    ns, K = 1500, 400
    O32, el = _random_o(ns, K, seed=99)
    Od = O32.astype(np.complex128)
    S, _, _ = V.sr_fisher(ctx, torch.from_numpy(O32).to(DEV), dev_c128(el), nu_rel=0.0, gram=1)
    S = S.cpu().numpy()
    S_ref, _ = osr.fisher_and_force(Od, el)
    Ob = _centred(Od, None).astype(np.complex64).astype(np.complex128)
    a = np.abs(Ob.real) + np.abs(Ob.imag)
    M = a.T @ a
    cmax = np.maximum(np.abs(Ob.real), np.abs(Ob.imag)).max(axis=0)
    step = np.ldexp(1.0, -(14 - np.frexp(cmax)[1]))            # 2^-e_k
    floor = 2.0 ** -25 * 2 * (np.outer(a.sum(0), step) + np.outer(step, a.sum(0)))
    bound = 2.0 * (ns + 8) * U * M + 8 * 2.0 ** -22 * M + floor
    assert np.max(np.abs(S - S_ref) / bound) <= 1.0


def _c3_inputs(ctx):
    """O_k (complex64) and E_loc of one step of the SR-step workload (TFIM chain
    L = 64, complex RBM alpha = 4, K = 16 704, 1024 chains x 16 sweeps), from the
    library's sampler as the benchmark draws them."""
    cfg = si.WORKLOADS["tfim1d_L64_rbm_a4_sr"]
    N = cfg["Lx"]
    Nh = cfg["alpha"] * N
    p = si.rbm_params(N, Nh, std=cfg["std"], is_complex=True, seed=cfg["param_seed"])
    m = V.Model.rbm(ctx, N, Nh, True)
    m.set_params(torch.from_numpy(p).to(DEV))
    H = V.Hamiltonian.tfim(ctx, N, 1, True, cfg["J"], cfg["h"])
    smp = V.Sampler(ctx, m, H, proposal=V.PROP_FLIP, n_chains=cfg["n_chains"], therm_sweeps=20,
                    seed=cfg["sampler_seed"])
    ns = cfg["n_chains"] * cfg["samples_per_chain"]
    s, _, _ = smp.sample(ns)
    O = m.grad_log_psi(s, dtype=torch.complex64)
    el = m.local_energy(H, s)
    torch.cuda.synchronize()
    return O, el, cfg["nu_rel"]


def test_fisher_rows_and_solve_at_sr_step_shape(ctx):
    # the benchmark's launch: K = 16 704 (261 blocks of 64: K = 64 mod 256),
    # N_s = 16 384.  Sampled rows of S~ (first and last row of several tiles,
    # every column) against the oracle's rows; then x of the Cholesky path
    # against LAPACK on the library's own S~ and against the oracle's system.
    import scipy.linalg as sl

    O, el, nu = _c3_inputs(ctx)
    ns, K = O.shape
    assert K == 16704 and ns == 16384
    flush(f"fisher rows at the SR-step shape ns={ns} K={K}")
    S, F, info = V.sr_fisher(ctx, O, el, nu_rel=nu)
    rows = [0, 1, 63, 64, 127, 128, 255, 256, 8255, 8256, 16383, 16384, 16639, 16640, 16703]
    S_rows = S[rows].cpu().numpy()
    Od = O.cpu().numpy().astype(np.complex128)
    eh = el.cpu().numpy()
    R = osr.fisher_rows(Od, rows)
    R[np.arange(len(rows)), rows] *= 1.0 + nu
    M = _bound_matrix(Od, None, rows)
    worst = _check(S_rows, R, M, ns, nu, "sr-step rows")
    flush(f"  worst |dS| / bound over {len(rows)} rows = {worst:.3e}")
    F_ref = osr.force(Od, eh)
    _check_force(F.cpu().numpy(), F_ref, Od, eh, None)

    flush("  Cholesky solve at the SR-step shape vs LAPACK")
    x, sinfo = V.sr_solve(ctx, O, el, nu_rel=nu)
    x = x.cpu().numpy()
    St = S.cpu().numpy()
    del S
    Fh = F.cpu().numpy()
    c = sl.cho_factor(St, lower=True, check_finite=False)
    x_lapack = sl.cho_solve(c, -Fh, check_finite=False)
    del c
    rel = np.linalg.norm(x - x_lapack) / np.linalg.norm(x_lapack)
    flush(f"  |x - x_lapack| / |x_lapack| = {rel:.3e}, residual {sinfo['residual']:.2e}")
    assert rel <= 1e-9, rel
    # backward error against the oracle's own system: S~_ref x = Obar^H (Obar x)
    # + nu diag(S_ref) x, formed matrix-free from the float64 centred values
    Ob = _centred(Od, None)
    d_ref = np.einsum("nk,nk->k", Ob.conj(), Ob).real
    Sx = Ob.conj().T @ (Ob @ x) + nu * d_ref * x
    back = np.linalg.norm(Sx + F_ref) / np.linalg.norm(F_ref)
    # |dS x| <= ||dS||_F |x| with ||dS||_F <= 2 (N_s + 8) u ||M||_F <= 2 (N_s + 8) u sum_n |a_n|^2
    a2 = np.sum((np.abs(Ob.real) + np.abs(Ob.imag)) ** 2)
    bound = 2.0 * (ns + 8) * U * (1 + nu) * a2 * np.linalg.norm(x) / np.linalg.norm(F_ref) + 1e-12
    flush(f"  backward error vs the oracle's system {back:.3e} (bound {bound:.3e})")
    assert back <= bound
