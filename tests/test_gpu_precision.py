"""Float32 / bfloat16 RBM evaluation against the FP64 oracle, with the error
bound stated per result:
  * float32: theta accumulated in float32 (N terms), log cosh in float32:
        |d log psi| <= 8 eps32 [ sum_i |a_i| + sum_j (N |W_j|_max + |b_j| + |log cosh theta_j| + 1) ]
  * bfloat16, against the oracle on the bfloat16-rounded parameters: the same
    float32 bound (rounding the parameters is the only other difference);
  * bfloat16, against the oracle on the original parameters (quantisation):
        |d log psi| <= 2^-8 [ sum_i |a_i| + sum_j |tanh theta_j| (|b_j| + sum_i |W_ji|) ] + float32 bound
  * local energies: every slot ratio inherits the log psi difference error of
    its two configurations, so |dE_loc| <= sum_j |H_ss'_j psi(s'_j)/psi(s)| (e^delta - 1) with
    delta the bound on |d (log psi(s') - log psi(s))|."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import rbm as orbm, eloc as oeloc, lattice as olat
from gpu_common import dev_bits, dev_c128, flush

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2108_03409_amd import nqsvmc as V  # noqa: E402

EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    return V.Context(0)


def bf16_round(x):
    """Round-to-nearest-even to bfloat16, applied to real and imaginary parts."""
    def r(a):
        u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    return r(np.real(x)) + 1j * r(np.imag(x))


def f32_bound(p, bits, N, Nh):
    a, b, W = orbm.split(p, N, Nh)
    sig = 2.0 * bits - 1.0
    th = sig @ W.T + b
    per = np.sum(np.abs(a)) + np.sum(N * np.abs(W).max(axis=1) + np.abs(b) + np.abs(np.log(np.cosh(th))) + 1.0,
                                     axis=-1)
    return 8 * EPS32 * per


def quant_bound(p, bits, N, Nh):
    a, b, W = orbm.split(p, N, Nh)
    sig = 2.0 * bits - 1.0
    th = sig @ W.T + b
    return 2.0 ** -8 * (np.sum(np.abs(a)) + np.sum(np.abs(np.tanh(th)) * (np.abs(b) + np.abs(W).sum(1)), axis=1))


def wrapd(d):
    return np.abs(d.real) + np.abs((d.imag + np.pi) % (2 * np.pi) - np.pi)


@pytest.mark.parametrize("N,Nh,std,B", [(100, 400, 0.01, 200), (64, 256, 0.1, 300), (37, 70, 0.3, 129)])
def test_log_psi_precision(ctx, N, Nh, std, B):
    flush(f"precision log_psi N={N} Nh={Nh}")
    p = si.rbm_params(N, Nh, std=std, seed=N)
    bits = si.random_bits(B, N, seed=3)
    s = dev_bits(si.pack_bits(bits))
    m = V.Model.rbm(ctx, N, Nh, True)
    m.set_params(dev_c128(p))
    ref = orbm.log_psi(p, bits, Nh)
    m.set_precision(V.VMC_F32)
    e32 = wrapd(m.log_psi(s).cpu().numpy() - ref)
    assert np.all(e32 <= f32_bound(p, bits, N, Nh)), (e32.max(), f32_bound(p, bits, N, Nh).min())
    m.set_precision(V.VMC_BF16)
    got = m.log_psi(s).cpu().numpy()
    pq = bf16_round(p)
    eacc = wrapd(got - orbm.log_psi(pq, bits, Nh))
    assert np.all(eacc <= f32_bound(pq, bits, N, Nh)), eacc.max()
    eq = wrapd(got - ref)
    assert np.all(eq <= quant_bound(p, bits, N, Nh) + f32_bound(p, bits, N, Nh)), eq.max()
    flush(f"  max |d log psi|: f32 {e32.max():.2e}, bf16 accumulation {eacc.max():.2e}, bf16 total {eq.max():.2e}")
    m.set_precision(V.VMC_F64)
    assert np.max(wrapd(m.log_psi(s).cpu().numpy() - ref)) < 1e-10


@pytest.mark.parametrize("kind,Lx,Ly,Nh,std,B", [("heisenberg", 10, 10, 400, 0.01, 24), ("tfim", 64, 1, 256, 0.02, 24)])
def test_local_energy_precision(ctx, kind, Lx, Ly, Nh, std, B):
    flush(f"precision eloc {kind}")
    N = Lx * Ly
    p = si.rbm_params(N, Nh, std=std, seed=5)
    bits = si.random_bits_sz0(B, N, seed=6) if kind == "heisenberg" else si.random_bits(B, N, seed=6)
    s = dev_bits(si.pack_bits(bits))
    m = V.Model.rbm(ctx, N, Nh, True)
    m.set_params(dev_c128(p))
    H = V.Hamiltonian.heisenberg(ctx, Lx, Ly, True, 1.0) if kind == "heisenberg" else \
        V.Hamiltonian.tfim(ctx, Lx, Ly, True, 1.0, 1.0)
    h = 0.0 if kind == "heisenberg" else 1.0
    for prec, pr in [(V.VMC_F32, p), (V.VMC_BF16, bf16_round(p))]:
        m.set_precision(prec)
        got = m.local_energy(H, s).cpu().numpy()
        f = lambda b: orbm.log_psi(pr, b, Nh)
        ref = oeloc.local_energy(f, kind, bits, Lx, Ly, True, 1.0, h)
        for n, sb in enumerate(bits):
            sp, mel, cnt = olat.connected(kind, sb, Lx, Ly, True, 1.0, h)
            r = np.abs(mel[1:cnt] * np.exp(f(sp[1:cnt]) - f(sb[None])[0]))
            delta = 2 * f32_bound(pr, np.vstack([sb[None], sp[1:cnt]]), N, Nh).max()
            assert abs(got[n] - ref[n]) <= np.sum(r) * np.expm1(delta) + 1e-12, (prec, n)
    m.set_precision(V.VMC_F64)


# ---------------------------------------------------------------- CNN -------
# Float32 / bfloat16 CNN local energies (TFIM).  Per flip f the kernel forms
# the layer-1 change dA = log(1 + (cosh d - 1) + tanh(z1) sinh d) on the k x k
# changed positions, the layer-2 change dZ = W2 * dA on the matrix cores and
# the ratio as the product over the (2k-1)^2 window of
# fac = cosh dZ + tanh(z2) sinh dZ.  First-order error bound per window entry
# (eps = 2^-24; u = 2^-9 for bfloat16 operands, 0 for float32):
#   tanh z1:   e_t1 = 8 eps ((1 + |t1|^2)(sum |W1| + |b1|) + |t1|)
#   dA:        e_dA = (8 eps + u) |dA| + max |sinh 2 W1| / |1 + u_dA| e_t1
#   a1 (forward operand): e_a1 = 8 eps (1 + |a1|) + u |a1|
#   z2:        e_z2 = |W2| * ((1 + u) e_a1 + (u + C k^2 eps) |a1|) + 8 eps |b2|
#   tanh z2:   e_t2 = (1 + |t2|^2) e_z2 + 8 eps |t2|
#   dZ:        e_dZ = |W2| * ((1 + u) e_dA + (u + C k^2 eps) |dA|)
#   log fac:   |tanh z2'| e_dZ + |sinh dZ| / |fac| e_t2 + c eps   (c = 16 float32, 64 bfloat16)
# (* is the layer-2 correlation), and |dE_loc| <= h sum_f |psi(s_f)/psi(s)| expm1(sum_window).
from oracle import cnn as ocnn  # noqa: E402


def _corr(X, Wabs, k):
    """Y[f, c, y, x] = sum_{ci, dy, dx} Wabs[c, ci, dy, dx] X[f, ci, y + dy, x + dx] (periodic)."""
    Y = 0.0
    for dy in range(k):
        for dx in range(k):
            Y = Y + np.einsum("oi,biyx->boyx", Wabs[:, :, dy, dx], np.roll(X, (-dy, -dx), axis=(-2, -1)))
    return Y


def _windows(N, Lx, Ly, k, size):
    """mask[f, y, x]: position (y, x) = f - e for e in [0, size)^2."""
    m = np.zeros((N, Ly, Lx), dtype=bool)
    for f in range(N):
        y, x = divmod(f, Lx)
        for ey in range(size):
            for ex in range(size):
                m[f, (y - ey) % Ly, (x - ex) % Lx] = True
    return m


def _cnn_eloc_bound(p, sb, Lx, Ly, C, k, h, u, cf, g3=1):
    W1, b1, W2, b2 = ocnn.split(p, C, k)
    N = Lx * Ly
    flips = np.repeat(sb[None], N, axis=0)
    flips[np.arange(N), np.arange(N)] ^= 1
    _, z1, a1, z2 = ocnn.layers(p, sb[None], Lx, Ly, C, k)
    _, z1p, a1p, z2p = ocnn.layers(p, flips, Lx, Ly, C, k)
    E = EPS32
    t1 = np.abs(np.tanh(z1))
    S1 = (np.abs(W1).reshape(C, -1).sum(1) + np.abs(b1))[None, :, None, None]
    e_t1 = 8 * E * ((1 + t1 ** 2) * S1 + t1)
    dA = np.abs(a1p - a1) * _windows(N, Lx, Ly, k, k)[:, None]
    sh1 = np.abs(np.sinh(2 * W1)).reshape(C, -1).max(1)[None, :, None, None]
    one_u = np.abs(np.cosh(z1p) / np.cosh(z1))
    e_dA = ((8 * E + u) * dA + sh1 / one_u * e_t1) * (dA > 0)
    aW2 = np.abs(W2)
    e_a1 = 8 * E * (1 + np.abs(a1)) + u * np.abs(a1)
    e_z2 = _corr((1 + u) * e_a1 + (u + C * k * k * E) * np.abs(a1), aW2, k) + 8 * E * np.abs(b2)[None, :, None, None]
    t2 = np.abs(np.tanh(z2))
    e_t2 = (1 + t2 ** 2) * e_z2 + 8 * E * t2
    # g3 = 2: the window products take three real products per complex term, whose
    # accumulated rounding in Im is at most twice the four-product bound
    e_dZ = _corr((1 + u) * e_dA + (u + g3 * C * k * k * E) * dA, aW2, k)
    fac = np.abs(np.cosh(z2p) / np.cosh(z2))
    term = np.abs(np.tanh(z2p)) * e_dZ + np.abs(np.sinh(z2p - z2)) / fac * e_t2 + cf * E
    delta = np.sum(term * _windows(N, Lx, Ly, k, 2 * k - 1)[:, None], axis=(1, 2, 3))
    lp = ocnn.log_psi(p, np.vstack([sb[None], flips]), Lx, Ly, C, k)
    ratio = np.abs(np.exp(lp[1:] - lp[0]))
    return h * np.sum(ratio * np.expm1(delta))


@pytest.mark.parametrize("Lx,Ly,C,k,std,B", [(16, 16, 16, 4, 0.05, 3), (8, 8, 3, 3, 0.3, 5), (7, 7, 2, 4, 0.2, 5),
                                             (9, 7, 5, 3, 0.2, 4), (8, 8, 3, 3, 0.08, 5), (10, 10, 8, 3, 0.06, 4),
                                             (7, 9, 17, 2, 0.05, 3)])
def test_cnn_local_energy_precision(ctx, Lx, Ly, C, k, std, B):
    flush(f"precision cnn eloc {Lx}x{Ly} C={C} k={k}")
    p = si._normal_params(ocnn.num_params(C, k), std, True, seed=7 * Lx + C)
    m = V.Model.cnn(ctx, Lx, Ly, C, k)
    m.set_params(dev_c128(p))
    H = V.Hamiltonian.tfim(ctx, Lx, Ly, True, 1.0, 3.0)
    bits = si.random_bits(B, Lx * Ly, seed=8)
    s = dev_bits(si.pack_bits(bits))
    f = lambda b: ocnn.log_psi(p, b, Lx, Ly, C, k)
    ref = oeloc.local_energy(f, "tfim", bits, Lx, Ly, True, 1.0, 3.0)
    for prec, u, cf, g3 in [(V.VMC_F32, 0.0, 16, 2), (V.VMC_BF16, 2.0 ** -9, 64, 1)]:
        m.set_precision(prec)
        got = m.local_energy(H, s).cpu().numpy()
        errs = []
        for n, sb in enumerate(bits):
            bnd = _cnn_eloc_bound(p, sb, Lx, Ly, C, k, 3.0, u, cf, g3)
            errs.append((abs(got[n] - ref[n]), bnd))
            assert abs(got[n] - ref[n]) <= bnd + 1e-12, (prec, n, abs(got[n] - ref[n]), bnd)
        rel = max(e / abs(r) for (e, _), r in zip(errs, ref))
        flush(f"  prec {prec}: max |dE|/|E| {rel:.2e}, max |dE| {max(e for e, _ in errs):.2e}, "
              f"min bound {min(b for _, b in errs):.2e}")
    m.set_precision(V.VMC_F64)
    got = m.local_energy(H, s).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.abs(ref).max())


def test_cnn_precision_small_torus_unsupported(ctx):
    m = V.Model.cnn(ctx, 4, 4, 2, 4)
    with pytest.raises(V.VMCError) as e:
        m.set_precision(V.VMC_F32)
    assert e.value.name == "UNSUPPORTED"
