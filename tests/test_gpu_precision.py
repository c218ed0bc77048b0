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
