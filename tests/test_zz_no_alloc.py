"""The no-allocation variant of the reverse-mode product of log psi
(vmc_log_psi_vjp_noalloc) against vmc_log_psi_vjp, through the C ABI: two
calls in a row on one model (the second with fewer samples, so the fixed
scratch holds the first call's data when the second starts), RBM and CNN, a
batch larger than one chunk of the fixed scratch, an empty batch, and a model
too large for the scratch."""
import numpy as np
import pytest

import synth_inputs as si
from gpu_common import DEV, dev_bits, dev_c128, flush

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2108_03409_amd import nqsvmc as V  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    return V.Context(0)


def _model(ctx, kind):
    if kind == "rbm":
        N, Nh = 64, 256
        m = V.Model.rbm(ctx, N, Nh, True)
        m.set_params(dev_c128(si.rbm_params(N, Nh, std=0.05, seed=21)))
        return m, N
    Lx, Ly, C, k = 6, 5, 3, 3
    m = V.Model.cnn(ctx, Lx, Ly, C, k)
    m.set_params(dev_c128(si.cnn_params(C, k, std=0.2, seed=22)))
    return m, Lx * Ly


def _abs_sum(m, s, g):
    """sum_n |g_n| |O_nk| from the library's own O (chunks of 500 samples):
    the sum of the magnitudes of the terms both products add"""
    acc = torch.zeros(m.K, dtype=torch.float64, device=DEV)
    for b0 in range(0, s.shape[0], 500):
        O = m.grad_log_psi(s[b0:b0 + 500].contiguous())
        acc += (g[b0:b0 + 500].abs()[:, None] * O.abs()).sum(0)
    return acc.cpu().numpy()


def _close(a, b, B, terms):
    # both sum the same B float64 terms g_n conj(O_nk), in chunks and orders
    # of their own: |a - b| <= 2 (B + 64) 2^-53 sum_n |g_n| |O_nk| per entry
    return np.all(np.abs(a - b) <= 2.0 * (B + 64) * 2.0 ** -53 * terms + 1e-300)


@pytest.mark.parametrize("kind,B1,B2", [("rbm", 9000, 300), ("cnn", 700, 5)])
def test_noalloc_matches_vjp_twice(ctx, kind, B1, B2):
    # 9 000 RBM samples need two chunks of the 32 MiB scratch (about 3.3 kB each)
    m, N = _model(ctx, kind)
    for B, seed in ((B1, 1), (B2, 2)):
        flush(f"noalloc vjp {kind} B={B}")
        rng = np.random.default_rng(seed)
        s = dev_bits(si.pack_bits(si.random_bits(B, N, seed=seed)))
        g = dev_c128(rng.normal(size=B) + 1j * rng.normal(size=B))
        ref = m.log_psi_vjp(s, g)
        out = torch.full((m.K,), complex(np.nan, np.nan), dtype=torch.complex128, device=DEV)
        m.log_psi_vjp_noalloc(s, g, out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert _close(a, b, B, _abs_sum(m, s, g)), np.max(np.abs(a - b))


def test_noalloc_empty_batch_and_limits(ctx):
    m, N = _model(ctx, "rbm")
    out = torch.full((m.K,), complex(1.0, 1.0), dtype=torch.complex128, device=DEV)
    empty = torch.empty((0, 1), dtype=torch.int64, device=DEV)
    m.log_psi_vjp_noalloc(empty, torch.empty(0, dtype=torch.complex128, device=DEV), out)
    assert torch.count_nonzero(out).item() == 0
    # RBM N = 1024, N_h = 1024: its fixed part, 512 (N_h + 1)(N + 1) bytes, exceeds 32 MiB
    big = V.Model.rbm(ctx, 1024, 1024, True)
    s = torch.zeros((4, 16), dtype=torch.int64, device=DEV)
    g = torch.ones(4, dtype=torch.complex128, device=DEV)
    o2 = torch.empty(big.K, dtype=torch.complex128, device=DEV)
    with pytest.raises(V.VMCError) as e:
        big.log_psi_vjp_noalloc(s, g, o2)
    assert e.value.name == "WORKSPACE"
