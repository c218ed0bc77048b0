"""GPU MADE proposal against the oracle: log q, NLL gradients, Adam training,
autoregressive samples (bit-exact replay), and the mixed MADE/local Metropolis
chain (bit-exact replay, |psi|^2 histogram)."""
import numpy as np
import pytest
from scipy import stats

import synth_inputs as si
from oracle import made as omade, rbm as orbm, eloc as oeloc, metropolis as omet
from gpu_common import dev_bits, host_bits, dev_c128, flush

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2108_03409_amd import nqsvmc as V  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    return V.Context(0)


def _made(ctx, N, H, scale, seed):
    p = si.made_params(N, H, seed=seed) * scale
    p[H * N: H * N + H] = np.random.default_rng(seed).normal(0, 0.2, H)
    m = V.MADE(ctx, N, H)
    m.set_params(torch.from_numpy(p).to("cuda:0"))
    return m, p


@pytest.mark.parametrize("N,H,B", [(10, 16, 300), (64, 100, 200), (400, 512, 64), (3, 70, 65)])
def test_log_q(ctx, N, H, B):
    flush(f"made log_q N={N} H={H}")
    m, p = _made(ctx, N, H, 2.0, seed=N + H)
    bits = si.random_bits(B, N, seed=1)
    got = m.log_q(dev_bits(si.pack_bits(bits))).cpu().numpy()
    ref = omade.log_q(p, bits, N, H)
    assert np.max(np.abs(got - ref)) <= 1e-11 * max(1.0, np.abs(ref).max())
    assert np.array_equal(m.get_params().cpu().numpy(), p)


@pytest.mark.parametrize("N,H,B", [(10, 16, 300), (40, 64, 1000), (400, 512, 129)])
def test_nll_grad(ctx, N, H, B):
    flush(f"made grad N={N} H={H}")
    m, p = _made(ctx, N, H, 1.5, seed=3)
    bits = si.random_bits(B, N, seed=2)
    nll, g = m.nll_grad(dev_bits(si.pack_bits(bits)))
    nll_ref, g_ref = omade.nll_and_grad(p, bits, N, H)
    assert abs(nll - nll_ref) <= 1e-11 * abs(nll_ref)
    assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= 1e-11 * max(1e-3, np.abs(g_ref).max())


def test_train_matches_oracle(ctx):
    N, H, B = 10, 16, 500
    m, p = _made(ctx, N, H, 1.0, seed=4)
    rng = np.random.default_rng(1)
    base = rng.integers(0, 2, size=(B, 1)).repeat(N, 1)
    bits = (base ^ (rng.random((B, N)) < 0.1)).astype(np.uint8)
    nll = m.train(dev_bits(si.pack_bits(bits)), epochs=3, batch=128, lr=1e-2)
    p_ref, nll_ref = omade.train(p, bits, N, H, epochs=3, batch=128, lr=1e-2)
    assert abs(nll - nll_ref) <= 1e-9 * abs(nll_ref)
    assert np.max(np.abs(m.get_params().cpu().numpy() - p_ref)) <= 1e-9


@pytest.mark.parametrize("N,H,B,rows", [(10, 16, 500, None), (400, 512, 4096, [0, 17, 4095])])
def test_sample_replay(ctx, N, H, B, rows):
    flush(f"made sample N={N} H={H}")
    m, p = _made(ctx, N, H, 3.0, seed=5)
    s, lq = m.sample(B, seed=77, counter=(5 << 32) + 9)
    s = host_bits(s)
    lq = lq.cpu().numpy()
    idx = np.arange(B) if rows is None else np.array(rows)
    x_ref, lq_ref = omade.sample(p, len(idx), N, H, seed=77, lo=9, hi=5, rows=idx)
    for r, c in enumerate(idx):
        assert np.array_equal(s[c], si.pack_bits(x_ref[r])[0])
    assert np.max(np.abs(lq[idx] - lq_ref)) <= 1e-11 * max(1.0, np.abs(lq_ref).max())
    # log q of the samples through the batched path
    got = m.log_q(dev_bits(s[idx])).cpu().numpy()
    assert np.max(np.abs(got - lq_ref)) <= 1e-11 * max(1.0, np.abs(lq_ref).max())


def _mixed_setup(ctx, N, Nh, H, std, pg, n_chains, seed=101, therm=2):
    pr = si.rbm_params(N, Nh, std=std, is_complex=True, seed=8)
    model = V.Model.rbm(ctx, N, Nh, True)
    model.set_params(dev_c128(pr))
    Ham = V.Hamiltonian.tfim(ctx, N, 1, True, 1.0, 1.0)
    made, pm = _made(ctx, N, H, 2.0, seed=9)
    S = V.Sampler(ctx, model, Ham, proposal=V.PROP_MADE_MIX, n_chains=n_chains, therm_sweeps=therm, p_global=pg,
                  seed=seed)
    S.set_proposal_made(made)
    return model, Ham, made, S, pr, pm


def test_mixed_chain_replay(ctx):
    flush("mixed replay")
    N, Nh, H, nc, per = 10, 10, 16, 8, 6
    model, Ham, made, S, pr, pm = _mixed_setup(ctx, N, Nh, H, 0.4, 0.3, nc)
    s, lp, acc = S.sample(nc * per)
    a, ga, ng = S.stats()
    s = host_bits(s).reshape(per, nc, -1)
    f = lambda b: orbm.log_psi(pr, b, Nh)
    ch = omet.Chains(f, N, "made_mix", seed=101, chain_ids=np.arange(nc), therm_sweeps=2, made=(pm, N, H),
                     p_global=0.3)
    os_, ol = ch.sample(per)
    for c in range(nc):
        for k in range(per):
            assert np.array_equal(s[k, c], si.pack_bits(os_[k, c])[0]), (k, c)
    assert ng == ch.n_global and ng > 0
    assert abs(ga - ch.acc_global / ch.n_global) < 1e-12


def test_mixed_chain_histogram(ctx):
    flush("mixed histogram")
    N, Nh, H = 10, 10, 16
    # 20 thermalisation sweeps, then every 10th of 1000 sweeps: the chi-square
    # test assumes independent draws, so the kept samples must be well
    # separated compared with the chain's autocorrelation time
    model, Ham, made, S, pr, pm = _mixed_setup(ctx, N, Nh, H, 0.5, 0.5, 1024, seed=3, therm=20)
    s, _, _ = S.sample(1024 * 1000)
    a, ga, ng = S.stats()
    flush(f"  acceptance {a:.3f}, global acceptance {ga:.3f} of {ng} global proposals")
    assert ng > 0 and 0 < ga < 1
    dec = host_bits(s).reshape(1000, 1024)[::10].reshape(-1).astype(np.int64)
    cd = np.bincount(dec, minlength=2 ** N)
    _, prob, _ = oeloc.exact_probabilities(lambda b: orbm.log_psi(pr, b, Nh), N)
    res = stats.chisquare(cd, prob * cd.sum())
    assert res.pvalue > 1e-4, res


def test_trained_proposal_is_accepted_more(ctx):
    # train q on the chain's own samples: global acceptance must rise
    flush("made training gain")
    N, Nh, H = 10, 10, 32
    model, Ham, made, S, pr, pm = _mixed_setup(ctx, N, Nh, H, 0.6, 0.5, 512, seed=11)
    S.sample(512 * 20)
    _, ga0, _ = S.stats()
    local = V.Sampler(ctx, model, Ham, proposal=V.PROP_FLIP, n_chains=1024, therm_sweeps=20, seed=12)
    data, _, _ = local.sample(1024 * 32)
    made.train(data, epochs=20, batch=256, lr=3e-3)
    S.set_proposal_made(made)
    S.sample(512 * 20)
    _, ga1, _ = S.stats()
    assert ga1 > ga0 + 0.1, (ga0, ga1)
