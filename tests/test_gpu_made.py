"""GPU MADE proposal against the oracle: log q, NLL gradients, Adam training,
autoregressive samples (bit-exact replay), and the mixed MADE/local Metropolis
chain (bit-exact replay, |psi|^2 histogram)."""
import numpy as np
import pytest
from scipy import stats

import synth_inputs as si
from oracle import made as omade, rbm as orbm, eloc as oeloc, metropolis as omet
from gpu_common import dev_bits, host_bits, dev_c128, flush, assert_logpsi_close

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


def _mixed_setup(ctx, N, Nh, H, std, G, n_chains, seed=101, therm=2, sweep=0, made_scale=2.0):
    pr = si.rbm_params(N, Nh, std=std, is_complex=True, seed=8)
    model = V.Model.rbm(ctx, N, Nh, True)
    model.set_params(dev_c128(pr))
    Ham = V.Hamiltonian.tfim(ctx, N, 1, True, 1.0, 1.0)
    made, pm = _made(ctx, N, H, made_scale, seed=9)
    S = V.Sampler(ctx, model, Ham, proposal=V.PROP_MADE_MIX, n_chains=n_chains, therm_sweeps=therm, global_steps=G,
                  seed=seed, sweep_steps=sweep)
    S.set_proposal_made(made)
    return model, Ham, made, S, pr, pm


@pytest.mark.parametrize("N,H,G,sweep", [(10, 16, 1, 0), (10, 16, 3, 4), (3, 70, 2, 0), (37, 100, 1, 5)])
def test_mixed_chain_replay(ctx, N, H, G, sweep):
    # global MADE steps of all chains, then flips: the chains replay the
    # oracle's, and so do the global-proposal counts and acceptance; (3, 70) has
    # more in-block units than the staged path holds, (37, 100) spans three
    # 16-site blocks with a ragged last one
    flush(f"mixed replay N={N} H={H} G={G} sweep={sweep}")
    Nh, nc, per = N, 19, 5
    model, Ham, made, S, pr, pm = _mixed_setup(ctx, N, Nh, H, 0.15, G, nc, sweep=sweep, made_scale=0.5)
    s, lp, acc = S.sample(nc * per)
    a, ga, ng = S.stats()
    s = host_bits(s).reshape(per, nc, -1)
    f = lambda b: orbm.log_psi(pr, b, Nh)
    ch = omet.Chains(f, N, "made_mix", seed=101, chain_ids=np.arange(nc), therm_sweeps=2, made=(pm, N, H),
                     global_steps=G, sweep_steps=sweep or None)
    os_, ol = ch.sample(per)
    for c in range(nc):
        for k in range(per):
            assert np.array_equal(s[k, c], si.pack_bits(os_[k, c])[0]), (k, c)
    assert ng == nc * G * (per + 2) and ch.n_global == ng   # the first call includes 2 thermalisation sweeps
    assert 0 < ch.acc_global < ch.n_global and abs(ga - ch.acc_global / ch.n_global) < 1e-12
    assert_logpsi_close(lp.cpu().numpy().reshape(per, nc), ol, rtol=1e-10)
    # a second call continues the same chains (and the state blob carries the global counter)
    blob = S.get_state()
    s2, _, _ = S.sample(nc * 2)
    os2, _ = ch.sample(2)
    assert np.array_equal(host_bits(s2).reshape(2, nc, -1), si.pack_bits(os2.reshape(-1, N)).reshape(2, nc, -1))
    S.set_state(blob)
    s3, _, _ = S.sample(nc * 2)
    assert torch.equal(s2, s3)


def test_mixed_chain_replay_two_waves_per_chain(ctx):
    # N_h > 256 with few chains: the local sweeps run two waves per chain, which
    # hand theta to the global steps and take it back between the launches
    flush("mixed replay, two waves per chain")
    N, Nh, H, G, nc, per = 12, 300, 16, 2, 19, 3
    pr = si.rbm_params(N, Nh, std=0.1, is_complex=True, seed=8)
    model = V.Model.rbm(ctx, N, Nh, True)
    model.set_params(dev_c128(pr))
    Ham = V.Hamiltonian.tfim(ctx, N, 1, True, 1.0, 1.0)
    made, pm = _made(ctx, N, H, 0.5, seed=9)
    S = V.Sampler(ctx, model, Ham, proposal=V.PROP_MADE_MIX, n_chains=nc, therm_sweeps=2, global_steps=G, seed=101)
    S.set_proposal_made(made)
    s, lp, _ = S.sample(nc * per)
    s = host_bits(s).reshape(per, nc, -1)
    ch = omet.Chains(lambda b: orbm.log_psi(pr, b, Nh), N, "made_mix", seed=101, chain_ids=np.arange(nc),
                     therm_sweeps=2, made=(pm, N, H), global_steps=G)
    os_, ol = ch.sample(per)
    for c in range(nc):
        for k in range(per):
            assert np.array_equal(s[k, c], si.pack_bits(os_[k, c])[0]), (k, c)
    assert_logpsi_close(lp.cpu().numpy().reshape(per, nc), ol, rtol=1e-10)
    assert 0 < ch.acc_global < ch.n_global and ch.near_ties == 0


def test_mixed_chain_replay_after_new_parameters(ctx):
    # the proposals of the next global step, with their theta, are formed ahead
    # of the step; new RBM parameters between two calls must not leave a stale
    # theta behind: the second call replays the oracle's chains under the new
    # parameters (an SR loop changes them between every two calls)
    flush("mixed replay across a parameter change")
    N, Nh, H, G, nc, per = 10, 10, 16, 1, 19, 3
    model, Ham, made, S, pr, pm = _mixed_setup(ctx, N, Nh, H, 0.15, G, nc, made_scale=0.5)
    s1, _, _ = S.sample(nc * per)
    pr2 = si.rbm_params(N, Nh, std=0.4, is_complex=True, seed=21)
    model.set_params(dev_c128(pr2))
    s2, lp2, _ = S.sample(nc * per)
    ch = omet.Chains(lambda b: orbm.log_psi(pr, b, Nh), N, "made_mix", seed=101, chain_ids=np.arange(nc),
                     therm_sweeps=2, made=(pm, N, H), global_steps=G)
    o1, _ = ch.sample(per)
    ch.f = lambda b: orbm.log_psi(pr2, b, Nh)
    ch.logpsi = ch.f(ch.states)
    o2, ol2 = ch.sample(per)
    for o, s in ((o1, s1), (o2, s2)):
        s = host_bits(s).reshape(per, nc, -1)
        for c in range(nc):
            for k in range(per):
                assert np.array_equal(s[k, c], si.pack_bits(o[k, c])[0]), (k, c)
    assert_logpsi_close(lp2.cpu().numpy().reshape(per, nc), ol2, rtol=1e-10)
    assert ch.near_ties == 0


def test_mixed_chain_replay_at_learned_proposal_shape(ctx):
    # the learned-proposal workload's shape: 20 x 20 lattice, RBM alpha = 2, a
    # MADE 400 -> 512 -> 400, 4096 chains with two global steps per sweep;
    # four chains replayed by the oracle over two thermalisation and two
    # recorded sweeps (weak weights on both networks so that global proposals
    # are accepted often enough to exercise both outcomes)
    flush("mixed replay 20x20, 4096 chains")
    L, H, nc, G = 20, 512, 4096, 2
    N = L * L
    Nh = 2 * N
    p = si.rbm_params(N, Nh, std=0.01, is_complex=True, seed=5)
    model = V.Model.rbm(ctx, N, Nh, True)
    model.set_params(dev_c128(p))
    Ham = V.Hamiltonian.tfim(ctx, L, L, True, 1.0, 3.0)
    pm = si.made_params(N, H, seed=205) * 0.3
    made = V.MADE(ctx, N, H)
    made.set_params(torch.from_numpy(pm).to("cuda:0"))
    S = V.Sampler(ctx, model, Ham, proposal=V.PROP_MADE_MIX, n_chains=nc, therm_sweeps=2, global_steps=G, seed=77)
    S.set_proposal_made(made)
    s, _, _ = S.sample(nc * 2)
    a, ga, ng = S.stats()
    flush(f"  acceptance {a:.3f}, global {ga:.3f} of {ng}")
    s = host_bits(s).reshape(2, nc, -1)
    rows = np.array([0, 17, 2048, 4095])
    f = lambda b: orbm.log_psi(p, b, Nh)
    ch = omet.Chains(f, N, "made_mix", seed=77, chain_ids=rows, therm_sweeps=2, made=(pm, N, H), global_steps=G)
    os_, _ = ch.sample(2)
    for r, c in enumerate(rows):
        for k in range(2):
            assert np.array_equal(s[k, c], si.pack_bits(os_[k, r])[0]), (k, c)
    assert 0 < ch.acc_global < ch.n_global


def test_mixed_chain_histogram(ctx):
    flush("mixed histogram")
    N, Nh, H = 10, 10, 16
    # 20 thermalisation sweeps, then every 10th of 1000 sweeps: the chi-square
    # test assumes independent draws, so the kept samples must be well
    # separated compared with the chain's autocorrelation time (the exact
    # sweep kernel of this state and proposal, one global step and 10 flips,
    # has its second eigenvalue at 0.37: tau ~ 1.6 sweeps; global acceptance
    # 0.37 and flip acceptance 0.63 at stationarity)
    model, Ham, made, S, pr, pm = _mixed_setup(ctx, N, Nh, H, 0.1, 1, 1024, seed=3, therm=20, made_scale=0.5)
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
    model, Ham, made, S, pr, pm = _mixed_setup(ctx, N, Nh, H, 0.6, 1, 512, seed=11)
    S.sample(512 * 20)
    _, ga0, _ = S.stats()
    local = V.Sampler(ctx, model, Ham, proposal=V.PROP_FLIP, n_chains=1024, therm_sweeps=20, seed=12)
    data, _, _ = local.sample(1024 * 32)
    made.train(data, epochs=20, batch=256, lr=3e-3)
    S.set_proposal_made(made)
    S.sample(512 * 20)
    _, ga1, _ = S.stats()
    assert ga1 > ga0 + 0.1, (ga0, ga1)


def test_trained_proposal_decorrelates_the_order_parameter(ctx):
    # 8 x 8 bond-RBM at the 2D Ising critical coupling (local flips slow down
    # there): a MADE trained on thermalised local-chain samples, one global step
    # per sweep, lowers the integrated autocorrelation time of |M| in sweeps
    from paper_2108_03409_amd import stats as pstats
    flush("made: tau_int(|M|) mixed vs local, 8x8 critical")
    L, H, nc, R = 8, 128, 512, 400
    N = L * L
    p = si.bond_rbm_params(L, L, si.W_CRITICAL)
    Nh = (len(p) - N) // (N + 1)
    model = V.Model.rbm(ctx, N, Nh, True)
    model.set_params(dev_c128(p))
    Ham = V.Hamiltonian.tfim(ctx, L, L, True, 1.0, 3.0)
    src = V.Sampler(ctx, model, Ham, proposal=V.PROP_FLIP, n_chains=1024, therm_sweeps=200, seed=31)
    data, _, _ = src.sample(1024 * 16)
    made = V.MADE(ctx, N, H)
    made.set_params(torch.from_numpy(si.made_params(N, H, seed=205)).to("cuda:0"))
    made.train(data, epochs=40, batch=256, lr=2e-3)
    taus = {}
    for name, prop in [("local", V.PROP_FLIP), ("mixed", V.PROP_MADE_MIX)]:
        S = V.Sampler(ctx, model, Ham, proposal=prop, n_chains=nc, therm_sweeps=50, seed=41, global_steps=1)
        if prop == V.PROP_MADE_MIX:
            S.set_proposal_made(made)
        s, _, _ = S.sample(nc * R)
        pop = np.bitwise_count(host_bits(s)).sum(axis=1).astype(np.float64)
        mag = (np.abs(2.0 * pop - N) / N).reshape(R, nc)
        taus[name] = pstats.ess(mag)[1]
        if prop == V.PROP_MADE_MIX:
            flush(f"  global acceptance {S.stats()[1]:.3f}")
    flush(f"  tau_int(|M|): local {taus['local']:.2f}, mixed {taus['mixed']:.2f} sweeps")
    assert taus["mixed"] < 0.7 * taus["local"], taus
