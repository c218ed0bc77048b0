"""Throughput of the NQS-VMC hot path on one MI355X.

One step = one stochastic-reconfiguration step (the paper's Algorithm 1 plus
the parameter update): Metropolis sampling, log psi, log-derivatives O_k,
local energies, S / F with the shifted Cholesky solve, theta <- theta + tau x.

Default workload: 1D transverse-field Ising chain L = 64 (periodic, J = h = 1),
complex RBM alpha = 4 (16 704 parameters, N(0, 0.01)), 16 384 samples per step
(1024 chains x 16 sweeps of 64 single-spin-flip proposals), S from complex64
O_k on the matrix path, float64 Cholesky with relative diagonal shift 1e-3.

Prints one JSON line (rank 0): SR steps/s with per-phase times, local
energies/s, the roofline of the dominant kernel (live HIP-event timing on the
library's stream) and the FP64 oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth_inputs as si  # noqa: E402

# fp32_valu_TF: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz, without
# packed-FP32 instructions (the build disables them)
PEAK = {"hbm_GBs": 8000.0, "fp32_mfma_TF": 157.3, "fp64_TF": 78.6, "fp64_valu_TF": 78.6, "bf16_mfma_TF": 2500.0,
        "fp16_mfma_TF": 2500.0, "fp32_valu_TF": 78.6}
METRIC = "local energies/s & SR steps/s vs roofline; ESS/s learned vs local proposal"

# HBM bytes per launch of k_herk_mfma_f32 on the default workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB: the factors a
# plain 2 GiB device copy reads); reported only while herk.hip is the source
# that was profiled.
HERK_TRAFFIC = {"source_sha256_16": "56b04f15ff98737a", "bytes": 158760895488.0}


def herk_traffic():
    import hashlib
    path = os.path.join(ROOT, "paper_2108_03409_amd", "csrc", "herk.hip")
    try:
        h = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return HERK_TRAFFIC["bytes"] if h == HERK_TRAFFIC["source_sha256_16"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tfim1d_L64_rbm_a4_sr",
                    choices=["tfim1d_L64_rbm_a4_sr", "heis2d_10x10_rbm_a4", "tfim2d_16x16_cnn",
                             "tfim2d_20x20_rbm_a2_made", "tfim2d_20x20_rbm_a2_sr", "tfim1d_L50_ar_sr"])
    ap.add_argument("--global-steps", type=int, default=1,
                    help="MADE mix: global proposals of all chains at the start of every sweep")
    ap.add_argument("--record-sweeps", type=int, default=256, help="MADE mix: recorded sweeps per chain")
    ap.add_argument("--made-epochs", type=int, default=100, help="MADE mix: training epochs")
    ap.add_argument("--made-lr", type=float, default=1e-3, help="MADE mix: Adam learning rate")
    ap.add_argument("--made-hidden", type=int, default=None, help="MADE mix: hidden units (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="SR-step workload only (skip the local-energy and learned-proposal workloads)")
    ap.add_argument("--tau", type=float, default=1e-2)
    ap.add_argument("--prec", choices=["f64", "f32", "bf16"], default="f64",
                    help="network evaluation precision of log psi / local energies")
    ap.add_argument("--peaks", action="store_true",
                    help="measure HBM copy bandwidth and MFMA rates (f64, f32, bf16) instead of a workload")
    ap.add_argument("--solver", choices=["cholesky", "cg"], default="cholesky",
                    help="SR solve: dense Cholesky of S (default) or matrix-free conjugate gradient")
    ap.add_argument("--cg-tol", type=float, default=1e-8, help="conjugate gradient: relative residual target")
    ap.add_argument("--gram", type=int, choices=[0, 1], default=0,
                    help="S Gram kernel: 0 float32 matrix cores, 1 split float16 (hi + lo) matrix cores")
    return ap.parse_args()


def set_prec(V, model, prec):
    model.set_precision({"f64": V.VMC_F64, "f32": V.VMC_F32, "bf16": V.VMC_BF16}[prec])


def herk_flops(ns, K):
    """Complex Hermitian rank-ns update, lower triangle with diagonal: K(K+1)/2 outputs x ns
    complex multiply-adds x 8 real flops."""
    return 4.0 * ns * K * (K + 1)


def chol_flops(K):
    """Complex Cholesky: K^3/6 complex multiply-adds x 8 real flops (leading order)."""
    return 4.0 * K ** 3 / 3.0


def cnn_eloc_flops(N, C, k):
    """Per CNN local energy (TFIM, N flips): the forward layer-2 correlation
    (C^2 k^2 N complex multiply-adds) plus, per flip, the window change
    dZ = W2 * dA with C^2 k^4 complex multiply-adds; 8 real flops each."""
    return 8.0 * C * C * k * k * N * (1 + k * k)


def eloc_flops(N, Nh, n_slots):
    """Per local energy: theta = b + sum_i +-W_ji (2 N Nh real flops) and, per non-zero
    off-diagonal slot, N_h complex multiply, subtract and multiply (14 real flops)."""
    return 2.0 * N * Nh + 14.0 * Nh * n_slots


def cpu_baseline(cfg, p, N, Nh, n_chains, per_chain, runs=10, warm=3):
    """The float64 oracle on a bounded sample of the same step, each phase
    scaled to the full step.  Timed with the BLAS pool limited to one thread
    and to all the host threads the process may use (threadpoolctl), each the
    median over `runs` runs after `warm` warm-ups.  Per phase the speed-up of
    the second over the first shows how many of those threads it really used
    (the oracle's Metropolis, local-energy, Cholesky and solve loops are
    Python loops over small numpy operations: they stay near 1)."""
    from threadpoolctl import threadpool_limits
    from oracle import rbm as orbm, eloc as oeloc, metropolis as omet, sr as osr

    all_threads = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    f = lambda b: orbm.log_psi(p, b, Nh)
    K = len(p)
    ns_full = n_chains * per_chain
    n_ch, n_ev, n_el, n_sf, Ks, Kp = 32, 512, 64, 256, 4096, 1024
    bits = si.random_bits(n_ev, N, seed=7)
    O = orbm.grad_log_psi(p, bits, Nh)
    el = oeloc.local_energy(f, "tfim", bits[:n_el], N, 1, True, 1.0, 1.0)
    Os = np.ascontiguousarray(O[:n_sf, :Ks])
    els = np.resize(el, n_sf)
    S, F = osr.fisher_and_force(Os, els)
    A = osr.shifted(S[:Kp, :Kp], 1e-3)
    L, _, _ = osr.cholesky(A)
    del S
    work = {   # phase: (callable on the bounded sample, factor to the full step)
        "sample": (lambda: omet.Chains(f, N, "flip", seed=103, chain_ids=np.arange(n_ch), therm_sweeps=0).sample(1),
                   ns_full / n_ch),
        "log_psi": (lambda: orbm.log_psi(p, bits, Nh), ns_full / n_ev),
        "grad": (lambda: orbm.grad_log_psi(p, bits, Nh), ns_full / n_ev),
        "eloc": (lambda: oeloc.local_energy(f, "tfim", bits[:n_el], N, 1, True, 1.0, 1.0), ns_full / n_el),
        "S_F": (lambda: osr.fisher_and_force(Os, els), (ns_full / n_sf) * (K / Ks) ** 2),
        "cholesky": (lambda: osr.cholesky(A), (K / Kp) ** 3),
        "solve": (lambda: osr.back_sub_h(L, osr.forward_sub(L, -F[:Kp])), (K / Kp) ** 2),
    }
    out = {}
    for label, nthr in (("one_thread", 1), ("all_threads", all_threads)):
        wall = {k: [] for k in work}
        with threadpool_limits(limits=nthr):
            for r in range(warm + runs):
                for k, (fn, _) in work.items():
                    t0 = time.perf_counter()
                    fn()
                    if r >= warm:
                        wall[k].append(time.perf_counter() - t0)
        phase_s = {k: float(np.median(wall[k])) * work[k][1] for k in work}
        out[label] = {"value": 1.0 / sum(phase_s.values()), "blas_threads": nthr,
                      "phase_s": {k: round(v, 3) for k, v in phase_s.items()}}
    one, best = out["one_thread"], out["all_threads"]
    best["speedup_over_one_thread"] = {k: round(one["phase_s"][k] / max(best["phase_s"][k], 1e-12), 2) for k in work}
    return {
        "value": best["value"], "unit": "SR steps/s", "cores": all_threads, "kind": "oracle",
        "sample": (f"float64 oracle, median of {runs} runs after {warm} warm-ups, on: {n_ch} chains x 1 sweep "
                   f"(scaled to {n_chains} x {per_chain}), log psi and O_k on {n_ev} samples, E_loc on {n_el} "
                   f"(each scaled to {ns_full} samples), S/F on {n_sf} samples x the first {Ks} parameters (scaled "
                   f"by samples x (K/{Ks})^2), Cholesky and triangular solves on the leading {Kp} x {Kp} block of "
                   f"S~ (scaled by (K/{Kp})^3 and ^2); every phase extrapolated; value = all {all_threads} host "
                   f"threads in the BLAS pool; one_thread = the same with one"),
        "one_thread": one, "all_threads": best,
    }


def bench_eloc(args, V, torch):
    print(json.dumps(eloc_result(V, torch, args.workload, args.prec, args.steps, args.warmup)), flush=True)


def eloc_result(V, torch, workload, prec, steps, warmup):
    """Local energies/s: one step = sample + local energies of every sample."""
    cfg = si.WORKLOADS[workload]
    dev = "cuda:0"
    ctx = V.Context(0)
    Lx, Ly = cfg["Lx"], cfg["Ly"]
    N = Lx * Ly
    if cfg["net"] == "rbm":
        Nh = cfg["alpha"] * N
        p = si.rbm_params(N, Nh, std=cfg["std"], is_complex=True, seed=cfg["param_seed"])
        model = V.Model.rbm(ctx, N, Nh, True)
        # non-zero off-diagonal slots: N flips (TFIM); about N anti-aligned bonds of 2N (Heisenberg, Sz = 0)
        work = eloc_flops(N, Nh, N)
    else:
        p = si.cnn_params(cfg["channels"], cfg["kernel"], std=cfg["std"], seed=cfg["param_seed"])
        model = V.Model.cnn(ctx, Lx, Ly, cfg["channels"], cfg["kernel"])
        Nh = None
        work = cnn_eloc_flops(N, cfg["channels"], cfg["kernel"])
    model.set_params(torch.from_numpy(p).to(dev))
    if cfg["ham"] == "heisenberg":
        H = V.Hamiltonian.heisenberg(ctx, Lx, Ly, True, cfg["J"])
    else:
        H = V.Hamiltonian.tfim(ctx, Lx, Ly, True, cfg["J"], cfg["h"])
    ns = cfg["n_chains"] * cfg["samples_per_chain"]
    el = torch.empty(ns, dtype=torch.complex128, device=dev)
    sampler = V.Sampler(ctx, model, H, proposal=V.PROP_EXCHANGE if cfg["proposal"] == "exchange" else V.PROP_FLIP,
                        n_chains=cfg["n_chains"], therm_sweeps=20, seed=cfg["sampler_seed"])
    get_samples = lambda: sampler.sample(ns)[0]
    set_prec(V, model, prec)

    last = {}

    def step():
        s = get_samples()
        model.local_energy(H, s, out=el)
        last["s"] = s

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    eloc_ms = ctx.get_timing("eloc")[0] / steps
    samp_ms = ctx.get_timing("sample")[0] / steps
    ctx.set_timing(False)
    ms_step = (t1 - t0) * 1e3 / steps
    out = {
        "metric": METRIC, "value": round(ns / (ms_step * 1e-3), 1), "unit": "local energies/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic", "config": {"workload": workload, "samples": ns},
        "phases_ms": {"sample": round(samp_ms, 3), "eloc": round(eloc_ms, 3)},
        "eloc_kernel_per_s": round(ns / (eloc_ms * 1e-3), 1),
        "mean_energy": float(el.real.mean().item()),
    }
    if prec != "f64":
        # the error of this precision against the float64 path (itself pinned to
        # the oracle at 1e-10) on the first 4 096 samples of the last step
        nref = min(ns, 4096)
        set_prec(V, model, "f64")
        ref = model.local_energy(H, last["s"][:nref])
        set_prec(V, model, prec)
        got = el[:nref]
        rel = ((got - ref).abs() / ref.abs().clamp_min(1e-300)).max().item()
        out["error_vs_f64"] = {"samples": nref, "max_rel_eloc": float(rel),
                               "rel_mean_energy": float(abs((got.mean() - ref.mean()) / ref.mean()).item())}
    achieved = ns * work / (eloc_ms * 1e-3) / 1e12
    effective = None
    if cfg["net"] == "cnn" and prec == "f32":
        # the float32 window products issue three real products per complex term
        # (6 flops per multiply-add); the conventional count is kept as effective_TF
        C, k = cfg["channels"], cfg["kernel"]
        effective = achieved
        work = 8.0 * C * C * k * k * N + 6.0 * C * C * k ** 4 * N
        achieved = ns * work / (eloc_ms * 1e-3) / 1e12
    if cfg["net"] == "cnn" and prec != "f64":
        peak, bound = (PEAK["bf16_mfma_TF"], "mfma") if prec == "bf16" else (PEAK["fp32_mfma_TF"], "mfma")
        kern = f"k_cnn_eloc_lp<{prec}>"
    elif cfg["net"] == "cnn":
        peak, bound, kern = PEAK["fp64_valu_TF"], "alu", "k_cnn_eloc"
    else:
        # the slot ratios (14 N_h flop per slot) are vector ALU work: float64,
        # or float32 without packed instructions in the low-precision path
        peak, bound = PEAK["fp64_valu_TF"] if prec == "f64" else PEAK["fp32_valu_TF"], "alu"
        kern = "k_eloc" if prec == "f64" else "k_eloc_lowp"
    out["roofline"] = {"kernel": kern, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
                       "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                       "work": f"{work:.4e} flop per local energy x {ns} per launch"}
    if effective is not None:
        out["roofline"]["effective_TF"] = round(effective, 3)
    return out


def bench_made(args, V, torch):
    print(json.dumps(made_result(V, torch, args.workload, args.global_steps, args.record_sweeps, args.made_epochs,
                                 args.made_lr, args.made_hidden)), flush=True)


def made_result(V, torch, workload, global_steps, record_sweeps, made_epochs, made_lr, made_hidden=None):
    """Effective samples/s of the energy series: trained MADE mixed with flips
    against flips alone, on the critical bond-RBM state of a 20 x 20 lattice."""
    from paper_2108_03409_amd import stats as pstats

    cfg = si.WORKLOADS[workload]
    dev = "cuda:0"
    Lx, Ly = cfg["Lx"], cfg["Ly"]
    N = Lx * Ly
    ctx = V.Context(0)
    p = si.bond_rbm_params(Lx, Ly, si.W_CRITICAL)
    Nh = (len(p) - N) // (N + 1)
    model = V.Model.rbm(ctx, N, Nh, True)
    model.set_params(torch.from_numpy(p).to(dev))
    H = V.Hamiltonian.tfim(ctx, Lx, Ly, True, cfg["J"], cfg["h"])
    nc = cfg["n_chains"]
    # training data from thermalised local chains
    t0 = time.perf_counter()
    src = V.Sampler(ctx, model, H, proposal=V.PROP_FLIP, n_chains=nc, therm_sweeps=200, seed=cfg["sampler_seed"] + 1000)
    data, _, _ = src.sample(cfg["train_samples"])
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    mh = made_hidden or cfg["made_hidden"]
    made = V.MADE(ctx, N, mh)
    made.set_params(torch.from_numpy(si.made_params(N, mh, seed=cfg["made_seed"])).to(dev))
    t0 = time.perf_counter()
    nll = made.train(data, epochs=made_epochs, batch=1024, lr=made_lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    G = global_steps
    R = record_sweeps
    res = {}
    for name, prop in [("local", V.PROP_FLIP), ("mixed", V.PROP_MADE_MIX)]:
        S = V.Sampler(ctx, model, H, proposal=prop, n_chains=nc, therm_sweeps=100, seed=cfg["sampler_seed"],
                      global_steps=G)
        if prop == V.PROP_MADE_MIX:
            S.set_proposal_made(made)
        S.sample(nc)                       # thermalisation + one sweep, untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, _, acc = S.sample(nc * R)
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        a, ga, ng = S.stats()
        el = model.local_energy(H, s).real.cpu().numpy().reshape(R, nc)
        n_eff, tau = pstats.ess(el)
        # |magnetisation| per site: the slow observable of the critical state
        pop = np.bitwise_count(s.cpu().numpy().view(np.uint64)).sum(axis=1).astype(np.float64)
        mag = (np.abs(2.0 * pop - N) / N).reshape(R, nc)
        m_eff, m_tau = pstats.ess(mag)
        res[name] = {"ess": n_eff, "tau_int_sweeps": tau, "sample_s": t_s, "ess_per_s": n_eff / t_s,
                     "accept": a, "global_accept": ga, "n_global": ng,
                     "energy": float(el.mean()), "sigma_energy": float(np.sqrt(el.var() / n_eff)),
                     "ess_abs_m": m_eff, "tau_int_abs_m_sweeps": m_tau, "ess_abs_m_per_s": m_eff / t_s,
                     "abs_m": float(mag.mean())}
    ratio = res["mixed"]["ess_per_s"] / res["local"]["ess_per_s"]
    out = {
        "metric": METRIC, "value": round(res["mixed"]["ess_per_s"], 2), "unit": "effective samples/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(res["mixed"]["sample_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (bond-RBM at the 2D Ising critical coupling)",
        "config": {"workload": workload, "n_chains": nc, "record_sweeps": R, "global_steps": G,
                   "made_hidden": mh, "train_samples": cfg["train_samples"], "made_epochs": made_epochs,
                   "made_lr": made_lr},
        "local": res["local"], "mixed": res["mixed"], "ess_per_s_ratio_mixed_over_local": round(ratio, 3),
        "abs_m_ess_per_s_ratio_mixed_over_local": round(res["mixed"]["ess_abs_m_per_s"] /
                                                        res["local"]["ess_abs_m_per_s"], 3),
        # the same ratio with the proposal's training and its data charged to the mixed run
        "ess_per_s_ratio_incl_training": round(res["mixed"]["ess"] / (res["mixed"]["sample_s"] + t_train + t_data) /
                                               res["local"]["ess_per_s"], 3),
        "train_s": round(t_train, 3), "train_data_s": round(t_data, 3), "final_nll": nll,
    }
    return out


def ar_eloc_flops(N, H):
    """Multiply-adds (2 flop each) one TFIM local energy of the autoregressive
    state needs: the forward pass (live W1 and W2 entries) plus, per flipped
    site d, the hidden units of degree > d and the live W2 entries leaving them."""
    m = np.arange(H) % (N - 1) + 1
    fwd = m.sum() + (N - m).sum()
    per = sum(int((m > d).sum() + (N - m[m > d]).sum()) for d in range(N))
    return 2.0 * (fwd + per)


def bench_ar_sr(args, V, torch):
    """SR steps/s of the autoregressive state: one step = direct samples,
    O_k, local energies, the shifted solve of the real SR equation, update."""
    cfg = si.WORKLOADS[args.workload]
    dev = "cuda:0"
    N, Hh = cfg["Lx"] * cfg["Ly"], cfg["hidden"]
    ns = cfg["n_chains"] * cfg["samples_per_chain"]
    ctx = V.Context(0)
    model = V.Model.autoregressive(ctx, N, Hh)
    K = model.K
    theta = torch.from_numpy(si.ar_params(N, Hh, seed=cfg["param_seed"], std=cfg["std"])).to(dev)
    model.set_params(theta)
    H = V.Hamiltonian.tfim(ctx, cfg["Lx"], cfg["Ly"], cfg["periodic"], cfg["J"], cfg["h"])
    sampler = V.Sampler(ctx, model, H, n_chains=cfg["n_chains"], seed=cfg["sampler_seed"])
    O = torch.empty((ns, K), dtype=torch.float32, device=dev)  # real parameters: real O_k
    el = torch.empty(ns, dtype=torch.complex128, device=dev)

    def step():
        nonlocal theta
        s, _, _ = sampler.sample(ns)
        model.grad_log_psi(s, out=O)
        model.local_energy(H, s, out=el)
        x, info = V.sr_solve(ctx, O, el, nu_rel=cfg["nu_rel"], eps_abs=cfg["eps_abs"], mode=V.SR_REAL)
        theta = theta + args.tau * x.real
        model.set_params(theta)
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = {}
    for ph in ["sample", "grad", "eloc", "sr.center", "sr.herk", "sr.chol", "sr.trsv", "sr.resid"]:
        ms, n = ctx.get_timing(ph)
        phases[ph] = round(ms / max(n, 1), 3)
    ctx.set_timing(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    herk_ms = phases["sr.herk"]
    # real S = Obar^T Obar, lower triangle: Ns K (K + 1) flop (two real samples per complex row)
    real_flops = herk_flops(ns, K) / 4.0
    herk_achieved = real_flops / (herk_ms * 1e-3) / 1e12
    eloc_ms = phases["eloc"]
    ew = ar_eloc_flops(N, Hh)
    out = {
        "metric": METRIC, "value": round(1e3 / ms_step, 4), "unit": "SR steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (S Gram from real f32 O_k on f32 matrix cores)",
        "data": "synthetic (seeded autoregressive-state parameters N(0, 0.1), direct samples)",
        "config": {"workload": (f"SR step ({args.workload}): TFIM chain L={N} PBC J={cfg['J']} h={cfg['h']}, "
                                f"autoregressive state (masked network, {Hh} hidden units, K={K} live real "
                                f"parameters), {ns} direct samples, nu_rel={cfg['nu_rel']}, "
                                f"eps_abs={cfg['eps_abs']}"),
                   "global_batch": ns, "K": K, "parallelism": "single GPU"},
        "phases_ms": phases,
        "local_energies_per_s": round(ns / (eloc_ms * 1e-3), 1),
        "eloc_roofline": {"kernel": "k_ar_eloc", "bound": "alu",
                          "achieved_TF": round(ns * ew / (eloc_ms * 1e-3) / 1e12, 3),
                          "peak": PEAK["fp64_valu_TF"], "work": f"{ew:.4e} flop (multiply-adds) per local energy"},
        "grad_GBs": round(4.0 * ns * K / (phases["grad"] * 1e-3) / 1e9, 1),
        "roofline": {"kernel": "k_herk_mfma_f32<real> + k_herk_reduce (S = Obar^T Obar, sample range split)",
                     "bound": "mfma", "achieved": round(herk_achieved, 3), "peak": PEAK["fp32_mfma_TF"],
                     "unit": "TFLOP/s", "frac": round(herk_achieved / PEAK["fp32_mfma_TF"], 4), "traffic": None,
                     "work": f"Ns*K*(K+1) = {real_flops:.4e} flop per solve (Ns={ns}, K={K})"},
        "energy": infos[-1]["e_mean"].real, "energy_per_site": infos[-1]["e_mean"].real / N,
        "residual": infos[-1]["residual"],
    }
    print(json.dumps(out), flush=True)


def bench_peaks(args, V, torch):
    """Measured peaks next to the nominal ones: a 16-byte-vector device copy of
    2 GiB (4 GiB moved) and the MFMA loops, each timed with HIP events on the
    library's stream over `steps` launches after `warmup`."""
    ctx = V.Context(0)
    nb = 2 << 30
    src = torch.empty(nb // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    out = {"metric": "measured peaks", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup}
    for _ in range(args.warmup):
        V.calib_copy(ctx, src, dst)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(args.steps):
        V.calib_copy(ctx, src, dst)
    ms, n = ctx.get_timing("calib.copy")
    ctx.set_timing(False)
    gbs = 2 * nb * n / (ms * 1e-3) / 1e9
    out["hbm_copy"] = {"GB/s": round(gbs, 1), "nominal": PEAK["hbm_GBs"], "frac": round(gbs / PEAK["hbm_GBs"], 4),
                       "bytes_moved_per_launch": 2 * nb, "ms_per_launch": round(ms / n, 4)}
    for _ in range(args.warmup):
        V.calib_read(ctx, src)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(args.steps):
        V.calib_read(ctx, src)
    ms, n = ctx.get_timing("calib.read")
    ctx.set_timing(False)
    gbs = nb * n / (ms * 1e-3) / 1e9
    out["hbm_read"] = {"GB/s": round(gbs, 1), "nominal": PEAK["hbm_GBs"], "frac": round(gbs / PEAK["hbm_GBs"], 4),
                       "bytes_read_per_launch": nb, "ms_per_launch": round(ms / n, 4)}
    nominal = {"f64": PEAK["fp64_TF"], "f32": PEAK["fp32_mfma_TF"], "bf16": PEAK["bf16_mfma_TF"]}
    for kind, iters in [("f64", 2000), ("f32", 2000), ("bf16", 1000)]:
        for _ in range(args.warmup):
            V.calib_mfma(ctx, kind, 2048, iters)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        fl = 0.0
        for _ in range(args.steps):
            fl += V.calib_mfma(ctx, kind, 2048, iters)
        ms, n = ctx.get_timing("calib.mfma")
        ctx.set_timing(False)
        tf = fl / (ms * 1e-3) / 1e12
        out[f"mfma_{kind}"] = {"TFLOP/s": round(tf, 1), "nominal": nominal[kind], "frac": round(tf / nominal[kind], 4),
                               "ms_per_launch": round(ms / n, 4)}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; sharding over several GPUs is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2108_03409_amd import nqsvmc as V

    if args.peaks:
        return bench_peaks(args, V, torch)
    if args.workload in ("heis2d_10x10_rbm_a4", "tfim2d_16x16_cnn"):
        return bench_eloc(args, V, torch)
    if args.workload == "tfim2d_20x20_rbm_a2_made":
        return bench_made(args, V, torch)
    if args.workload == "tfim1d_L50_ar_sr":
        return bench_ar_sr(args, V, torch)

    cfg = si.WORKLOADS[args.workload]
    N = cfg["Lx"] * cfg["Ly"]
    Nh = cfg["alpha"] * N
    n_chains, per_chain = cfg["n_chains"], cfg["samples_per_chain"]
    ns = n_chains * per_chain
    dev = "cuda:0"

    p = si.rbm_params(N, Nh, std=cfg["std"], is_complex=True, seed=cfg["param_seed"])
    ctx = V.Context(0)
    model = V.Model.rbm(ctx, N, Nh, True)
    K = model.K
    if K > 65536:
        args.solver = "cg"  # a dense K x K S would not fit: the matrix-free solve is the only option
    theta = torch.from_numpy(p).to(dev)
    model.set_params(theta)
    set_prec(V, model, args.prec)
    H = V.Hamiltonian.tfim(ctx, cfg["Lx"], cfg["Ly"], cfg["periodic"], cfg["J"], cfg["h"])
    sampler = V.Sampler(ctx, model, H, proposal=V.PROP_FLIP, n_chains=n_chains, therm_sweeps=20,
                        seed=cfg["sampler_seed"])
    O = torch.empty((ns, K), dtype=torch.complex64, device=dev)
    el = torch.empty(ns, dtype=torch.complex128, device=dev)

    def step():
        nonlocal theta
        s, _, acc = sampler.sample(ns)
        model.grad_log_psi(s, out=O)
        model.local_energy(H, s, out=el)
        if args.solver == "cg":
            x, info = V.sr_solve_cg(ctx, O, el, nu_rel=cfg["nu_rel"], tol=args.cg_tol, max_iter=5000)
        else:
            x, info = V.sr_solve(ctx, O, el, nu_rel=cfg["nu_rel"], gram=args.gram)
        theta = theta + args.tau * x
        model.set_params(theta)
        return info, acc

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = {}
    for ph in ["sample", "log_psi", "grad", "eloc", "sr.center", "sr.herk", "sr.chol", "sr.trsv", "sr.cg", "sr.resid"]:
        ms, n = ctx.get_timing(ph)
        phases[ph] = round(ms / max(n, 1), 3)
    ctx.set_timing(False)
    ms_step = (t1 - t0) * 1e3 / args.steps

    if args.solver == "cg":
        # dominant kernels: the two passes over O per CG product (HBM-bound)
        iters = infos[-1][0]["iterations"] + 1  # + the true-residual product
        cg_ms = phases["sr.cg"] + phases["sr.resid"]
        gbs = iters * 2 * 8.0 * ns * K / (cg_ms * 1e-3) / 1e9
        roofline = {"kernel": "k_ov + k_ohu (S v = Obar^H (Obar v), two passes over complex64 O)", "bound": "hbm",
                    "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                    "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": None,
                    "work": f"2 x 8 Ns K = {16.0 * ns * K:.4e} bytes per product, {iters} products"}
    else:
        # dominant kernel: the Gram (S) kernel, one launch per step.  It forms
        # each complex product from three real ones (Gauss's identity), so the
        # matrix-core work its algorithm needs is 3/4 of the conventional
        # complex count 4 Ns K (K + 1); the latter is kept as effective_TF.
        herk_ms = phases["sr.herk"]
        conv = herk_flops(ns, K)
        work = 0.75 * conv if args.gram == 0 else conv
        herk_achieved = work / (herk_ms * 1e-3) / 1e12
        hpeak = PEAK["fp32_mfma_TF"] if args.gram == 0 else PEAK["fp16_mfma_TF"]
        hname = ("k_herk_c_dma<12,3> (S = Obar^H Obar, float32 matrix cores, three real products per complex term)"
                 if args.gram == 0 else "k_herk16 (S = Obar^H Obar, split-float16 matrix cores)")
        roofline = {"kernel": hname, "bound": "mfma", "achieved": round(herk_achieved, 3),
                    "peak": hpeak, "unit": "TFLOP/s", "frac": round(herk_achieved / hpeak, 4),
                    "traffic": herk_traffic() if args.gram == 0 else None,
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)",
                    "algorithmic_bytes": 8.0 * ns * K + 16.0 * K * K,
                    "work": (f"3*Ns*K*(K+1) = {work:.4e} flop per launch (Ns={ns}, K={K}): three real "
                             "products per complex term, lower triangle with the diagonal" if args.gram == 0 else
                             f"4*Ns*K*(K+1) = {work:.4e} flop per launch (Ns={ns}, K={K})"),
                    "effective_TF": round(conv / (herk_ms * 1e-3) / 1e12, 3),
                    "effective_work": f"4*Ns*K*(K+1) = {conv:.4e} flop, the conventional complex count"}
    # the reverse-mode product of log psi (the autograd backward) at the same batch,
    # outside the timed steps: out_k = sum_n g_n conj(O_nk), O recomputed, never stored
    s_last, _, _ = sampler.sample(ns)
    gvec = torch.randn(ns, dtype=torch.complex128, device=dev)
    model.log_psi_vjp(s_last, gvec)
    ctx.set_timing(True)
    for _ in range(5):
        model.log_psi_vjp(s_last, gvec)
    vjp_ms = ctx.get_timing("vjp")[0] / 5
    ctx.set_timing(False)
    chol_ms = phases["sr.chol"]
    eloc_ms = phases["eloc"]
    eloc_per_s = ns / (eloc_ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_step, 4),
        "unit": "SR steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("c64 O_k; S on the " + ("float32 matrix cores (3 real products per complex term)"
                  if args.gram == 0 else "float16 matrix cores (split hi+lo)") +
                  "; f64 E_loc, Cholesky and triangular solves"),
        "data": "synthetic (seeded RBM parameters N(0,0.01), Metropolis samples)",
        "config": {"workload": (f"SR step ({args.workload}): TFIM {cfg['Lx']}x{cfg['Ly']} PBC J={cfg['J']} "
                                f"h={cfg['h']}, complex RBM alpha={cfg['alpha']} (K={K}), {ns} samples "
                                f"({n_chains} chains x {per_chain} sweeps), nu_rel={cfg['nu_rel']}"),
                   "global_batch": ns, "K": K, "parallelism": "single GPU", "gram": args.gram, "prec": args.prec,
                   "solver": args.solver},
        "phases_ms": phases,
        "local_energies_per_s": round(eloc_per_s, 1),
        "eloc_roofline": {"kernel": "k_eloc<4>", "bound": "alu",
                          "achieved_TF": round(ns * eloc_flops(N, Nh, N) / (eloc_ms * 1e-3) / 1e12, 3),
                          "peak": PEAK["fp64_valu_TF"]},
        "chol_TF": round(chol_flops(K) / (chol_ms * 1e-3) / 1e12, 3) if chol_ms > 0 else None,
        "log_psi_vjp_ms": round(vjp_ms, 3),
        "roofline": roofline,
        "energy": infos[-1][0]["e_mean"].real, "residual": infos[-1][0]["residual"],
        "cg_iterations": infos[-1][0].get("iterations"),
        "accept": round(infos[-1][1], 4),
    }
    if not args.no_cpu_baseline and args.workload == "tfim1d_L64_rbm_a4_sr":
        out["cpu_baseline"] = cpu_baseline(cfg, p, N, Nh, n_chains, per_chain)
    if not args.no_extra and args.workload == "tfim1d_L64_rbm_a4_sr":
        out["other_workloads"] = other_workloads(V, torch)
    print(json.dumps(out), flush=True)


def other_workloads(V, torch):
    """The rest of the metric on its own workloads, short runs: local
    energies/s of the Heisenberg RBM (bfloat16 and float64) and of the CNN
    (bfloat16 and float32), and the learned proposal's effective samples/s
    against local moves (64 recorded sweeps)."""
    res = {}
    for name, wl, prec, steps, warm in [("heis2d_10x10_rbm_a4_bf16", "heis2d_10x10_rbm_a4", "bf16", 10, 3),
                                        ("heis2d_10x10_rbm_a4_f64", "heis2d_10x10_rbm_a4", "f64", 10, 3),
                                        ("tfim2d_16x16_cnn_bf16", "tfim2d_16x16_cnn", "bf16", 3, 1),
                                        ("tfim2d_16x16_cnn_f32", "tfim2d_16x16_cnn", "f32", 3, 1)]:
        r = eloc_result(V, torch, wl, prec, steps, warm)
        res[name] = {"local_energies_per_s": r["value"], "eloc_kernel_per_s": r["eloc_kernel_per_s"],
                     "ms_per_step": r["ms_per_step"], "phases_ms": r["phases_ms"], "roofline": r["roofline"]}
        if "error_vs_f64" in r:
            res[name]["error_vs_f64"] = r["error_vs_f64"]
        torch.cuda.empty_cache()
    m = made_result(V, torch, "tfim2d_20x20_rbm_a2_made", 1, 64, 100, 1e-3)
    res["tfim2d_20x20_rbm_a2_made"] = {
        k: m[k] for k in ("ess_per_s_ratio_mixed_over_local", "abs_m_ess_per_s_ratio_mixed_over_local",
                          "ess_per_s_ratio_incl_training", "train_s", "final_nll")}
    for side in ("local", "mixed"):
        res["tfim2d_20x20_rbm_a2_made"][side] = {
            k: m[side][k] for k in ("ess_per_s", "tau_int_sweeps", "ess_abs_m_per_s", "tau_int_abs_m_sweeps",
                                    "sample_s", "global_accept", "sigma_energy")}
    return res


if __name__ == "__main__":
    main()
