"""Ground-state search of the periodic TFIM chain with the translation-symmetric
ELU network, following the paper's example (Sec. 5.1): SR with learning rate
tau, N_MC Monte Carlo samples per step, diagonal shift nu_n = nu_0 0.95^n and a
pseudo-inverse cutoff.  Prints one JSON line per report interval and a final
line with the deviation from the exact energy of the Pfeuty solution.

    python -m paper_2108_03409_amd.ground_state --L 20 --alpha 2 --steps 1000
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time


def pfeuty_energy(L: int, g: float) -> float:
    """Exact ground-state energy of H = -sum Z Z - g sum X on a periodic chain of
    L sites (even-parity sector, fermion momenta pi (2 m + 1) / L)."""
    return -sum(math.sqrt(1.0 + g * g - 2.0 * g * math.cos(math.pi * (2 * m + 1) / L)) for m in range(L))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=10)
    ap.add_argument("--alpha", type=int, default=2)
    ap.add_argument("--g", type=float, default=0.7)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--samples", type=int, default=40000)
    ap.add_argument("--chains", type=int, default=4000)
    ap.add_argument("--tau", type=float, default=1e-2)
    ap.add_argument("--nu0", type=float, default=10.0)
    ap.add_argument("--nu-min", type=float, default=0.0, help="floor of the decaying diagonal shift")
    ap.add_argument("--therm", type=int, default=20, help="thermalisation sweeps of the chains")
    ap.add_argument("--eps-pinv", type=float, default=1e-8)
    ap.add_argument("--init-std", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--report", type=int, default=100)
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import nqsvmc as V
    from .driver import GroundStateSearch, geometric_shift

    ctx = V.Context(0)
    model = V.Model.symelu(ctx, args.L, args.alpha)
    ham = V.Hamiltonian.tfim(ctx, args.L, 1, True, 1.0, args.g)
    rng = np.random.default_rng(args.seed)
    theta = torch.from_numpy(rng.normal(0.0, args.init_std, model.K).astype(np.complex128)).to(f"cuda:{ctx.device}")
    per_chain = -(-args.samples // args.chains)
    gs = GroundStateSearch(ctx, model, ham, theta, n_chains=args.chains, sweeps_per_step=per_chain, tau=args.tau,
                           nu=geometric_shift(args.nu0, 0.95, args.nu_min), mode=V.SR_REAL, o_dtype=torch.float64,
                           eps_pinv=args.eps_pinv, therm_sweeps=args.therm, seed=args.seed)
    e0 = pfeuty_energy(args.L, args.g)
    t0 = time.perf_counter()
    tail = []
    for n in range(args.steps):
        info = gs.step()
        e, var = info["e_mean"].real, info["e_var"]
        tail.append((e, var))
        if (n + 1) % args.report == 0 or n + 1 == args.steps:
            print(json.dumps({"step": n + 1, "energy": e, "rel_error": (e - e0) / abs(e0), "variance": var,
                              "accept": info["accept"], "seconds": round(time.perf_counter() - t0, 2)}), flush=True)
    last = tail[-min(50, len(tail)):]
    em = sum(x[0] for x in last) / len(last)
    vm = sum(x[1] for x in last) / len(last)
    print(json.dumps({"L": args.L, "alpha": args.alpha, "g": args.g, "K": model.K, "samples_per_step":
                      per_chain * args.chains, "steps": args.steps, "E0": e0, "energy_last50": em,
                      "rel_error_last50": (em - e0) / abs(e0), "variance_last50": vm,
                      "seconds": round(time.perf_counter() - t0, 2)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
