"""Ground-state search by stochastic reconfiguration on the library's kernels.

One iteration is Algorithm 1 of the paper followed by the Euler update of
imaginary-time TDVP (Sec. 3.1): draw samples with the Metropolis chains, form
O_k and the local energies, solve (S + nu_n diag S + eps I) x = -F, and set
theta <- theta + tau x.  The diagonal shift decays geometrically, as in the
ground-state example of Sec. 5 (nu_n = max(nu_0 q^n, nu_min)).  Every step of
the iteration runs in the HIP library; this module only sequences the calls.
"""
from __future__ import annotations

import torch

from . import nqsvmc as V


def geometric_shift(nu0: float = 10.0, q: float = 0.95, nu_min: float = 1e-3):
    return lambda n: max(nu0 * q ** n, nu_min)


class GroundStateSearch:
    def __init__(self, ctx: V.Context, model: V.Model, ham: V.Hamiltonian, theta: torch.Tensor, *,
                 n_chains: int = 256, sweeps_per_step: int = 8, tau: float = 0.05, nu=None,
                 eps_abs: float = 0.0, mode: int = V.SR_COMPLEX, o_dtype=torch.complex64, gram: int = 0,
                 proposal: int = V.PROP_FLIP, therm_sweeps: int = 20, seed: int = 1):
        self.ctx, self.model, self.ham = ctx, model, ham
        self.theta = theta.to(torch.complex128).contiguous()
        self.model.set_params(self.theta)
        self.sampler = V.Sampler(ctx, model, ham, proposal=proposal, n_chains=n_chains,
                                 therm_sweeps=therm_sweeps, seed=seed)
        self.n_samples = n_chains * sweeps_per_step
        self.tau, self.eps_abs, self.mode, self.gram = tau, eps_abs, mode, gram
        self.nu = nu if nu is not None else geometric_shift()
        dev = self.theta.device
        self.O = torch.empty((self.n_samples, model.K), dtype=o_dtype, device=dev)
        self.el = torch.empty(self.n_samples, dtype=torch.complex128, device=dev)
        self.n = 0

    def step(self) -> dict:
        s, _, acc = self.sampler.sample(self.n_samples)
        self.model.grad_log_psi(s, out=self.O)
        self.model.local_energy(self.ham, s, out=self.el)
        x, info = V.sr_solve(self.ctx, self.O, self.el, nu_rel=self.nu(self.n), eps_abs=self.eps_abs,
                             mode=self.mode, gram=self.gram)
        self.theta = self.theta + self.tau * x
        self.model.set_params(self.theta)
        self.n += 1
        info["accept"] = acc
        info["step"] = self.n
        return info

    def run(self, n_steps: int, callback=None) -> list:
        out = []
        for _ in range(n_steps):
            info = self.step()
            out.append(info)
            if callback is not None:
                callback(info)
        return out
