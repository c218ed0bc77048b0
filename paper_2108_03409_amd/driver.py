"""Ground-state search by stochastic reconfiguration on the library's kernels.

One iteration is Algorithm 1 of the paper followed by the Euler update of
imaginary-time TDVP (Sec. 3.1): draw samples with the Metropolis chains, form
O_k and the local energies, solve (S + nu_n diag S + eps I) x = -F (through the
pseudo-inverse of that matrix when a cutoff eps_pinv is given, as in the
paper's ground-state example), and set theta <- theta + tau x.  The diagonal shift decays geometrically, as in the
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
                 proposal: int = V.PROP_FLIP, therm_sweeps: int = 20, seed: int = 1, eps_pinv: float = 0.0):
        self.ctx, self.model, self.ham = ctx, model, ham
        self.theta = theta.to(torch.complex128).contiguous()
        self.model.set_params(self.theta)
        self.sampler = V.Sampler(ctx, model, ham, proposal=proposal, n_chains=n_chains,
                                 therm_sweeps=therm_sweeps, seed=seed)
        self.n_samples = n_chains * sweeps_per_step
        self.tau, self.eps_abs, self.mode, self.gram = tau, eps_abs, mode, gram
        self.eps_pinv = eps_pinv  # > 0: pseudo-inverse cutoff on top of the diagonal shift (Sec. 3.3)
        self.nu = nu if nu is not None else geometric_shift()
        dev = self.theta.device
        self.O = torch.empty((self.n_samples, model.K), dtype=o_dtype, device=dev)
        self.el = torch.empty(self.n_samples, dtype=torch.complex128, device=dev)
        self.n = 0

    def step(self) -> dict:
        s, _, acc = self.sampler.sample(self.n_samples)
        self.model.grad_log_psi(s, out=self.O)
        self.model.local_energy(self.ham, s, out=self.el)
        if self.eps_pinv > 0.0:
            x, info = V.sr_solve_eig(self.ctx, self.O, self.el, nu_rel=self.nu(self.n), eps_abs=self.eps_abs,
                                     mode=self.mode, gram=self.gram, eps_pinv=self.eps_pinv)
        else:
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


class TDVP:
    """Time-dependent variational principle (Sec. 3): theta' = x with
    (S + eps I) x = -[[gamma F]], gamma = i for real time (psi' = -i H psi) and
    gamma = 1 for imaginary time, integrated by the Euler or the second-order
    Heun scheme of the paper's integrator options.  Expectations come either
    from Metropolis samples of the library's sampler or, for small systems,
    from all 2^N configurations weighted by |psi|^2 (exact TDVP).  The paper
    advises against the diagonal shift for time evolution, so only a small
    additive eps_abs regularises S by default."""

    def __init__(self, ctx: V.Context, model: V.Model, ham: V.Hamiltonian, theta: torch.Tensor, *,
                 real_time: bool = True, eps_abs: float = 1e-8, nu_rel: float = 0.0, exact_states=None,
                 sampler: V.Sampler | None = None, n_samples: int = 0, mode: int = V.SR_COMPLEX,
                 eps_pinv: float = 0.0, soft_pinv: bool = True, eps_snr: float = 0.0):
        self.ctx, self.model, self.ham = ctx, model, ham
        self.theta = theta.to(torch.complex128).contiguous()
        self.gamma = 1j if real_time else 1.0
        self.eps_abs, self.nu_rel, self.mode = eps_abs, nu_rel, mode
        # eigen-decomposition regularisation (Sec. 3.3) when a cutoff is set
        self.eps_pinv, self.soft_pinv, self.eps_snr = eps_pinv, soft_pinv, eps_snr
        self.states = exact_states  # device (2^N, W) int64 or None
        self.sampler, self.n_samples = sampler, n_samples
        self.t = 0.0
        self.last_info = None

    def _batch(self):
        if self.states is not None:
            lp = self.model.log_psi(self.states)
            w = torch.exp(2.0 * (lp.real - lp.real.max()))
            return self.states, (w / w.sum()).contiguous()
        s, _, _ = self.sampler.sample(self.n_samples)
        return s, None

    def rhs(self, theta: torch.Tensor) -> torch.Tensor:
        self.model.set_params(theta.contiguous())
        s, w = self._batch()
        O = self.model.grad_log_psi(s, torch.complex128)
        el = self.model.local_energy(self.ham, s)
        if self.eps_pinv > 0.0 or self.eps_snr > 0.0:
            x, info = V.sr_solve_eig(self.ctx, O, el, weights=w, nu_rel=self.nu_rel, eps_abs=self.eps_abs,
                                     mode=self.mode, gamma=self.gamma, eps_pinv=self.eps_pinv, soft=self.soft_pinv,
                                     eps_snr=self.eps_snr)
        else:
            x, info = V.sr_solve(self.ctx, O, el, weights=w, nu_rel=self.nu_rel, eps_abs=self.eps_abs,
                                 mode=self.mode, gamma=self.gamma)
        self.last_info = info
        return x

    def fisher_norm(self, theta: torch.Tensor, v: torch.Tensor) -> float:
        """(1 / N_p) sqrt(v^dagger S v) with S at theta (Sec. 4.3 "Stepper")."""
        self.model.set_params(theta.contiguous())
        s, w = self._batch()
        O = self.model.grad_log_psi(s, torch.complex128)
        q = V.fisher_quad(self.ctx, O, v, weights=w)
        return max(q, 0.0) ** 0.5 / v.numel()

    def step_adaptive(self, stepper: "AdaptiveHeun") -> dict:
        """One accepted step of the adaptive Heun integrator; the step size is
        stepper.dt on entry and is updated for the next step."""
        theta0 = self.theta
        t_new, theta, dt_used = stepper.step(self.t, lambda y: self.rhs(y), theta0,
                                             lambda v: self.fisher_norm(theta0, v))
        self.theta = theta
        self.model.set_params(self.theta)
        self.t = t_new
        info = dict(self.last_info or {})
        info["dt"] = dt_used
        return info

    def step(self, dt: float, method: str = "heun") -> dict:
        k1 = self.rhs(self.theta)
        if method == "euler":
            self.theta = self.theta + dt * k1
        elif method == "heun":
            k2 = self.rhs(self.theta + dt * k1)
            self.theta = self.theta + 0.5 * dt * (k1 + k2)
        else:
            raise ValueError("method must be 'euler' or 'heun'")
        self.model.set_params(self.theta)
        self.t += dt
        return self.last_info


class AdaptiveHeun:
    """Second-order adaptive integrator of the paper's stepper module (Sec. 4.3):
    one Heun step of size tau and two of size tau / 2 give y^(tau) and
    y^(tau/2); with delta = ||y^(tau) - y^(tau/2)|| the step size becomes
    tau (eps / delta)^(1/3).  Readings: a step is accepted when delta <= eps
    (otherwise it is recomputed with the reduced tau), the accepted value is the
    two-half-step solution, and the factor is clamped to [min_factor, max_factor].
    f(y) returns dy/dt; norm(v) is the user's measure (e.g. the Fisher norm)."""

    def __init__(self, dt: float = 1e-3, tol: float = 1e-6, min_factor: float = 0.2, max_factor: float = 2.0,
                 dt_min: float = 1e-12, dt_max: float = float("inf"), max_tries: int = 50):
        self.dt, self.tol = dt, tol
        self.min_factor, self.max_factor = min_factor, max_factor
        self.dt_min, self.dt_max, self.max_tries = dt_min, dt_max, max_tries
        self.n_rejected = 0

    @staticmethod
    def _heun(f, y, k1, h):
        return y + 0.5 * h * (k1 + f(y + h * k1))

    def step(self, t, f, y, norm):
        """Returns (t + tau_used, y_new, tau_used)."""
        k1 = f(y)
        for _ in range(self.max_tries):
            h = self.dt
            y_full = self._heun(f, y, k1, h)
            y_mid = self._heun(f, y, k1, 0.5 * h)
            y_half = self._heun(f, y_mid, f(y_mid), 0.5 * h)
            delta = norm(y_full - y_half)
            factor = (self.tol / delta) ** (1.0 / 3.0) if delta > 0 else self.max_factor
            factor = min(self.max_factor, max(self.min_factor, factor))
            accept = delta <= self.tol or h <= self.dt_min
            self.dt = min(self.dt_max, max(self.dt_min, h * factor))
            if accept:
                return t + h, y_half, h
            self.n_rejected += 1
        raise RuntimeError("adaptive step size did not reach the tolerance")
