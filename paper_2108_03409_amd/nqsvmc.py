"""ctypes binding of libnqsvmc.so (include/nqsvmc.h), argument marshalling only.

Every step of the path runs in the library's HIP kernels; torch supplies device
memory (tensor.data_ptr()) and the HIP stream.  Importing this module does not
load the library; the first handle does, and raises if it is missing.

Configurations are passed as int64 tensors holding the packed uint64 words
(same bytes), complex buffers as complex128 / complex64 tensors.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnqsvmc.so")

VMC_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "NOT_PD", -5: "NONFINITE", -6: "UNSUPPORTED",
          -7: "WORKSPACE"}
VMC_F64, VMC_F32, VMC_BF16 = 0, 1, 2
DT_F64, DT_C128, DT_C64, DT_F32 = 0, 1, 2, 3
PROP_FLIP, PROP_EXCHANGE, PROP_MADE_MIX = 0, 1, 2
SR_COMPLEX, SR_REAL, SR_IMAG = 0, 1, 2

_lib = None


class VMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class SamplerOpts(C.Structure):
    _fields_ = [("proposal", C.c_int), ("n_chains", C.c_int), ("sweep_steps", C.c_int),
                ("therm_sweeps", C.c_int), ("global_steps", C.c_int), ("seed", C.c_uint64)]


class SROpts(C.Structure):
    _fields_ = [("nu_rel", C.c_double), ("eps_abs", C.c_double), ("mode", C.c_int),
                ("gamma_re", C.c_double), ("gamma_im", C.c_double), ("gram", C.c_int)]


class CGOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int)]


class EigOpts(C.Structure):
    _fields_ = [("eps_pinv", C.c_double), ("soft", C.c_int), ("eps_snr", C.c_double), ("tol", C.c_double),
                ("max_sweeps", C.c_int)]


class SRInfo(C.Structure):
    _fields_ = [("e_mean", C.c_double * 2), ("e_var", C.c_double), ("residual", C.c_double),
                ("min_pivot", C.c_double), ("fail_index", C.c_int64)]


P = C.c_void_p
I64 = C.c_int64
_SIGS = {
    "vmc_version": ([], C.c_char_p),
    "vmc_ctx_create": ([C.c_int, P, C.POINTER(P)], C.c_int),
    "vmc_ctx_destroy": ([P], C.c_int),
    "vmc_ctx_sync": ([P], C.c_int),
    "vmc_last_error": ([P], C.c_char_p),
    "vmc_ctx_set_workspace_limit": ([P, C.c_size_t], C.c_int),
    "vmc_ctx_set_timing": ([P, C.c_int], C.c_int),
    "vmc_ctx_get_timing": ([P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(I64)], C.c_int),
    "vmc_model_create_rbm": ([P, C.c_int, C.c_int, C.c_int, C.POINTER(P)], C.c_int),
    "vmc_model_create_cnn": ([P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(P)], C.c_int),
    "vmc_model_create_autoregressive": ([P, C.c_int, C.c_int, C.POINTER(P)], C.c_int),
    "vmc_model_create_table": ([P, C.c_int, P, C.POINTER(P)], C.c_int),
    "vmc_model_create_symelu": ([P, C.c_int, C.c_int, C.POINTER(P)], C.c_int),
    "vmc_model_num_params": ([P, C.POINTER(I64)], C.c_int),
    "vmc_model_num_sites": ([P, C.POINTER(C.c_int)], C.c_int),
    "vmc_model_set_params": ([P, P, C.c_int], C.c_int),
    "vmc_model_get_params": ([P, P, C.c_int], C.c_int),
    "vmc_model_set_precision": ([P, C.c_int], C.c_int),
    "vmc_model_destroy": ([P], C.c_int),
    "vmc_ham_create_tfim": ([P, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.POINTER(P)], C.c_int),
    "vmc_ham_create_heisenberg": ([P, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(P)], C.c_int),
    "vmc_ham_max_connected": ([P, C.POINTER(C.c_int)], C.c_int),
    "vmc_ham_num_bonds": ([P, C.POINTER(C.c_int)], C.c_int),
    "vmc_ham_connected": ([P, P, I64, P, P, P], C.c_int),
    "vmc_ham_destroy": ([P], C.c_int),
    "vmc_log_psi": ([P, P, I64, P], C.c_int),
    "vmc_local_energy": ([P, P, P, I64, P, P], C.c_int),
    "vmc_grad_log_psi": ([P, P, I64, P, C.c_int], C.c_int),
    "vmc_log_psi_vjp": ([P, P, I64, P, P], C.c_int),
    "vmc_log_psi_vjp_noalloc": ([P, P, I64, P, P], C.c_int),
    "vmc_sampler_create": ([P, P, P, C.POINTER(SamplerOpts), C.POINTER(P)], C.c_int),
    "vmc_sample": ([P, I64, P, P, C.POINTER(I64), C.POINTER(C.c_double)], C.c_int),
    "vmc_sampler_get_state": ([P, P, C.POINTER(C.c_size_t)], C.c_int),
    "vmc_sampler_set_state": ([P, P, C.c_size_t], C.c_int),
    "vmc_sampler_set_proposal_made": ([P, P], C.c_int),
    "vmc_sampler_get_stats": ([P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(I64)], C.c_int),
    "vmc_sampler_destroy": ([P], C.c_int),
    "vmc_sr_solve": ([P, P, C.c_int, P, P, I64, I64, C.POINTER(SROpts), P, C.POINTER(SRInfo)], C.c_int),
    "vmc_sr_fisher": ([P, P, C.c_int, P, P, I64, I64, C.POINTER(SROpts), P, P, C.POINTER(SRInfo)], C.c_int),
    "vmc_sr_solve_cg": ([P, P, C.c_int, P, P, I64, I64, C.POINTER(SROpts), C.POINTER(CGOpts), P, C.POINTER(SRInfo),
                         C.POINTER(C.c_int)], C.c_int),
    "vmc_sr_solve_eig": ([P, P, C.c_int, P, P, I64, I64, C.POINTER(SROpts), C.POINTER(EigOpts), P,
                          C.POINTER(SRInfo), P, P, C.POINTER(C.c_int)], C.c_int),
    "vmc_eigh": ([P, P, I64, C.c_double, C.c_int, P, P, C.POINTER(C.c_int)], C.c_int),
    "vmc_fisher_quad": ([P, P, C.c_int, P, I64, I64, P, C.POINTER(C.c_double)], C.c_int),
    "vmc_made_create": ([P, C.c_int, C.c_int, C.POINTER(P)], C.c_int),
    "vmc_made_num_params": ([P, C.POINTER(I64)], C.c_int),
    "vmc_made_set_params": ([P, P], C.c_int),
    "vmc_made_get_params": ([P, P], C.c_int),
    "vmc_made_log_q": ([P, P, I64, P], C.c_int),
    "vmc_made_nll_grad": ([P, P, I64, P, C.POINTER(C.c_double)], C.c_int),
    "vmc_made_train": ([P, P, I64, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double)], C.c_int),
    "vmc_made_sample": ([P, I64, C.c_uint64, C.c_uint64, P, P], C.c_int),
    "vmc_made_destroy": ([P], C.c_int),
    "vmc_calib_copy": ([P, P, P, I64], C.c_int),
    "vmc_calib_read": ([P, P, I64, P], C.c_int),
    "vmc_calib_mfma": ([P, C.c_int, C.c_int, C.c_int, P, C.POINTER(C.c_double)], C.c_int),
}
EXPORTS = tuple(_SIGS)


def load(path: str = LIB_PATH):
    """Loads the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnqsvmc.so not found at {path}; run __graft_entry__.build() first")
    lib = C.CDLL(path)
    for name, (args, res) in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc, ctx_ptr=None):
    if rc != VMC_OK:
        msg = load().vmc_last_error(ctx_ptr).decode()
        raise VMCError(rc, msg)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("buffers must be device tensors")
    if not t.is_contiguous():
        raise ValueError("buffers must be contiguous")
    return C.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0, stream=None):
        lib = load()
        self.device = device
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = P()
        _check(lib.vmc_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def sync(self):
        _check(load().vmc_ctx_sync(self.h), self.h)

    def set_workspace_limit(self, nbytes: int):
        _check(load().vmc_ctx_set_workspace_limit(self.h, nbytes), self.h)

    def set_timing(self, enable: bool):
        _check(load().vmc_ctx_set_timing(self.h, int(enable)), self.h)

    def get_timing(self, phase: str):
        """(total milliseconds, number of brackets) of a library phase."""
        ms = C.c_double()
        n = I64()
        _check(load().vmc_ctx_get_timing(self.h, phase.encode(), C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            load().vmc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        k = I64()
        _check(load().vmc_model_num_params(h, C.byref(k)), ctx.h)
        self.K = k.value
        n = C.c_int()
        _check(load().vmc_model_num_sites(h, C.byref(n)), ctx.h)
        self.N = n.value
        self.W = (self.N + 63) // 64

    @classmethod
    def rbm(cls, ctx, n_visible, n_hidden, is_complex=True):
        h = P()
        _check(load().vmc_model_create_rbm(ctx.h, n_visible, n_hidden, int(is_complex), C.byref(h)), ctx.h)
        return cls(ctx, h)

    @classmethod
    def cnn(cls, ctx, Lx, Ly, channels, kernel):
        h = P()
        _check(load().vmc_model_create_cnn(ctx.h, Lx, Ly, channels, kernel, C.byref(h)), ctx.h)
        return cls(ctx, h)

    @classmethod
    def symelu(cls, ctx, L, alpha):
        """Translation-symmetric ELU network on a ring (the paper's ground-state ansatz)."""
        h = P()
        _check(load().vmc_model_create_symelu(ctx.h, L, alpha, C.byref(h)), ctx.h)
        return cls(ctx, h)

    @classmethod
    def table(cls, ctx, n_sites, logpsi=None):
        """Tabulated log-amplitudes (2^n_sites complex128, device); test model."""
        h = P()
        lp = None if logpsi is None else logpsi.to(torch.complex128).contiguous()
        _check(load().vmc_model_create_table(ctx.h, n_sites, _ptr(lp), C.byref(h)), ctx.h)
        return cls(ctx, h)

    @classmethod
    def autoregressive(cls, ctx, n_sites, n_hidden):
        """psi = sqrt(q) of a masked autoregressive network; samplers on it draw
        independent samples directly (no Markov chain)."""
        h = P()
        _check(load().vmc_model_create_autoregressive(ctx.h, n_sites, n_hidden, C.byref(h)), ctx.h)
        return cls(ctx, h)

    def set_params(self, params: torch.Tensor):
        dt = {torch.complex128: DT_C128, torch.complex64: DT_C64, torch.float64: DT_F64}[params.dtype]
        assert params.numel() == self.K
        _check(load().vmc_model_set_params(self.h, _ptr(params), dt), self.ctx.h)

    def get_params(self, dtype=torch.complex128) -> torch.Tensor:
        out = torch.empty(self.K, dtype=dtype, device=f"cuda:{self.ctx.device}")
        _check(load().vmc_model_get_params(self.h, _ptr(out), DT_C128 if dtype == torch.complex128 else DT_C64),
               self.ctx.h)
        return out

    def set_precision(self, prec: int):
        _check(load().vmc_model_set_precision(self.h, prec), self.ctx.h)

    def log_psi(self, s: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        B = s.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.complex128, device=s.device)
        _check(load().vmc_log_psi(self.h, _ptr(s), B, _ptr(out)), self.ctx.h)
        return out

    def local_energy(self, H: "Hamiltonian", s: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        B = s.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.complex128, device=s.device)
        _check(load().vmc_local_energy(self.h, H.h, _ptr(s), B, None, _ptr(out)), self.ctx.h)
        return out

    def grad_log_psi(self, s: torch.Tensor, dtype=torch.complex128, out: torch.Tensor | None = None):
        B = s.shape[0]
        if out is None:
            out = torch.empty((B, self.K), dtype=dtype, device=s.device)
        dt = {torch.complex128: DT_C128, torch.complex64: DT_C64, torch.float64: DT_F64,
              torch.float32: DT_F32}[out.dtype]
        _check(load().vmc_grad_log_psi(self.h, _ptr(s), B, _ptr(out), dt), self.ctx.h)
        return out

    def log_psi_vjp(self, s: torch.Tensor, g: torch.Tensor) -> torch.Tensor:
        """sum_n g_n conj(O_nk) for a complex128 cotangent g of shape (B,)."""
        out = torch.empty(self.K, dtype=torch.complex128, device=s.device)
        g = g.to(torch.complex128).contiguous()
        _check(load().vmc_log_psi_vjp(self.h, _ptr(s), s.shape[0], _ptr(g), _ptr(out)), self.ctx.h)
        return out

    def log_psi_vjp_noalloc(self, s: torch.Tensor, g: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """log_psi_vjp into a caller-provided out (K complex128) without any
        allocation inside the library (fixed scratch; calls must not overlap)."""
        g = g.to(torch.complex128).contiguous()
        _check(load().vmc_log_psi_vjp_noalloc(self.h, _ptr(s), s.shape[0], _ptr(g), _ptr(out)), self.ctx.h)
        return out

    def close(self):
        if getattr(self, "h", None):
            load().vmc_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hamiltonian:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        m = C.c_int()
        _check(load().vmc_ham_max_connected(h, C.byref(m)), ctx.h)
        self.M_max = m.value
        nb = C.c_int()
        _check(load().vmc_ham_num_bonds(h, C.byref(nb)), ctx.h)
        self.n_bonds = nb.value

    @classmethod
    def tfim(cls, ctx, Lx, Ly, periodic, J, h):
        hh = P()
        _check(load().vmc_ham_create_tfim(ctx.h, Lx, Ly, int(periodic), J, h, C.byref(hh)), ctx.h)
        return cls(ctx, hh)

    @classmethod
    def heisenberg(cls, ctx, Lx, Ly, periodic, J):
        hh = P()
        _check(load().vmc_ham_create_heisenberg(ctx.h, Lx, Ly, int(periodic), J, C.byref(hh)), ctx.h)
        return cls(ctx, hh)

    def connected(self, s: torch.Tensor):
        B, W = s.shape
        sp = torch.empty((B, self.M_max, W), dtype=torch.int64, device=s.device)
        mel = torch.empty((B, self.M_max), dtype=torch.float64, device=s.device)
        cnt = torch.empty(B, dtype=torch.int32, device=s.device)
        _check(load().vmc_ham_connected(self.h, _ptr(s), B, _ptr(sp), _ptr(mel), _ptr(cnt)), self.ctx.h)
        return sp, mel, cnt

    def close(self):
        if getattr(self, "h", None):
            load().vmc_ham_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sampler:
    def __init__(self, ctx: Context, model: Model, ham: Hamiltonian, *, proposal=PROP_FLIP, n_chains=16,
                 sweep_steps=0, therm_sweeps=20, global_steps=0, seed=0):
        self.ctx, self.model, self.ham = ctx, model, ham
        self.opts = SamplerOpts(proposal, n_chains, sweep_steps, therm_sweeps, global_steps, seed)
        h = P()
        _check(load().vmc_sampler_create(ctx.h, model.h, ham.h, C.byref(self.opts), C.byref(h)), ctx.h)
        self.h = h
        self.n_chains = n_chains

    def sample(self, n_samples: int):
        per = -(-n_samples // self.n_chains)
        n = per * self.n_chains
        dev = f"cuda:{self.ctx.device}"
        s = torch.empty((n, self.model.W), dtype=torch.int64, device=dev)
        lp = torch.empty(n, dtype=torch.complex128, device=dev)
        nw = I64()
        acc = C.c_double()
        _check(load().vmc_sample(self.h, n_samples, _ptr(s), _ptr(lp), C.byref(nw), C.byref(acc)), self.ctx.h)
        assert nw.value == n
        return s, lp, acc.value

    def set_proposal_made(self, made: "MADE"):
        _check(load().vmc_sampler_set_proposal_made(self.h, made.h), self.ctx.h)

    def stats(self):
        """(acceptance, global acceptance, number of global proposals) of the last sample call."""
        a, g, n = C.c_double(), C.c_double(), I64()
        _check(load().vmc_sampler_get_stats(self.h, C.byref(a), C.byref(g), C.byref(n)), self.ctx.h)
        return a.value, g.value, n.value

    def get_state(self) -> bytes:
        n = C.c_size_t(0)
        _check(load().vmc_sampler_get_state(self.h, None, C.byref(n)), self.ctx.h)
        buf = C.create_string_buffer(n.value)
        _check(load().vmc_sampler_get_state(self.h, buf, C.byref(n)), self.ctx.h)
        return buf.raw[: n.value]

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(load().vmc_sampler_set_state(self.h, buf, len(blob)), self.ctx.h)

    def close(self):
        if getattr(self, "h", None):
            load().vmc_sampler_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MADE:
    """Masked autoregressive proposal network (float64 parameters on the device)."""

    def __init__(self, ctx: Context, n_in: int, n_hidden: int):
        self.ctx, self.N, self.H = ctx, n_in, n_hidden
        self.W = (n_in + 63) // 64
        h = P()
        _check(load().vmc_made_create(ctx.h, n_in, n_hidden, C.byref(h)), ctx.h)
        self.h = h
        k = I64()
        _check(load().vmc_made_num_params(h, C.byref(k)), ctx.h)
        self.P = k.value

    def set_params(self, p: torch.Tensor):
        assert p.dtype == torch.float64 and p.numel() == self.P
        _check(load().vmc_made_set_params(self.h, _ptr(p)), self.ctx.h)

    def get_params(self) -> torch.Tensor:
        out = torch.empty(self.P, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        _check(load().vmc_made_get_params(self.h, _ptr(out)), self.ctx.h)
        return out

    def log_q(self, s: torch.Tensor) -> torch.Tensor:
        out = torch.empty(s.shape[0], dtype=torch.float64, device=s.device)
        _check(load().vmc_made_log_q(self.h, _ptr(s), s.shape[0], _ptr(out)), self.ctx.h)
        return out

    def nll_grad(self, s: torch.Tensor):
        g = torch.empty(self.P, dtype=torch.float64, device=s.device)
        nll = C.c_double()
        _check(load().vmc_made_nll_grad(self.h, _ptr(s), s.shape[0], _ptr(g), C.byref(nll)), self.ctx.h)
        return nll.value, g

    def train(self, s: torch.Tensor, epochs: int, batch: int, lr: float) -> float:
        nll = C.c_double()
        _check(load().vmc_made_train(self.h, _ptr(s), s.shape[0], epochs, batch, lr, C.byref(nll)), self.ctx.h)
        return nll.value

    def sample(self, B: int, seed: int, counter: int = 0):
        dev = f"cuda:{self.ctx.device}"
        s = torch.empty((B, self.W), dtype=torch.int64, device=dev)
        lq = torch.empty(B, dtype=torch.float64, device=dev)
        _check(load().vmc_made_sample(self.h, B, seed, counter, _ptr(s), _ptr(lq)), self.ctx.h)
        return s, lq

    def close(self):
        if getattr(self, "h", None):
            load().vmc_made_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sr_solve(ctx: Context, O: torch.Tensor, eloc: torch.Tensor, *, weights=None, nu_rel=1e-3, eps_abs=0.0,
             mode=SR_COMPLEX, gamma=1.0, gram=0, raise_on_error=True):
    """Returns (x, info dict).  O: (N, K) complex64/complex128, or float32/float64
    for real log-derivatives; eloc: (N,) complex128."""
    N, K = O.shape
    dt = {torch.complex128: DT_C128, torch.complex64: DT_C64, torch.float64: DT_F64, torch.float32: DT_F32}[O.dtype]
    x = torch.empty(K, dtype=torch.complex128, device=O.device)
    g = complex(gamma)
    opts = SROpts(nu_rel, eps_abs, mode, g.real, g.imag, gram)
    info = SRInfo()
    rc = load().vmc_sr_solve(ctx.h, _ptr(O), dt, _ptr(eloc), _ptr(weights), N, K, C.byref(opts), _ptr(x),
                             C.byref(info))
    d = dict(e_mean=complex(info.e_mean[0], info.e_mean[1]), e_var=info.e_var, residual=info.residual,
             min_pivot=info.min_pivot, fail_index=info.fail_index, status=ERRORS.get(rc, "OK") if rc else "OK")
    if rc != VMC_OK and raise_on_error:
        _check(rc, ctx.h)
    return (x if rc == VMC_OK else None), d


def sr_fisher(ctx: Context, O: torch.Tensor, eloc: torch.Tensor, *, weights=None, nu_rel=0.0, eps_abs=0.0,
              mode=SR_COMPLEX, gram=0):
    """Test export: (S~ (K, K) complex128, F (K,) complex128, info) exactly as
    sr_solve forms them (for SR_IMAG the matrix is i Im S)."""
    N, K = O.shape
    dt = {torch.complex128: DT_C128, torch.complex64: DT_C64, torch.float64: DT_F64, torch.float32: DT_F32}[O.dtype]
    S = torch.empty((K, K), dtype=torch.complex128, device=O.device)
    F = torch.empty(K, dtype=torch.complex128, device=O.device)
    opts = SROpts(nu_rel, eps_abs, mode, 1.0, 0.0, gram)
    info = SRInfo()
    _check(load().vmc_sr_fisher(ctx.h, _ptr(O), dt, _ptr(eloc), _ptr(weights), N, K, C.byref(opts), _ptr(S), _ptr(F),
                                C.byref(info)), ctx.h)
    return S, F, dict(e_mean=complex(info.e_mean[0], info.e_mean[1]), e_var=info.e_var)


def sr_solve_cg(ctx: Context, O: torch.Tensor, eloc: torch.Tensor, *, weights=None, nu_rel=1e-3, eps_abs=0.0,
                mode=SR_COMPLEX, gamma=1.0, tol=1e-10, max_iter=1000, raise_on_error=True):
    """The shifted SR system by preconditioned conjugate gradient (S never
    formed).  Returns (x, info dict with 'iterations')."""
    N, K = O.shape
    dt = DT_C128 if O.dtype == torch.complex128 else DT_C64
    x = torch.empty(K, dtype=torch.complex128, device=O.device)
    g = complex(gamma)
    opts = SROpts(nu_rel, eps_abs, mode, g.real, g.imag, 0)
    cg = CGOpts(tol, max_iter)
    info = SRInfo()
    it = C.c_int()
    rc = load().vmc_sr_solve_cg(ctx.h, _ptr(O), dt, _ptr(eloc), _ptr(weights), N, K, C.byref(opts), C.byref(cg),
                                _ptr(x), C.byref(info), C.byref(it))
    d = dict(e_mean=complex(info.e_mean[0], info.e_mean[1]), e_var=info.e_var, residual=info.residual,
             iterations=it.value, status=ERRORS.get(rc, "OK") if rc else "OK")
    if rc != VMC_OK and raise_on_error:
        _check(rc, ctx.h)
    return (x if rc == VMC_OK else None), d


def sr_solve_eig(ctx: Context, O: torch.Tensor, eloc: torch.Tensor, *, weights=None, nu_rel=0.0, eps_abs=0.0,
                 mode=SR_COMPLEX, gamma=1.0, gram=0, eps_pinv=0.0, soft=False, eps_snr=0.0, want_snr=False,
                 tol=0.0, max_sweeps=0, raise_on_error=True):
    """The TDVP / SR equation regularised through the eigendecomposition of S~
    (pseudo-inverse cutoffs, signal-to-noise filter).  Returns (x, info) with
    info['evals'] (device, unordered), info['snr'] (device or None), info['sweeps']."""
    N, K = O.shape
    dt = {torch.complex128: DT_C128, torch.complex64: DT_C64, torch.float64: DT_F64, torch.float32: DT_F32}[O.dtype]
    dev = O.device
    x = torch.empty(K, dtype=torch.complex128, device=dev)
    ev = torch.empty(K, dtype=torch.float64, device=dev)
    snr = torch.empty(K, dtype=torch.float64, device=dev) if (want_snr or eps_snr > 0) else None
    g = complex(gamma)
    opts = SROpts(nu_rel, eps_abs, mode, g.real, g.imag, gram)
    eo = EigOpts(eps_pinv, int(bool(soft)), eps_snr, tol, max_sweeps)
    info = SRInfo()
    sw = C.c_int()
    rc = load().vmc_sr_solve_eig(ctx.h, _ptr(O), dt, _ptr(eloc), _ptr(weights), N, K, C.byref(opts), C.byref(eo),
                                 _ptr(x), C.byref(info), _ptr(ev), _ptr(snr), C.byref(sw))
    d = dict(e_mean=complex(info.e_mean[0], info.e_mean[1]), e_var=info.e_var, residual=info.residual,
             min_eval=info.min_pivot, evals=ev, snr=snr, sweeps=sw.value, status=ERRORS.get(rc, "OK") if rc else "OK")
    if rc != VMC_OK and raise_on_error:
        _check(rc, ctx.h)
    return (x if rc == VMC_OK else None), d


def fisher_quad(ctx: Context, O: torch.Tensor, v: torch.Tensor, weights=None) -> float:
    """v^dagger S v with S the connected covariance of the rows of O (weights normalised)."""
    N, K = O.shape
    dt = {torch.complex128: DT_C128, torch.complex64: DT_C64, torch.float64: DT_F64, torch.float32: DT_F32}[O.dtype]
    v = v.to(torch.complex128).contiguous()
    out = C.c_double()
    _check(load().vmc_fisher_quad(ctx.h, _ptr(O), dt, _ptr(weights), N, K, _ptr(v), C.byref(out)), ctx.h)
    return out.value


def eigh(ctx: Context, A: torch.Tensor, *, tol=0.0, max_sweeps=0):
    """Hermitian eigendecomposition on the device: (evals (K,) float64 unordered,
    V (K, K) complex128 with eigenvectors as columns, sweeps)."""
    K = A.shape[0]
    A = A.to(torch.complex128).contiguous()
    ev = torch.empty(K, dtype=torch.float64, device=A.device)
    V = torch.empty((K, K), dtype=torch.complex128, device=A.device)
    sw = C.c_int()
    _check(load().vmc_eigh(ctx.h, _ptr(A), K, tol, max_sweeps, _ptr(ev), _ptr(V), C.byref(sw)), ctx.h)
    return ev, V, sw.value


class NQSLogPsi(torch.autograd.Function):
    """log psi_theta(s) as a differentiable function of the complex parameter
    vector theta: forward runs the library's network kernels, backward its
    vector-Jacobian kernels (grad_theta = sum_n grad_out_n conj(O_n), torch's
    convention for holomorphic functions).  The model's parameters are set to
    theta on every call."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, s: torch.Tensor, model: "Model"):
        model.set_params(theta.detach().to(torch.complex128).contiguous())
        ctx.model = model
        ctx.save_for_backward(theta, s)
        return model.log_psi(s)

    @staticmethod
    def backward(ctx, grad_out):
        theta, s = ctx.saved_tensors
        model = ctx.model
        model.set_params(theta.detach().to(torch.complex128).contiguous())
        g = model.log_psi_vjp(s, grad_out)
        return g.to(theta.dtype), None, None


def log_psi_autograd(model: "Model", theta: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    return NQSLogPsi.apply(theta, s, model)


def version() -> str:
    return load().vmc_version().decode()


def calib_copy(ctx: Context, src: torch.Tensor, dst: torch.Tensor):
    """Device copy of src into dst (same byte size): the HBM bandwidth reference."""
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nb
    _check(load().vmc_calib_copy(ctx.h, _ptr(src), _ptr(dst), nb), ctx.h)


def calib_read(ctx: Context, src: torch.Tensor):
    """Read-only pass over src: the read bandwidth reference."""
    nb = src.numel() * src.element_size()
    out = torch.empty(8192 * 2, dtype=torch.int64, device=src.device)
    _check(load().vmc_calib_read(ctx.h, _ptr(src), nb, _ptr(out)), ctx.h)


CALIB_BF16 = 16
CALIB_KINDS = {"f64": DT_F64, "f32": DT_F32, "bf16": CALIB_BF16}


def calib_mfma(ctx: Context, kind: str, n_groups: int, iters: int) -> float:
    """Runs the matrix-core loop of one type; returns the flops issued."""
    dt = torch.float64 if kind == "f64" else torch.float32
    out = torch.empty(n_groups * 256, dtype=dt, device=f"cuda:{ctx.device}")
    fl = C.c_double()
    _check(load().vmc_calib_mfma(ctx.h, CALIB_KINDS[kind], n_groups, iters, _ptr(out), C.byref(fl)), ctx.h)
    return fl.value

