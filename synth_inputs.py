"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module holds no arithmetic of the variational Monte Carlo method: it only
draws parameters and spin configurations from seeded NumPy generators and
packs 0/1 spin arrays into the bit layout the library and the oracle both read.

Bit layout of a configuration of N spins: W = ceil(N / 64) little-endian
uint64 words; site i lives in word i // 64, bit i % 64; a set bit is spin up
(sigma = +1), a clear bit spin down (sigma = -1).  Bits at and above N in the
last word are zero.

Parameter draws follow the workload descriptions: "N(0, std)" means standard
deviation ``std``; complex parameters draw all real parts first, then all
imaginary parts, in the flat parameter order of the network.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "n_words", "pack_bits", "unpack_bits", "random_bits", "random_bits_sz0",
    "rbm_num_params", "rbm_params", "cnn_num_params", "cnn_params",
    "made_num_params", "made_params", "WORKLOADS",
]


def n_words(n_sites: int) -> int:
    return (n_sites + 63) // 64


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """(B, N) array of 0/1 -> (B, W) uint64 packed configurations."""
    bits = np.asarray(bits, dtype=np.uint64)
    if bits.ndim == 1:
        bits = bits[None, :]
    B, N = bits.shape
    W = n_words(N)
    out = np.zeros((B, W), dtype=np.uint64)
    for i in range(N):
        out[:, i // 64] |= bits[:, i] << np.uint64(i % 64)
    return out


def unpack_bits(words: np.ndarray, n_sites: int) -> np.ndarray:
    """(B, W) uint64 -> (B, N) uint8 array of 0/1."""
    words = np.asarray(words, dtype=np.uint64)
    if words.ndim == 1:
        words = words[None, :]
    out = np.zeros((words.shape[0], n_sites), dtype=np.uint8)
    for i in range(n_sites):
        out[:, i] = ((words[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)).astype(np.uint8)
    return out


def random_bits(batch: int, n_sites: int, seed: int) -> np.ndarray:
    """Uniformly random configurations, (B, N) uint8."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(batch, n_sites), dtype=np.uint8)


def random_bits_sz0(batch: int, n_sites: int, seed: int) -> np.ndarray:
    """Uniformly random configurations with exactly N/2 up spins, (B, N) uint8."""
    if n_sites % 2:
        raise ValueError("Sz=0 needs an even number of sites")
    rng = np.random.default_rng(seed)
    base = np.zeros(n_sites, dtype=np.uint8)
    base[: n_sites // 2] = 1
    return np.stack([rng.permutation(base) for _ in range(batch)])


def rbm_num_params(n_visible: int, n_hidden: int) -> int:
    return n_visible + n_hidden + n_visible * n_hidden


def _normal_params(K: int, std: float, is_complex: bool, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.normal(0.0, std, size=K)
    if not is_complex:
        return re.astype(np.float64)
    im = rng.normal(0.0, std, size=K)
    return (re + 1j * im).astype(np.complex128)


def rbm_params(n_visible: int, n_hidden: int, *, std: float = 0.01,
               is_complex: bool = True, seed: int = 0) -> np.ndarray:
    """Flat RBM parameters [a (N), b (N_h), W (N_h x N, row-major)]."""
    return _normal_params(rbm_num_params(n_visible, n_hidden), std, is_complex, seed)


def bond_rbm_params(Lx: int, Ly: int, w: float) -> np.ndarray:
    """RBM parameters with one hidden unit per nearest-neighbour bond of the
    periodic Lx x Ly lattice (bond order: per site, +x then +y): W[b, i] =
    W[b, j] = w for bond b = (i, j), all other parameters 0.  |psi|^2 is then
    the classical Ising weight prod_b exp(K s_i s_j) with K = ln cosh(2 w)."""
    N = Lx * Ly
    bl = []
    for y in range(Ly):
        for x in range(Lx):
            i = y * Lx + x
            bl.append((i, y * Lx + (x + 1) % Lx))
            bl.append((i, ((y + 1) % Ly) * Lx + x))
    Nh = len(bl)
    W = np.zeros((Nh, N), dtype=np.complex128)
    for b, (i, j) in enumerate(bl):
        W[b, i] = w
        W[b, j] = w
    return np.concatenate([np.zeros(N + Nh, dtype=np.complex128), W.ravel()])


# the coupling of bond_rbm_params that puts |psi|^2 at the critical point of the
# square-lattice Ising model: ln cosh(2 w) = K_c = ln(1 + sqrt 2) / 2
W_CRITICAL = 0.5 * np.arccosh(np.exp(0.5 * np.log(1.0 + np.sqrt(2.0))))


def cnn_num_params(channels: int, kernel: int) -> int:
    return channels * kernel * kernel + channels + channels * channels * kernel * kernel + channels


def cnn_params(channels: int, kernel: int, *, std: float = 0.05, seed: int = 0) -> np.ndarray:
    """Flat CNN parameters [W1 (C,1,k,k), b1 (C), W2 (C,C,k,k), b2 (C)], complex."""
    return _normal_params(cnn_num_params(channels, kernel), std, True, seed)


def made_num_params(n_in: int, n_hidden: int) -> int:
    return n_hidden * n_in + n_hidden + n_in * n_hidden + n_in


def ar_params(n_sites: int, n_hidden: int, *, seed: int, std: float = 0.5) -> np.ndarray:
    """Live parameters of the autoregressive state (N H + H + N reals), i.i.d.
    normal with standard deviation ``std``."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=n_sites * n_hidden + n_hidden + n_sites).astype(np.float64)


def symelu_params(L: int, alpha: int, *, seed: int, std: float = 0.1) -> np.ndarray:
    """Real parameters [W (alpha x L), b (alpha)] of the translation-symmetric ELU
    network, i.i.d. normal with standard deviation ``std``."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=alpha * (L + 1)).astype(np.float64)


def made_params(n_in: int, n_hidden: int, *, seed: int = 205) -> np.ndarray:
    """Flat MADE parameters [W1 (H x N), b1 (H), W2 (N x H), b2 (N)], float64,
    uniform in +-1/sqrt(fan_in) (a common dense-layer initialisation)."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(-1, 1, size=(n_hidden, n_in)) / np.sqrt(n_in)
    b1 = np.zeros(n_hidden)
    w2 = rng.uniform(-1, 1, size=(n_in, n_hidden)) / np.sqrt(n_hidden)
    b2 = np.zeros(n_in)
    return np.concatenate([w1.ravel(), b1, w2.ravel(), b2]).astype(np.float64)


# The workloads the library is built and measured for.  Sizes only; the
# arithmetic lives elsewhere.
WORKLOADS = {
    "tfim1d_L10_rbm_real": dict(
        ham="tfim", Lx=10, Ly=1, periodic=True, J=1.0, h=1.0,
        net="rbm", alpha=1, is_complex=False, std=0.01, param_seed=1,
        n_chains=16, samples_per_chain=64, sampler_seed=101, proposal="flip"),
    "heis2d_10x10_rbm_a4": dict(
        ham="heisenberg", Lx=10, Ly=10, periodic=True, J=1.0, h=0.0,
        net="rbm", alpha=4, is_complex=True, std=0.01, param_seed=2,
        n_chains=1024, samples_per_chain=8, sampler_seed=102, proposal="exchange"),
    "tfim1d_L64_rbm_a4_sr": dict(
        ham="tfim", Lx=64, Ly=1, periodic=True, J=1.0, h=1.0,
        net="rbm", alpha=4, is_complex=True, std=0.01, param_seed=3,
        n_chains=1024, samples_per_chain=16, sampler_seed=103, proposal="flip",
        nu_rel=1e-3),
    # SR at the learned-proposal lattice scale: K = 321 200 (no dense S)
    "tfim2d_20x20_rbm_a2_sr": dict(
        ham="tfim", Lx=20, Ly=20, periodic=True, J=1.0, h=3.0,
        net="rbm", alpha=2, is_complex=True, std=0.01, param_seed=6,
        n_chains=1024, samples_per_chain=4, sampler_seed=106, proposal="flip",
        nu_rel=1e-3),
    # SR step with an autoregressive state and direct sampling, at the scale of
    # the paper's SR-step benchmark (50-site periodic TFIM chain, about 1.5 k
    # parameters, 3e5 samples): 29 hidden units give 1 529 live parameters
    "tfim1d_L50_ar_sr": dict(
        ham="tfim", Lx=50, Ly=1, periodic=True, J=1.0, h=1.0,
        net="ar", hidden=29, std=0.1, param_seed=7,
        n_chains=1000, samples_per_chain=300, sampler_seed=107, proposal="direct",
        nu_rel=1e-3, eps_abs=1e-8),
    "tfim2d_16x16_cnn": dict(
        ham="tfim", Lx=16, Ly=16, periodic=True, J=1.0, h=3.0,
        net="cnn", channels=16, kernel=4, std=0.05, param_seed=4,
        n_chains=4096, samples_per_chain=8, sampler_seed=104, proposal="flip"),
    "tfim2d_20x20_rbm_a2_made": dict(
        ham="tfim", Lx=20, Ly=20, periodic=True, J=1.0, h=3.0,
        net="rbm", alpha=2, is_complex=True, param_seed=5,
        n_chains=4096, train_samples=65536, made_hidden=512, sampler_seed=105,
        made_seed=205, proposal="made_mix"),
}
