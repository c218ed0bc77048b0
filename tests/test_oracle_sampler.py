"""Pins of oracle.philox and oracle.metropolis: rocRAND's Philox4x32-10 (a
library routine compiled here for the host), detailed balance of the exact
transition matrix, Sz conservation and the oracle chain's histogram."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox, metropolis, rbm, eloc, lattice
import synth_inputs as si

ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seed, sub, off;
  while (scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine e(seed, sub, off * 4ULL);
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


@pytest.fixture(scope="module")
def rocrand_host():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "p.cpp")
    open(src, "w").write(ROCRAND_PROBE)
    exe = os.path.join(d, "p")
    r = subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot build the rocRAND host probe: " + r.stderr[-300:])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_host):
    rng = np.random.default_rng(0)
    cases = [(0, 0, 0), (2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 // 4 - 1)]
    cases += [(int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 2 ** 40)))
              for _ in range(200)]
    inp = "\n".join(f"{a} {b} {c}" for a, b, c in cases) + "\n"
    out = subprocess.run([rocrand_host], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([list(map(int, l.split())) for l in out.strip().splitlines()], dtype=np.uint64)
    ctr = np.array([[off & 0xFFFFFFFF, (off >> 32) & 0xFFFFFFFF, sub & 0xFFFFFFFF, sub >> 32]
                    for seed, sub, off in cases], dtype=np.uint64).astype(np.uint32)
    key = np.array([philox.seed_key(seed) for seed, _, _ in cases])
    mine = philox.philox4x32_10(ctr, key)
    assert np.array_equal(mine.astype(np.uint64), got)


def test_maps():
    assert philox.to_index(0, 10) == 0
    assert philox.to_index(0xFFFFFFFF, 10) == 9
    assert philox.to_uniform(0, 0) == 0.0
    assert philox.to_uniform(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    x = philox.philox4x32_10(np.stack([np.arange(20000), np.zeros(20000), np.zeros(20000), np.zeros(20000)], 1).astype(np.uint32),
                             philox.seed_key(7))
    u = philox.to_uniform(x[:, 1], x[:, 2])
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    counts = np.bincount(philox.to_index(x[:, 0], 10), minlength=10)
    assert stats.chisquare(counts).pvalue > 1e-4


@pytest.mark.parametrize("prop", ["flip", "exchange"])
def test_transition_matrix_stationary(prop):
    n = 8
    p = si.rbm_params(n, n, std=0.5, seed=2)
    f = lambda x: rbm.log_psi(p, x, n)
    bl = lattice.bonds(n, 1, True)
    states = None
    if prop == "exchange":
        states = np.array([s for s in eloc.all_states(n) if s.sum() == n // 2])
    P, states, lp = metropolis.transition_matrix(f, prop, n, bl, states)
    pi = np.exp(2 * (lp.real - lp.real.max()))
    pi /= pi.sum()
    assert np.all(P >= -1e-15) and np.allclose(P.sum(1), 1.0, atol=1e-14)
    assert np.max(np.abs(pi @ P - pi)) < 1e-14
    # detailed balance
    D = pi[:, None] * P
    assert np.max(np.abs(D - D.T)) < 1e-15


def test_exchange_conserves_sz_and_init_is_balanced():
    n = 16
    key = philox.seed_key(3)
    s0 = metropolis.initial_states(32, n, key, True)
    assert np.all(s0.sum(1) == n // 2)
    bl = lattice.bonds(4, 4, True)
    s = s0
    for t in range(50):
        s, _ = metropolis.propose("exchange", s, t, key, np.arange(32), bl)
        assert np.all(s.sum(1) == n // 2)


def test_oracle_chain_histogram_matches_born_distribution():
    n = 6
    p = si.rbm_params(n, n, std=0.6, seed=13)
    f = lambda x: rbm.log_psi(p, x, n)
    ch = metropolis.Chains(f, n, "flip", seed=101, chain_ids=np.arange(64), therm_sweeps=5)
    s, _ = ch.sample(200)
    codes = (s.reshape(-1, n).astype(np.int64) << np.arange(n)).sum(1)
    counts = np.bincount(codes, minlength=2 ** n)
    _, prob, _ = eloc.exact_probabilities(f, n)
    # sweeps are correlated; a 1e-4 threshold on this (slightly over-dispersed) test
    res = stats.chisquare(counts, prob * counts.sum())
    assert res.pvalue > 1e-4, res
