"""Pins of oracle.lattice: the paper's worked operator example, Kronecker-built
Hamiltonians, the Pfeuty closed form and exact diagonalisation."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import lattice, eloc
import kron_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_sigma_x_example():
    # Sec. 4.2 "Operators": sigma^x on site 1 of [0,0,0,0] -> [0,1,0,0], element 1.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "sigma_x_example.txt"))
            if l.strip() and not l.startswith("#")]
    for n, site, cin, cout, mel in rows:
        n, site, mel = int(n), int(site), float(mel)
        s = np.array([int(c) for c in cin], dtype=np.uint8)
        # sigma^x_site alone == the TFIM with J = 0 and h = -1, slot 1 + site
        sp, m, cnt = lattice.connected("tfim", s, n, 1, False, 0.0, -1.0)
        assert cnt == 1 + n
        assert "".join(map(str, sp[1 + site])) == cout
        assert m[1 + site] == mel


def test_bond_counts():
    assert len(lattice.bonds(10, 1, True)) == 10
    assert len(lattice.bonds(10, 1, False)) == 9
    assert len(lattice.bonds(10, 10, True)) == 200
    assert len(lattice.bonds(4, 3, False)) == 3 * 3 + 4 * 2
    assert lattice.max_connected("tfim", 16, 16, True) == 257
    assert lattice.max_connected("heisenberg", 10, 10, True) == 201
    # every site appears in exactly 2 * dim bonds on a periodic lattice
    deg = np.zeros(100, int)
    for i, j in lattice.bonds(10, 10, True):
        deg[i] += 1
        deg[j] += 1
    assert np.all(deg == 4)


def _codes(n):
    return np.arange(2 ** n, dtype=np.int64)


@pytest.mark.parametrize("kind,Lx,Ly,per,J,h", [
    ("tfim", 6, 1, True, 1.0, 0.7),
    ("tfim", 5, 1, False, -0.4, 1.3),
    ("tfim", 3, 3, True, 1.0, 3.0),
    ("heisenberg", 6, 1, True, 1.0, 0.0),
    ("heisenberg", 3, 3, True, 0.8, 0.0),
    ("heisenberg", 4, 2, False, 1.0, 0.0),
])
def test_elements_match_kronecker_hamiltonian(kind, Lx, Ly, per, J, h):
    n = Lx * Ly
    H_enum = lattice.sparse_hamiltonian(kind, Lx, Ly, per, J, h).toarray()
    Hk = (kron_ref.tfim(Lx, Ly, per, J, h) if kind == "tfim"
          else kron_ref.heisenberg(Lx, Ly, per, J)).toarray()
    perm = kron_ref.code_to_kron(_codes(n), n)
    Hk = Hk[np.ix_(perm, perm)]
    assert np.max(np.abs(Hk.imag)) == 0.0
    # the Kronecker sum accumulates bond terms one by one; the enumeration forms
    # coupling * integer in one product, so allow last-bit differences
    assert np.array_equal(H_enum != 0, Hk.real != 0)
    assert np.max(np.abs(H_enum - Hk.real)) <= 1e-13 * max(1.0, np.max(np.abs(Hk.real)))


def test_slot_order_and_padding():
    s = np.array([1, 0, 0, 1, 1, 0], dtype=np.uint8)
    sp, mel, cnt = lattice.connected("heisenberg", s, 6, 1, True, 1.0)
    bl = lattice.bonds(6, 1, True)
    anti = [b for b in bl if s[b[0]] != s[b[1]]]
    assert cnt == 1 + len(anti)
    assert mel[0] == 1.0 * (len(bl) - 2 * len(anti))
    for m, (i, j) in enumerate(anti, start=1):
        exp = s.copy()
        exp[i], exp[j] = s[j], s[i]
        assert np.array_equal(sp[m], exp) and mel[m] == 2.0
    assert np.all(mel[cnt:] == 0.0) and np.all(sp[cnt:] == s)
    # TFIM with h = 0 keeps only the diagonal slot
    sp, mel, cnt = lattice.connected("tfim", s, 6, 1, True, 1.0, 0.0)
    assert cnt == 1 and np.all(mel[1:] == 0.0)


@pytest.mark.parametrize("L,h", [(10, 1.0), (10, 0.7), (8, 2.0)])
def test_pfeuty_closed_form_matches_ed(L, h):
    H = lattice.sparse_hamiltonian("tfim", L, 1, True, 1.0, h)
    e0 = sla.eigsh(H, k=1, which="SA", tol=1e-12)[0][0]
    assert abs(e0 - kron_ref.pfeuty_e0(L, h)) < 1e-9
    if h == 1.0:
        assert abs(e0 - (-2.0 / np.sin(np.pi / (2 * L)))) < 1e-9


@pytest.mark.slow
def test_heisenberg_4x4_sz0_ground_energy_matches_kronecker():
    n = 16
    codes = np.array([c for c in range(2 ** n) if bin(c).count("1") == 8], dtype=np.int64)
    H = lattice.sparse_hamiltonian("heisenberg", 4, 4, True, 1.0, basis=codes)
    e_enum = sla.eigsh(H, k=1, which="SA", tol=1e-12)[0][0]
    Hk = kron_ref.heisenberg(4, 4, True, 1.0)
    idx = kron_ref.code_to_kron(codes, n)
    e_kron = sla.eigsh(Hk[idx][:, idx].real, k=1, which="SA", tol=1e-12)[0][0]
    assert abs(e_enum - e_kron) < 1e-8
