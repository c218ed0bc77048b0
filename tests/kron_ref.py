"""Hamiltonians built independently of the oracle's enumeration: sums of
Kronecker products of 2x2 Pauli matrices (scipy.sparse).  Used only as pins.

Basis convention of these matrices: the Kronecker factor of site 0 is the most
significant; local index 0 is Z = +1.  ``code_to_kron`` maps the library's
integer state code (bit i = site i, bit set = Z = +1) to the row index here.
"""
import numpy as np
import scipy.sparse as sp

X = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
Y = sp.csr_matrix(np.array([[0.0, -1j], [1j, 0.0]]))
Z = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, -1.0]]))
I2 = sp.identity(2, format="csr")


def site_op(ops: dict, n: int):
    m = None
    for i in range(n):
        f = ops.get(i, I2)
        m = f if m is None else sp.kron(m, f, format="csr")
    return m


def lattice_bonds(Lx, Ly, periodic):
    """Nearest-neighbour pairs as a set of unordered pairs (no ordering implied)."""
    out = []
    for y in range(Ly):
        for x in range(Lx):
            i = y * Lx + x
            if x + 1 < Lx or periodic:
                out.append((i, y * Lx + (x + 1) % Lx))
            if Ly > 1 and (y + 1 < Ly or periodic):
                out.append((i, ((y + 1) % Ly) * Lx + x))
    return out


def tfim(Lx, Ly, periodic, J, h):
    n = Lx * Ly
    H = sp.csr_matrix((2 ** n, 2 ** n))
    for (i, j) in lattice_bonds(Lx, Ly, periodic):
        H = H - J * site_op({i: Z, j: Z}, n)
    for i in range(n):
        H = H - h * site_op({i: X}, n)
    return H.tocsr()


def heisenberg(Lx, Ly, periodic, J):
    n = Lx * Ly
    H = sp.csr_matrix((2 ** n, 2 ** n), dtype=np.complex128)
    for (i, j) in lattice_bonds(Lx, Ly, periodic):
        for P in (X, Y, Z):
            H = H + J * site_op({i: P, j: P}, n)
    return H.tocsr()


def code_to_kron(codes, n):
    codes = np.asarray(codes, dtype=np.int64)
    out = np.zeros_like(codes)
    for i in range(n):
        bit = (codes >> i) & 1
        out |= (1 - bit) << (n - 1 - i)
    return out


def pfeuty_e0(L, h, J=1.0):
    """Ground-state energy of the periodic TFIM chain (Pfeuty 1970, even-parity
    sector with antiperiodic fermion momenta k = pi (2m + 1) / L)."""
    k = np.pi * (2 * np.arange(L) + 1) / L
    return -np.sum(np.sqrt(J * J + h * h - 2 * J * h * np.cos(k)))
