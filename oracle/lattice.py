"""Lattices and the on-the-fly connected configurations of the Hamiltonians.

Paper: Sec. 4.2 "Operators", the operator mapping s -> {s'_j}, {O_ss'_j}
(eq:operator_mapping) and its sigma^x worked example; the transverse-field
Ising Hamiltonian of Sec. 5.1 (1D) and Sec. 5.2 (2D).

Readings (the paper does not fix them):
  * site index i = y * Lx + x; a set bit is sigma = +1 (z = +1).
  * bond list: for each site in index order, the bond to +x, then (2D) the
    bond to +y; periodic wraps, open boundaries drop the wrapping bonds.
  * TFIM:       H = -J sum_<ij> Z_i Z_j - h sum_i X_i
  * Heisenberg: H =  J sum_<ij> (X_i X_j + Y_i Y_j + Z_i Z_j)  (Pauli matrices,
    no Marshall rotation).  Per bond, XX + YY maps an anti-aligned pair to the
    swapped pair with element 2J and annihilates an aligned pair.
  * slot order: slot 0 is the diagonal (kept even when its element is 0);
    then off-diagonal terms in term order (sites for X, bonds for the
    exchange); slots with a zero element are dropped and the survivors are
    packed to the front; padding slots repeat s with element 0.
  * diagonal element = coupling times the exact integer (n_aligned - n_anti),
    one float64 product.
"""
from __future__ import annotations

import numpy as np


def bonds(Lx: int, Ly: int, periodic: bool) -> list[tuple[int, int]]:
    """Nearest-neighbour bonds in the canonical order described above."""
    out = []
    for y in range(Ly):
        for x in range(Lx):
            i = y * Lx + x
            if x + 1 < Lx or (periodic and Lx > 1):
                out.append((i, y * Lx + (x + 1) % Lx))
            if Ly > 1 and (y + 1 < Ly or periodic):
                out.append((i, ((y + 1) % Ly) * Lx + x))
    return out


def max_connected(kind: str, Lx: int, Ly: int, periodic: bool) -> int:
    n = Lx * Ly
    return 1 + (n if kind == "tfim" else len(bonds(Lx, Ly, periodic)))


def connected(kind: str, s: np.ndarray, Lx: int, Ly: int, periodic: bool,
              J: float, h: float = 0.0):
    """Connected configurations of one 0/1 configuration ``s`` (length N).

    Returns (sp, mel, count): sp is (M_max, N) uint8, mel is (M_max,) float64,
    count the number of leading slots that carry a non-zero element (slot 0
    always counts).
    """
    s = np.asarray(s, dtype=np.uint8)
    N = Lx * Ly
    assert s.shape == (N,)
    bl = bonds(Lx, Ly, periodic)
    n_al = sum(1 for (i, j) in bl if s[i] == s[j])
    n_anti = len(bl) - n_al
    slots_sp = [s.copy()]
    if kind == "tfim":
        slots_mel = [-J * float(n_al - n_anti)]
        if h != 0.0:
            for l in range(N):
                sp = s.copy()
                sp[l] ^= 1
                slots_sp.append(sp)
                slots_mel.append(-h)
    elif kind == "heisenberg":
        slots_mel = [J * float(n_al - n_anti)]
        if J != 0.0:
            for (i, j) in bl:
                if s[i] != s[j]:
                    sp = s.copy()
                    sp[i], sp[j] = s[j], s[i]
                    slots_sp.append(sp)
                    slots_mel.append(2.0 * J)
    else:
        raise ValueError(kind)
    M = max_connected(kind, Lx, Ly, periodic)
    count = len(slots_mel)
    sp_out = np.repeat(s[None, :], M, axis=0)
    mel_out = np.zeros(M, dtype=np.float64)
    sp_out[:count] = np.stack(slots_sp)
    mel_out[:count] = slots_mel
    return sp_out, mel_out, count


def connected_batch(kind, S, Lx, Ly, periodic, J, h=0.0):
    """``connected`` applied to each row of the (B, N) array S."""
    res = [connected(kind, s, Lx, Ly, periodic, J, h) for s in np.asarray(S)]
    sp = np.stack([r[0] for r in res])
    mel = np.stack([r[1] for r in res])
    cnt = np.array([r[2] for r in res], dtype=np.int32)
    return sp, mel, cnt


def sparse_hamiltonian(kind, Lx, Ly, periodic, J, h=0.0, basis=None):
    """Sparse H over ``basis`` (list of integer states, bit i = site i) or over
    all 2^N states, assembled from ``connected``.  Used for exact
    diagonalisation in the pins."""
    import scipy.sparse as sp_

    N = Lx * Ly
    if basis is None:
        basis = np.arange(2 ** N, dtype=np.int64)
    basis = np.asarray(basis, dtype=np.int64)
    index = {int(b): k for k, b in enumerate(basis)}
    rows, cols, vals = [], [], []
    for k, b in enumerate(basis):
        s = ((int(b) >> np.arange(N)) & 1).astype(np.uint8)
        sp, mel, cnt = connected(kind, s, Lx, Ly, periodic, J, h)
        for m in range(cnt):
            if mel[m] == 0.0:
                continue
            code = int(np.sum(sp[m].astype(np.int64) << np.arange(N)))
            rows.append(k)
            cols.append(index[code])
            vals.append(mel[m])
    n = len(basis)
    return sp_.csr_matrix((vals, (rows, cols)), shape=(n, n))
