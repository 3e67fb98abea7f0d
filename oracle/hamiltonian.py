"""The Hubbard Hamiltonian of Eq. (1) in the sector basis, from its definition.

H = -sum_{bonds (i,j)} t_ij sum_s (c+_{i,s} c_{j,s} + c+_{j,s} c_{i,s})
    + U sum_i n_{i,up} n_{i,dn}

The interaction is diagonal: on an occupation state it counts the doubly
occupied sites (Sec. II.B).  Each kinetic term is applied with the explicit
operator algebra of oracle.fock; the index of every result is found by binary
search over the stored sorted key list (Sec. II.C).
"""
from dataclasses import dataclass
from math import comb
from typing import Sequence

import numpy as np
import scipy.sparse as sp

from .fock import sector_list, popcount, index_in_sorted, composite_keys, apply_hop_vec


@dataclass
class Problem:
    n_sites: int
    bond_i: Sequence[int]
    bond_j: Sequence[int]
    bond_t: Sequence[float]
    U: float
    n_up: int
    n_dn: int

    @staticmethod
    def from_workload(w) -> "Problem":
        return Problem(w.n_sites, [b.i for b in w.bonds], [b.j for b in w.bonds],
                       [b.t for b in w.bonds], float(w.U), w.n_up, w.n_dn)

    @property
    def up_list(self) -> np.ndarray:
        return sector_list(self.n_sites, self.n_up)

    @property
    def dn_list(self) -> np.ndarray:
        return sector_list(self.n_sites, self.n_dn)

    @property
    def D(self) -> int:
        return comb(self.n_sites, self.n_up) * comb(self.n_sites, self.n_dn)

    def terms(self):
        """Every kinetic term as (a, b, spin, amplitude) for amplitude * c+_a c_b."""
        for i, j, t in zip(self.bond_i, self.bond_j, self.bond_t):
            for spin in (0, 1):
                yield (i, j, spin, -float(t))
                yield (j, i, spin, -float(t))


def diag_values(p: Problem, phi_up: np.ndarray, phi_dn: np.ndarray) -> np.ndarray:
    """U times the number of doubly occupied sites."""
    return float(p.U) * popcount(np.asarray(phi_up, np.uint64) & np.asarray(phi_dn, np.uint64)).astype(np.float64)


def build_csr(p: Problem, with_diag: bool = True) -> sp.csr_matrix:
    """Explicit sparse H (column r holds H|r>), diagonal always stored.

    Feasible for D up to a few million.
    """
    N = p.n_sites
    up, dn = p.up_list, p.dn_list
    keys = composite_keys(up, dn, N)
    D = len(keys)
    PU = keys >> np.uint64(N)
    PD = keys & np.uint64((1 << N) - 1)
    cols_all = np.arange(D, dtype=np.int64)
    rows, cols, vals = [], [], []
    if with_diag:
        rows.append(cols_all)
        cols.append(cols_all)
        vals.append(diag_values(p, PU, PD))
    for a, b, spin, amp in p.terms():
        ok, sign, nu, nd = apply_hop_vec(PU, PD, spin, a, b)
        if not np.any(ok):
            continue
        newkey = (nu[ok] << np.uint64(N)) | nd[ok]
        rows.append(index_in_sorted(keys, newkey))
        cols.append(cols_all[ok])
        vals.append(amp * sign[ok])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    H = sp.coo_matrix((v, (r, c)), shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H


def hv_rows(p: Problem, x: np.ndarray, rows: np.ndarray, with_abs: bool = False):
    """(H x)[r] for the listed rows only, without building H.

    For each term amplitude * c+_a c_b, the source states r' that it sends
    onto |r> are those with c+_b c_a |r> != 0.  The matrix element
    <r| c+_a c_b |r'> is then evaluated by applying c+_a c_b to |r'> and
    reading its sign.  Indices come from binary search in the sector lists.
    with_abs: also return each row's sum of |terms| and its number of terms
    (the diagonal counts as one term), the scale of a rounding bound.
    """
    N = p.n_sites
    up, dn = p.up_list, p.dn_list
    Ddn = len(dn)
    rows = np.asarray(rows, dtype=np.int64)
    PU = up[rows // Ddn]
    PD = dn[rows % Ddn]
    y = diag_values(p, PU, PD) * x[rows]
    yabs = np.abs(y)
    nterm = np.ones(len(rows), dtype=np.int64)
    for a, b, spin, amp in p.terms():
        ok, _, su, sd = apply_hop_vec(PU, PD, spin, b, a)   # candidate sources
        if not np.any(ok):
            continue
        ok2, sign, tu, td = apply_hop_vec(su, sd, spin, a, b)  # c+_a c_b on the source
        ok &= ok2
        if not np.any(ok):
            continue
        assert np.all(tu[ok] == PU[ok]) and np.all(td[ok] == PD[ok])
        src = index_in_sorted(up, su[ok]) * Ddn + index_in_sorted(dn, sd[ok])
        contrib = np.zeros(len(rows))
        contrib[ok] = amp * sign[ok] * x[src]
        y += contrib
        yabs += np.abs(contrib)
        nterm += ok
    if with_abs:
        return y, yabs, nterm
    return y


def nnz_structural(p: Problem) -> int:
    """Structural nonzeros of H: D diagonal entries plus one per allowed hop."""
    N = p.n_sites
    total = p.D
    for spin, lst, other in ((0, p.up_list, p.dn_list), (1, p.dn_list, p.up_list)):
        zeros = np.zeros(len(lst), dtype=np.uint64)
        hops = 0
        for a, b, s, amp in p.terms():
            if s != spin:
                continue
            u, d = (lst, zeros) if spin == 0 else (zeros, lst)
            ok, _, _, _ = apply_hop_vec(u, d, spin, a, b)
            hops += int(np.count_nonzero(ok))
        total += hops * len(other)
    return total


def one_body_matrix(p: Problem) -> np.ndarray:
    """Single-particle hopping matrix h_ij = -t_ij (symmetric), for the U=0 limit."""
    h = np.zeros((p.n_sites, p.n_sites))
    for i, j, t in zip(p.bond_i, p.bond_j, p.bond_t):
        h[i, j] -= t
        h[j, i] -= t
    return h
