"""Eq. (1) on the tensor-product basis, for full-size reference energies.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): used by tests/ and by the
scripts under tests/golden/ that write stored expected values.

The basis is the tensor product of the two spin sectors (Sec. II.A) and a
vector of length D is the matrix X[idx_up, idx_dn] (composite index of
Sec. III).  Every kinetic term of Eq. (1) changes only the string of its own
spin, so H acts as

    (H x)[u, d] = sum_u' Tup[u, u'] X[u', d] + sum_d' Tdn[d, d'] X[u, d'] + V[u, d] X[u, d],

with V[u, d] = U popcount(phi_up(u) & phi_dn(d)) the interaction (Sec. II.B).

Tsigma is assembled term by term with the operator algebra of oracle.fock
applied to full basis states (phi_up, phi_dn): the string of the other spin
is held at a fixed partner string that the caller may choose, and target
indices come from binary search over the sorted sector list (Sec. II.C).
That the partner string does not change Tsigma is not assumed here: tests
build Tsigma with different partners and compare this product element by
element with the element-wise oracle (hamiltonian.build_csr, cmf.MatrixFree).

The products are sparse-times-dense library calls on row blocks run in a
thread pool; nothing else is restructured.
"""
from concurrent.futures import ThreadPoolExecutor
import os

import numpy as np
import scipy.sparse as sp

from .fock import apply_hop_vec, index_in_sorted, popcount


def spin_matrix(p, spin: int, partner: int = None) -> sp.csr_matrix:
    """Tsigma[target, source] = sum of amp * sign over the terms of `spin` (CSR, float64).

    partner: the other spin's string held fixed while the terms act (default:
    the first string of the other sector).
    """
    lst = p.up_list if spin == 0 else p.dn_list
    other = p.dn_list if spin == 0 else p.up_list
    if partner is None:
        partner = int(other[0]) if len(other) else 0
    part = np.full(len(lst), partner, dtype=np.uint64)
    src = np.arange(len(lst), dtype=np.int64)
    rows, cols, vals = [], [], []
    for a, b, s, amp in p.terms():
        if s != spin:
            continue
        u, d = (lst, part) if spin == 0 else (part, lst)
        ok, sign, nu, nd = apply_hop_vec(u, d, spin, a, b)      # amp * c+_a c_b on every source
        if not np.any(ok):
            continue
        new = nu if spin == 0 else nd
        keep = nd if spin == 0 else nu
        assert np.all(keep[ok] == np.uint64(partner))
        rows.append(index_in_sorted(lst, new[ok]))
        cols.append(src[ok])
        vals.append(amp * sign[ok])
    n = len(lst)
    if not rows:
        return sp.csr_matrix((n, n))
    T = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    T.sum_duplicates()
    return T


class KronH:
    """H x for one problem through the per-spin matrices (FP64)."""

    def __init__(self, p, nthreads: int = 0, partners=(None, None)):
        self.p = p
        self.up = p.up_list
        self.dn = p.dn_list
        self.Du, self.Dd = len(self.up), len(self.dn)
        self.D = self.Du * self.Dd
        self.Tup = spin_matrix(p, 0, partners[0])
        self.TdnT = spin_matrix(p, 1, partners[1]).T.tocsr()
        self.nthreads = nthreads or (os.cpu_count() or 1)

    def interaction_rows(self, u0: int, u1: int) -> np.ndarray:
        """V[u, d] for rows u0 <= u < u1."""
        return float(self.p.U) * popcount(self.up[u0:u1, None] & self.dn[None, :]).astype(np.float64)

    def rows(self, X: np.ndarray, u0: int, u1: int) -> np.ndarray:
        """(H x)[u, :] for u0 <= u < u1, X the (Du, Dd) view of x."""
        out = self.Tup[u0:u1] @ X
        out += X[u0:u1] @ self.TdnT
        out += self.interaction_rows(u0, u1) * X[u0:u1]
        return out

    def __call__(self, x: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(x, dtype=np.float64).reshape(self.Du, self.Dd)
        Y = np.empty_like(X)
        nb = max(1, min(self.Du, 4 * self.nthreads))
        cuts = [self.Du * i // nb for i in range(nb + 1)]

        def work(i):
            Y[cuts[i]:cuts[i + 1]] = self.rows(X, cuts[i], cuts[i + 1])

        with ThreadPoolExecutor(self.nthreads) as ex:
            list(ex.map(work, range(nb)))
        return Y.reshape(-1)
