"""Translation-symmetric Hubbard sectors in momentum space, from their definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. IV.A: on an L1 x L2 periodic cluster the Fourier transformed operators
c_k turn Eq. (1) into Eq. (4),
    H = sum_{k,s} eps_k n_{k,s} + (U/N) sum_{k,k',q} c+_{k+q,up} c+_{k'-q,dn} c_{k',dn} c_{k,up},
whose terms keep the total momentum K of a basis state, so each K is a sector.

* Orbital i is the momentum k_i = (2 pi/L1 * (i mod L1), 2 pi/L2 * (i div L1));
  momenta add component-wise modulo the Brillouin zone.  A momentum is named
  by its orbital index.
* A basis element is an (up string, down string) pair of orbital occupations
  whose momenta sum to K.  The sector lists every such pair ordered by the
  up string, then the down string, as integers -- the order the spin-full
  forward map of Sec. IV.A produces (its up part counts, for each set up bit,
  the states with a smaller up string; its down part ranks the down string
  among the down strings of the remaining momentum).  Index lookup is binary
  search in that stored list (Sec. II.C), not the perfect hash.
* Eq. (4) is applied term by term with the operator algebra of oracle.fock
  (normal-ordered strings, up operators left of down operators, orbital index
  growing right to left), every sign counted.
* eps_k is the Fourier transform of the bond list's hopping:
  eps_k = -(1/N) sum_bonds t_b 2 cos(k . (r_j - r_i)), which for the square
  lattice with t and t' is the band of Sec. IV.A (pinned in the tests).

forward_map_k / forward_map_k_spin / extended_counts are the paper's k-space
mapping written out in its own steps, kept here only so that the CPU tests can
check the reading of Eqs. (5)-(7) against the sorted list; nothing else in the
oracle uses them.
"""
from itertools import combinations
from math import comb

import numpy as np
import scipy.sparse as sp

from .fock import annihilate_sign, create_sign


def momentum(i, L1, L2):
    """Components (a, b) of orbital i's momentum, in units of (2 pi/L1, 2 pi/L2)."""
    return i % L1, i // L1


def k_add(a, b, L1, L2):
    a1, a2 = momentum(a, L1, L2)
    b1, b2 = momentum(b, L1, L2)
    return (a1 + b1) % L1 + L1 * ((a2 + b2) % L2)


def k_neg(a, L1, L2):
    a1, a2 = momentum(a, L1, L2)
    return (-a1) % L1 + L1 * ((-a2) % L2)


def k_sub(a, b, L1, L2):
    return k_add(a, k_neg(b, L1, L2), L1, L2)


def string_momentum(phi, L1, L2):
    """Total momentum (orbital index) of one occupation string."""
    k = 0
    phi = int(phi)
    for i in range(L1 * L2):
        if (phi >> i) & 1:
            k = k_add(k, i, L1, L2)
    return k


def band_from_bonds(L1, L2, bonds, tol=1e-12):
    """eps_k for every orbital k, the Fourier transform of a translation-invariant bond list.

    bonds: (i, j, t) with sites numbered s = x + L1*y.  Raises if the bond list
    is not invariant under the lattice translations (momentum would not be a
    good quantum number).
    """
    N = L1 * L2
    canon = {}
    for i, j, t in bonds:
        key = (min(i, j), max(i, j))
        canon[key] = canon.get(key, 0.0) + float(t)

    def shift(s, dx, dy):
        return (s % L1 + dx) % L1 + L1 * ((s // L1 + dy) % L2)

    for (i, j), t in canon.items():
        for dx, dy in ((1, 0), (0, 1)):
            a, b = shift(i, dx, dy), shift(j, dx, dy)
            if abs(canon.get((min(a, b), max(a, b)), 0.0) - t) > tol:
                raise ValueError("bond list is not translation invariant")
    eps = np.zeros(N)
    for k in range(N):
        k1, k2 = momentum(k, L1, L2)
        for i, j, t in bonds:
            dx = (j % L1) - (i % L1)
            dy = (j // L1) - (i // L1)
            eps[k] -= 2.0 * float(t) * np.cos(2 * np.pi * (k1 * dx / L1 + k2 * dy / L2)) / N
    return eps


def square_band(L1, L2, t, tp):
    """eps_k = -2t(cos kx + cos ky) - 4t' cos kx cos ky (the band quoted in Sec. IV.A)."""
    out = np.zeros(L1 * L2)
    for k in range(L1 * L2):
        k1, k2 = momentum(k, L1, L2)
        kx, ky = 2 * np.pi * k1 / L1, 2 * np.pi * k2 / L2
        out[k] = -2 * t * (np.cos(kx) + np.cos(ky)) - 4 * tp * np.cos(kx) * np.cos(ky)
    return out


def strings_by_momentum(L1, L2, n):
    """For each total momentum, the ascending list of n-electron strings carrying it."""
    N = L1 * L2
    out = [[] for _ in range(N)]
    for c in combinations(range(N), n):
        phi = sum(1 << p for p in c)
        out[string_momentum(phi, L1, L2)].append(phi)
    return [np.array(sorted(v), dtype=np.uint64) for v in out]


def sector_keys(L1, L2, n_up, n_dn, K):
    """Sorted keys (phi_up << N) | phi_dn of every basis element of total momentum K."""
    N = L1 * L2
    ups = strings_by_momentum(L1, L2, n_up)
    dns = strings_by_momentum(L1, L2, n_dn)
    parts = []
    all_up = sorted((int(u), k) for k in range(N) for u in ups[k])
    for u, ku in all_up:
        d = dns[k_sub(K, ku, L1, L2)]
        if len(d):
            parts.append((np.uint64(u) << np.uint64(N)) | d)
    keys = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)
    assert np.all(keys[1:] > keys[:-1])
    return keys


def split_keys(keys, N):
    return keys >> np.uint64(N), keys & np.uint64((1 << N) - 1)


def index_of(keys, up, dn, N):
    """Positions of (up, dn) pairs in the sorted key list; -1 where absent."""
    k = (np.asarray(up, np.uint64) << np.uint64(N)) | np.asarray(dn, np.uint64)
    pos = np.searchsorted(keys, k)
    pos = np.minimum(pos, max(len(keys) - 1, 0))
    hit = (len(keys) > 0) & (keys[pos] == k) if len(keys) else np.zeros(len(k), bool)
    return np.where(hit, pos, -1).astype(np.int64)


def _op(up, dn, spin, orb, create):
    """c+_{orb,spin} (create) or c_{orb,spin} on arrays of strings: (ok, parity, up', dn')."""
    s = up if spin == 0 else dn
    bit = np.uint64(1 << orb)
    if create:
        ok = (s & bit) == 0
        cnt = create_sign(up, dn, spin, orb)
        s2 = s | bit
    else:
        ok = (s & bit) != 0
        cnt = annihilate_sign(up, dn, spin, orb)
        s2 = s & ~bit
    return (ok, cnt, s2, dn) if spin == 0 else (ok, cnt, up, s2)


def apply_terms(L1, L2, eps, U, up, dn):
    """Every term of Eq. (4) on the basis states (up, dn): yields (coef, ok, up', dn').

    coef already carries the operator sign; entries with ok False vanish.
    """
    N = L1 * L2
    up = np.asarray(up, np.uint64)
    dn = np.asarray(dn, np.uint64)
    for k in range(N):
        for spin in (0, 1):
            ok, c1, u, d = _op(up, dn, spin, k, create=False)
            ok2, c2, u, d = _op(u, d, spin, k, create=True)
            ok &= ok2
            yield eps[k] * np.where((c1 + c2) % 2 == 1, -1.0, 1.0), ok, u, d
    for k in range(N):
        for kp in range(N):
            for q in range(N):
                ok, c, u, d = _op(up, dn, 0, k, create=False)                          # c_{k,up}
                o, cc, u, d = _op(u, d, 1, kp, create=False); ok &= o; c = c + cc      # c_{k',dn}
                o, cc, u, d = _op(u, d, 1, k_sub(kp, q, L1, L2), create=True); ok &= o; c = c + cc
                o, cc, u, d = _op(u, d, 0, k_add(k, q, L1, L2), create=True); ok &= o; c = c + cc
                yield (U / N) * np.where(c % 2 == 1, -1.0, 1.0), ok, u, d


def build_csr_k(L1, L2, eps, U, n_up, n_dn, K):
    """Explicit sparse H_K (column r holds H|r>), the diagonal always stored."""
    N = L1 * L2
    keys = sector_keys(L1, L2, n_up, n_dn, K)
    D = len(keys)
    up, dn = split_keys(keys, N)
    cols_all = np.arange(D, dtype=np.int64)
    rows, cols, vals = [cols_all], [cols_all], [np.zeros(D)]
    for coef, ok, u, d in apply_terms(L1, L2, eps, U, up, dn):
        if not np.any(ok):
            continue
        idx = index_of(keys, u[ok], d[ok], N)
        if np.any(idx < 0):
            raise AssertionError("a term left the momentum sector")
        rows.append(idx)
        cols.append(cols_all[ok])
        vals.append(coef[ok] if np.ndim(coef) else np.full(int(ok.sum()), coef))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H


def hv_rows_k(L1, L2, eps, U, keys, x, rows):
    """(H_K x)[r] for the listed rows only.  H_K is real symmetric, so row r is
    sum over the terms of H|r> of (coefficient) * x[index of the result].
    Also returns, per row, the sum of |coefficient * x| and the number of terms
    (for rounding bounds)."""
    N = L1 * L2
    rows = np.asarray(rows, np.int64)
    up, dn = split_keys(keys[rows], N)
    y = np.zeros(len(rows))
    a = np.zeros(len(rows))
    n = np.zeros(len(rows), np.int64)
    for coef, ok, u, d in apply_terms(L1, L2, eps, U, up, dn):
        if not np.any(ok):
            continue
        idx = index_of(keys, u[ok], d[ok], N)
        assert np.all(idx >= 0)
        c = coef[ok] if np.ndim(coef) else coef
        v = c * x[idx]
        np.add.at(y, np.nonzero(ok)[0], v)
        np.add.at(a, np.nonzero(ok)[0], np.abs(v))
        np.add.at(n, np.nonzero(ok)[0], 1)
    return y, a, n


# ---- the paper's k-space mapping (Eqs. 5-7), for checking the reading only --------------------

def extended_counts(L1, L2, n_max):
    """C[i][m][k]: m-electron strings on orbitals 0..i-1 with total momentum k.

    Recursion of Eq. (5), reading the added orbital of an i-orbital string as
    orbital i-1: C[i][m][k] = C[i-1][m][k] + C[i-1][m-1][k - k_{i-1}], starting
    from C[0][0][k] = 1 if k = 0 (the Gamma point) else 0.
    """
    N = L1 * L2
    C = np.zeros((N + 1, n_max + 1, N), dtype=object)
    C[0][0][0] = 1
    for i in range(1, N + 1):
        for m in range(n_max + 1):
            for k in range(N):
                C[i][m][k] = C[i - 1][m][k] + (C[i - 1][m - 1][k_sub(k, i - 1, L1, L2)] if m > 0 else 0)
    return C


def forward_map_k(phi, C, L1, L2):
    """(index among the strings of its momentum, that momentum): Eq. (6) accumulated bit by bit."""
    idx, m, k = 0, 0, 0
    for i in range(L1 * L2):
        if (int(phi) >> i) & 1:
            m += 1
            k = k_add(k, i, L1, L2)
            idx += C[i][m][k]
    return idx, k


def spinful_counts(C, L1, L2, n_dn):
    """Ctilde[i][m][k] = sum_{k_dn} C[i][m][k - k_dn] * C[N][n_dn][k_dn] (Eq. 7)."""
    N = L1 * L2
    n_max = C.shape[1] - 1
    Ct = np.zeros((N + 1, n_max + 1, N), dtype=object)
    for i in range(N + 1):
        for m in range(n_max + 1):
            for k in range(N):
                Ct[i][m][k] = sum(C[i][m][k_sub(k, kd, L1, L2)] * C[N][n_dn][kd] for kd in range(N))
    return Ct


def forward_map_k_spin(phi_up, phi_dn, C, Ct, L1, L2):
    """Index of (phi_up, phi_dn) in its momentum sector: the down string's own
    rank, plus for each up bit the spin-full count at the running momentum,
    which starts from the down string's momentum."""
    idx_dn, k = forward_map_k(phi_dn, C, L1, L2)
    idx, m = 0, 0
    for i in range(L1 * L2):
        if (int(phi_up) >> i) & 1:
            m += 1
            k = k_add(k, i, L1, L2)
            idx += Ct[i][m][k]
    return idx + idx_dn
