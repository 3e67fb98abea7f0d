"""Inversion-symmetric Hubbard subspaces, from their definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. IV.B: the site map i -> N-1-i (a chain reversed; for an Lx x Ly cluster
numbered s = x + Lx*y, the point inversion through its centre) applied to
every creation operator, F(c+_i) = c+_{N-1-i}, squares to one; when the bonds
are mirror symmetric it commutes with H and splits each (n_up, n_dn) sector
into parity P = +1 and P = -1 subspaces.

Definitions used here:

* F on a basis state is applied through the operator algebra: the image
  string reversed, and the sign of reordering the created operators back to
  the normal order of Sec. II.A (counted, not assumed).
* One string's classification (Sec. IV.B, the decision tree): at depth d the
  pair (bit N-1-d, bit d) is class A = (0, 1), B = (0, 0), C = (1, 1), or
  (1, 0), which is the mirror image of an A string; classification stops at
  the first A; a string whose pairs are all B or C is a palindrome.  A string
  is a representative when it is an A string or a palindrome.  Tree order:
  depth first, A before B before C at each depth; strings that stop at the
  same A node are ordered by their inner bits (d+1 .. N-2-d) as in the plain
  forward map; for odd N the middle bit of a palindrome orders 0 before 1.
* Two spins (the paper treats one string; reading stated in the design
  notes): a state's representative is decided by its up string, and by its
  down string when the up string is a palindrome.  Basis order: up
  representatives in tree order; behind a non-palindromic up string every
  down string in ascending order (the plain sector order of Sec. II.A);
  behind a palindromic up string the down representatives in tree order,
  down palindromes only when the state is itself even (F|s> = P|s>).
  Only the set of basis states and each state's basis vector are part of
  the method; a device layout may order them differently, and tests compare
  through the state a position holds.
* Basis vector of a representative r: (|r> + P F|r>) / sqrt(2), or |r> for a
  state with F|r> = +-|r> (kept only when F|r> = P|r>).
* H_P = B^T H B with B the matrix of those basis vectors and H the real-space
  oracle's H (oracle.hamiltonian): a plain projection.

The paper's single-string forward / backward inversion maps and its counts
S_i^m are written out at the end only so that the CPU tests can check the
reading of the tree order against the definitions above.
"""
from math import comb

import numpy as np
import scipy.sparse as sp

from .fock import sector_list, popcount, count_below
from .hamiltonian import build_csr


def reverse(phi, N):
    phi = int(phi)
    return sum(1 << (N - 1 - i) for i in range(N) if (phi >> i) & 1)


def mirror_symmetric(N, bond_i, bond_j, bond_t, tol=1e-12):
    """True when the bond list is invariant under i -> N-1-i."""
    bonds = {}
    for i, j, t in zip(bond_i, bond_j, bond_t):
        k = (min(i, j), max(i, j))
        bonds[k] = bonds.get(k, 0.0) + float(t)
    for (i, j), t in bonds.items():
        a, b = N - 1 - i, N - 1 - j
        if abs(bonds.get((min(a, b), max(a, b)), 0.0) - t) > tol:
            return False
    return True


def reorder_sign(phi_up, phi_dn, N):
    """Sign of F on the basis state: reordering the reversed creation strings.

    The state is prod over up sites (descending) then down sites (descending)
    of c+ on the vacuum; F sends site i to N-1-i, which reverses the order of
    each spin's operators; restoring descending order takes one transposition
    per pair of operators of the same spin (counted pair by pair here).
    """
    cnt = 0
    for phi in (phi_up, phi_dn):
        sites = [i for i in range(N - 1, -1, -1) if (int(phi) >> i) & 1]   # normal order
        img = [N - 1 - i for i in sites]                                      # after F, same slots
        for a in range(len(img)):
            for b in range(a + 1, len(img)):
                if img[a] < img[b]:
                    cnt += 1
    return -1 if cnt % 2 else 1


def classify(phi, N):
    """('A', d) | ('X', d) for the first asymmetric pair at depth d ((0,1) / (1,0)), or ('P', None)."""
    phi = int(phi)
    for d in range(N // 2):
        hi, lo = (phi >> (N - 1 - d)) & 1, (phi >> d) & 1
        if hi != lo:
            return ("A", d) if lo == 1 else ("X", d)
    return ("P", None)


def is_representative(phi, N):
    return classify(phi, N)[0] != "X"


def tree_key(phi, N):
    """Sort key of a representative string in the depth-first tree order."""
    phi = int(phi)
    key = []
    for d in range(N // 2):
        hi, lo = (phi >> (N - 1 - d)) & 1, (phi >> d) & 1
        if hi == 0 and lo == 1:
            width = N - 2 - 2 * d
            inner = (phi >> (d + 1)) & ((1 << width) - 1) if width > 0 else 0
            key += [0, count_below(inner, popcount(inner))]
            return tuple(key)
        if hi == lo:
            key.append(1 if hi == 0 else 2)
        else:
            raise ValueError("not a representative")
    if N % 2:
        key.append(3 + ((phi >> (N // 2)) & 1))
    return tuple(key)


def tree_order(N, n):
    """Representative strings of n electrons on N sites in tree order."""
    reps = [int(s) for s in sector_list(N, n) if is_representative(s, N)]
    return sorted(reps, key=lambda s: tree_key(s, N))


def full_row_order(N, n):
    """Down strings of a non-palindromic row: every string of the sector, ascending."""
    return [int(d) for d in sector_list(N, n)]


def basis(N, n_up, n_dn, P):
    """The parity-P basis as parallel arrays (up, dn, kind): kind 2 for a pair
    state (|r> + P F|r>)/sqrt(2), 1 for a state that F maps onto +-itself."""
    dn_all = full_row_order(N, n_dn)
    dn_reps = tree_order(N, n_dn)
    up, dn, kind = [], [], []
    for u in tree_order(N, n_up):
        if classify(u, N)[0] == "A":
            for d in dn_all:
                up.append(u); dn.append(d); kind.append(2)
        else:
            for d in dn_reps:
                if classify(d, N)[0] == "A":
                    up.append(u); dn.append(d); kind.append(2)
                elif reorder_sign(u, d, N) == P:   # F|s> = P|s>: the state is in this subspace
                    up.append(u); dn.append(d); kind.append(1)
    return np.array(up, np.uint64), np.array(dn, np.uint64), np.array(kind, np.int64)


def basis_matrix(N, n_up, n_dn, P):
    """B (D x D_P, sparse): column k is the k-th basis vector on the sorted full basis."""
    up_l, dn_l = sector_list(N, n_up), sector_list(N, n_dn)
    Ddn = len(dn_l)
    bu, bd, kind = basis(N, n_up, n_dn, P)

    def full_index(u, d):
        return int(np.searchsorted(up_l, np.uint64(u))) * Ddn + int(np.searchsorted(dn_l, np.uint64(d)))

    rows, cols, vals = [], [], []
    for k, (u, d, kd) in enumerate(zip(bu, bd, kind)):
        r = full_index(u, d)
        if kd == 1:
            rows.append(r); cols.append(k); vals.append(1.0)
        else:
            s = reorder_sign(u, d, N)
            rows += [r, full_index(reverse(u, N), reverse(d, N))]
            cols += [k, k]
            vals += [1 / np.sqrt(2), P * s / np.sqrt(2)]
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(up_l) * Ddn, len(bu)))


def inversion_matrix(N, n_up, n_dn):
    """F on the sorted full basis (a signed permutation)."""
    up_l, dn_l = sector_list(N, n_up), sector_list(N, n_dn)
    Ddn = len(dn_l)
    rows, cols, vals = [], [], []
    for iu, u in enumerate(up_l):
        for idn, d in enumerate(dn_l):
            tgt = int(np.searchsorted(up_l, np.uint64(reverse(u, N)))) * Ddn + \
                int(np.searchsorted(dn_l, np.uint64(reverse(d, N))))
            rows.append(tgt); cols.append(iu * Ddn + idn); vals.append(float(reorder_sign(u, d, N)))
    D = len(up_l) * Ddn
    return sp.csr_matrix((vals, (rows, cols)), shape=(D, D))


def build_csr_P(p, P):
    """H restricted to the parity-P subspace, B^T H B, in the basis order above."""
    if not mirror_symmetric(p.n_sites, p.bond_i, p.bond_j, p.bond_t):
        raise ValueError("bonds are not mirror symmetric")
    B = basis_matrix(p.n_sites, p.n_up, p.n_dn, P)
    H = build_csr(p)
    return (B.T @ H @ B).tocsr()


class RowIndex:
    """Position of any representative (up, dn) in the parity-P basis without
    listing the whole basis: row order of the up representatives, offsets, and
    the column of the down string within its row."""

    def __init__(self, N, n_up, n_dn, P):
        self.N, self.P = N, P
        self.ups = tree_order(N, n_up)
        self.dn_all = full_row_order(N, n_dn)
        self.dn_col_full = {d: k for k, d in enumerate(self.dn_all)}
        self.offsets, self.pal_cols = {}, {}
        off = 0
        for u in self.ups:
            self.offsets[u] = off
            if classify(u, N)[0] == "A":
                off += len(self.dn_all)
            else:
                cols = {}
                for d in tree_order(N, n_dn):
                    if classify(d, N)[0] == "A" or reorder_sign(u, d, N) == P:
                        cols[d] = len(cols)
                self.pal_cols[u] = cols
                off += len(cols)
        self.D = off

    def index(self, u, d):
        u, d = int(u), int(d)
        if u in self.pal_cols:
            return self.offsets[u] + self.pal_cols[u][d]
        return self.offsets[u] + self.dn_col_full[d]


def representative(u, d, N):
    """(rep_up, rep_dn, imaged): the representative of the orbit of (u, d) and whether (u, d) is its image."""
    cu = classify(u, N)[0]
    if cu == "A":
        return int(u), int(d), False
    if cu == "X":
        return reverse(u, N), reverse(d, N), True
    cd = classify(d, N)[0]
    if cd == "X":
        return int(u), reverse(d, N), True
    return int(u), int(d), False


def hv_rows_P(p, P, lookup, rows_up, rows_dn):
    """(H_P x) at the listed basis states (representatives), without building H_P.

    (H_P x)_t = <t_P| H |v> with |v> = sum_k x_k |k_P>: the full-space vector
    v at any state s is x at rep(s) times 1/sqrt(2) (pair states; times P F's
    sign for the image) or 1 (self-mapped states), and <t_P| reads the row of
    H at t (and at F t) with the same weights.  H's terms come from oracle's
    real-space operator algebra (hv_rows on single states).
    lookup(reps_up, reps_dn) -> the x component of each listed representative
    state (arrays), so x may be held in any order of the basis.
    Returns (y, sum of |terms|, number of terms).
    """
    from .fock import apply_hop
    N = p.n_sites
    # pass 1: every term of every row, with the representative it reads
    rows_terms, need = [], {}
    for u, d in zip(rows_up, rows_dn):
        u, d = int(u), int(d)
        s0 = reorder_sign(u, d, N)
        self_mapped = reverse(u, N) == u and reverse(d, N) == d
        orbit = [(u, d, 1.0)] if self_mapped else [(u, d, 1 / np.sqrt(2)),
                                                   (reverse(u, N), reverse(d, N), P * s0 / np.sqrt(2))]
        row = []
        for (su, sd, w_t) in orbit:
            # H|v> at state (su, sd): sum over the sources of the row (symmetric H)
            terms = [(float(p.U) * popcount(su & sd), su, sd)]
            for i, j, t in zip(p.bond_i, p.bond_j, p.bond_t):
                for spin in (0, 1):
                    for a_, b_ in ((i, j), (j, i)):
                        r = apply_hop(su, sd, spin, a_, b_)
                        if r is not None:
                            sign, nu, nd = r
                            terms.append((-float(t) * sign, nu, nd))
            for coef, nu, nd in terms:
                if coef == 0.0:
                    continue
                ru, rd, img = representative(nu, nd, N)
                sm = reverse(ru, N) == ru and reverse(rd, N) == rd
                if sm and reorder_sign(ru, rd, N) != P:
                    continue          # a self-mapped state of the other parity: no component here
                w_s = 1.0 if sm else (P * reorder_sign(ru, rd, N) / np.sqrt(2) if img else 1 / np.sqrt(2))
                need.setdefault((ru, rd), len(need))
                row.append((w_t * coef * w_s, (ru, rd)))
        rows_terms.append(row)
    # pass 2: the x components of every representative read, then the sums in term order
    keys = list(need)
    xv = np.asarray(lookup(np.array([k[0] for k in keys], np.uint64), np.array([k[1] for k in keys], np.uint64)),
                    dtype=np.float64) if keys else np.zeros(0)
    out, asum, nterm = [], [], []
    for row in rows_terms:
        acc, a = 0.0, 0.0
        for w, key in row:
            v = w * xv[need[key]]
            acc += v
            a += abs(v)
        out.append(acc)
        asum.append(a)
        nterm.append(len(row))
    return np.array(out), np.array(asum), np.array(nterm)


# ---- the paper's single-string maps (Sec. IV.B), for checking the reading only ------------------

def paper_counts(N, n_max):
    """S[i][m] (representatives with the palindromes) by the recursion S_i^m = C_{i-2}^{m-1} +
    S_{i-2}^m + S_{i-2}^{m-2}, from S_0^0 = 1 and S_1^m = 1 for m in {0, 1}."""
    S = [[0] * (n_max + 1) for _ in range(N + 1)]
    for i in range(N + 1):
        for m in range(n_max + 1):
            if i == 0:
                S[i][m] = 1 if m == 0 else 0
            elif i == 1:
                S[i][m] = 1 if m <= 1 else 0
            else:
                S[i][m] = (comb(i - 2, m - 1) if m >= 1 else 0) + S[i - 2][m] + (S[i - 2][m - 2] if m >= 2 else 0)
    return S


def paper_forward_map_inversion(phi, N, n):
    """Tree-order index of a representative: at each depth, an A pair ends with the inner
    string's plain rank; B skips the A node's strings; C skips the A and B nodes'."""
    S = paper_counts(N, n)
    phi, idx, m, i = int(phi), 0, n, N
    for d in range(N // 2):
        hi, lo = (phi >> (N - 1 - d)) & 1, (phi >> d) & 1
        a_cnt = comb(i - 2, m - 1) if m >= 1 else 0
        if hi == 0 and lo == 1:
            width = i - 2
            inner = (phi >> (d + 1)) & ((1 << width) - 1) if width > 0 else 0
            return idx + count_below(inner, m - 1)
        if hi == 0 and lo == 0:
            idx += a_cnt
        elif hi == 1 and lo == 1:
            idx += a_cnt + S[i - 2][m]
            m -= 2
        else:
            raise ValueError("not a representative")
        i -= 2
    return idx   # a palindrome: the last node holds only this string
