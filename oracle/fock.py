"""Occupation bit strings, sorted sector lists and fermion operator algebra.

Definitions followed (Sec. II.A):

* For one spin species, site i <-> bit i of an integer; a sector is every
  N-bit integer with n set bits, listed in ascending order.  The 4-site table
  of Sec. II.A lists (n=2) 3,5,6,9,10,12 and (n=3) 7,11,13,14.
* A basis element is created from the vacuum by the string
      prod_{i in up, descending i} c+_{i,up}  prod_{j in dn, descending j} c+_{j,dn} |0>
  i.e. up operators stand left of down operators and the site index grows
  from right to left.  Applying c_{j,s} or c+_{i,s} to such a string moves
  the operator past every operator standing to its left, one factor -1 each.
* Index lookup is binary search over the stored sorted list (Sec. II.C).
"""
from itertools import combinations
from math import comb

import numpy as np


def popcount(a):
    """Number of set bits of each element (numpy uint64 arrays or Python ints)."""
    if isinstance(a, (int, np.integer)):
        return bin(int(a)).count("1")
    return np.bitwise_count(np.asarray(a, dtype=np.uint64)).astype(np.int64)


def sector_list(N: int, n: int) -> np.ndarray:
    """All N-bit integers with exactly n set bits, ascending (uint64)."""
    if n < 0 or n > N:
        return np.zeros(0, dtype=np.uint64)
    vals = [sum(1 << p for p in c) for c in combinations(range(N), n)]
    out = np.array(sorted(vals), dtype=np.uint64)
    assert len(out) == comb(N, n)
    return out


def index_in_sorted(sorted_list: np.ndarray, keys) -> np.ndarray:
    """Binary search of keys in a sorted list; raises if a key is absent."""
    keys_arr = np.asarray(keys, dtype=np.uint64)
    pos = np.searchsorted(sorted_list, keys_arr)
    if np.any(pos >= len(sorted_list)) or np.any(sorted_list[np.minimum(pos, len(sorted_list) - 1)] != keys_arr):
        raise KeyError("state not in list")
    return pos.astype(np.int64)


def count_below(x: int, n: int) -> int:
    """Number of non-negative integers y < x with exactly n set bits.

    Plain counting: every such y agrees with x above some set bit i of x, has
    0 at bit i, and any n - (ones of x above i) bits among the i lower bits.
    Equals the position of x in the ascending sector list when popcount(x) = n.
    """
    x = int(x)
    total, ones_above = 0, 0
    for i in range(x.bit_length() - 1, -1, -1):
        if (x >> i) & 1:
            need = n - ones_above
            if 0 <= need <= i:
                total += comb(i, need)
            ones_above += 1
    return total


def composite_keys(up_list: np.ndarray, dn_list: np.ndarray, N: int) -> np.ndarray:
    """Sorted key list of the full basis: key = (phi_up << N) | phi_dn.

    Sorting by (phi_up, phi_dn) gives position = D_dn * idx_up + idx_dn,
    the composite index of the tensor-product basis.
    """
    ku = np.repeat(up_list, len(dn_list)) << np.uint64(N)
    kd = np.tile(dn_list, len(up_list))
    keys = ku | kd
    assert np.all(keys[1:] > keys[:-1])
    return keys


def _count_above(bits, i):
    """Number of set bits strictly above position i."""
    if isinstance(bits, (int, np.integer)):
        return popcount(int(bits) >> (i + 1))
    return popcount(np.asarray(bits, dtype=np.uint64) >> np.uint64(i + 1))


def annihilate_sign(phi_up, phi_dn, spin: int, j: int):
    """Operators standing left of c+_{j,spin} in the normal-ordered string.

    spin 0 = up, 1 = down.  Returns the count (the sign is (-1)**count).
    """
    if spin == 0:
        return _count_above(phi_up, j)
    return popcount(phi_up) + _count_above(phi_dn, j)


def create_sign(phi_up, phi_dn, spin: int, i: int):
    """Operators a new c+_{i,spin} must pass to reach its normal-ordered slot."""
    if spin == 0:
        return _count_above(phi_up, i)
    return popcount(phi_up) + _count_above(phi_dn, i)


def apply_hop(phi_up: int, phi_dn: int, spin: int, a: int, b: int):
    """Apply c+_{a,spin} c_{b,spin} to one basis state.

    Returns (sign, new_up, new_dn) or None when the result vanishes.
    """
    phi_up, phi_dn = int(phi_up), int(phi_dn)
    s = phi_up if spin == 0 else phi_dn
    if not (s >> b) & 1:
        return None
    count = annihilate_sign(phi_up, phi_dn, spin, b)
    s &= ~(1 << b)
    if spin == 0:
        u, d = s, phi_dn
    else:
        u, d = phi_up, s
    if (s >> a) & 1:
        return None
    count += create_sign(u, d, spin, a)
    s |= 1 << a
    if spin == 0:
        u = s
    else:
        d = s
    return (-1 if count % 2 else 1), u, d


def apply_hop_vec(phi_up: np.ndarray, phi_dn: np.ndarray, spin: int, a: int, b: int):
    """Vectorised c+_{a,spin} c_{b,spin} over arrays of basis states.

    Returns (mask, sign, new_up, new_dn); entries with mask False vanish.
    """
    phi_up = np.asarray(phi_up, dtype=np.uint64)
    phi_dn = np.asarray(phi_dn, dtype=np.uint64)
    s = phi_up if spin == 0 else phi_dn
    bb, ba = np.uint64(1 << b), np.uint64(1 << a)
    ok = (s & bb) != 0
    count = annihilate_sign(phi_up, phi_dn, spin, b)
    s1 = s & ~bb
    u1, d1 = (s1, phi_dn) if spin == 0 else (phi_up, s1)
    ok &= (s1 & ba) == 0
    count = count + create_sign(u1, d1, spin, a)
    s2 = s1 | ba
    u2, d2 = (s2, phi_dn) if spin == 0 else (phi_up, s2)
    sign = np.where(count % 2 == 1, -1.0, 1.0)
    return ok, sign, u2, d2
