"""Bond lists of periodic clusters (problem statements, not the method).

A bond (i, j, t) contributes -t (c+_i c_j + c+_j c_i) for each spin, the kinetic
term of the Hubbard Hamiltonian (Sec. II.B, Eq. 1).  Sites of an Lx x Ly
cluster are numbered row-major, s = x + Lx*y.  Every unordered pair appears at
most once; a periodic direction of length 2 would produce the same pair twice
and is rejected rather than silently doubled.
"""
from dataclasses import dataclass
from typing import List, Tuple


@dataclass(frozen=True)
class Bond:
    i: int
    j: int
    t: float


def _add(bonds: List[Bond], seen: set, a: int, b: int, t: float) -> None:
    if a == b:
        raise ValueError("self bond")
    key = (min(a, b), max(a, b))
    if key in seen:
        raise ValueError(f"duplicate bond {key}: lattice too small for its periodic wrap")
    seen.add(key)
    bonds.append(Bond(a, b, float(t)))


def single_bond(t: float = 1.0) -> List[Bond]:
    """Two sites joined by one bond (the two-site cluster)."""
    return [Bond(0, 1, float(t))]


def ring(L: int, t: float = 1.0, periodic: bool = True) -> List[Bond]:
    """1D chain of L sites, nearest-neighbour bonds (i, i+1), wrapped if periodic."""
    bonds, seen = [], set()
    for i in range(L - 1):
        _add(bonds, seen, i, i + 1, t)
    if periodic and L > 2:
        _add(bonds, seen, L - 1, 0, t)
    return bonds


def torus(Lx: int, Ly: int, t: float = 1.0) -> List[Bond]:
    """Periodic Lx x Ly square cluster, nearest-neighbour bonds."""
    bonds, seen = [], set()
    for y in range(Ly):
        for x in range(Lx):
            s = x + Lx * y
            _add(bonds, seen, s, (x + 1) % Lx + Lx * y, t)
            _add(bonds, seen, s, x + Lx * ((y + 1) % Ly), t)
    return bonds


def torus_nnn(Lx: int, Ly: int, t: float = 1.0, tp: float = 0.0) -> List[Bond]:
    """Periodic square cluster with nearest (t) and diagonal next-nearest (tp) bonds."""
    bonds = torus(Lx, Ly, t)
    seen = {(min(b.i, b.j), max(b.i, b.j)) for b in bonds}
    for y in range(Ly):
        for x in range(Lx):
            s = x + Lx * y
            _add(bonds, seen, s, (x + 1) % Lx + Lx * ((y + 1) % Ly), tp)
            _add(bonds, seen, s, (x + 1) % Lx + Lx * ((y - 1) % Ly), tp)
    return bonds


def as_arrays(bonds: List[Bond]) -> Tuple[list, list, list]:
    return [b.i for b in bonds], [b.j for b in bonds], [b.t for b in bonds]
