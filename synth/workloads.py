"""Named Hubbard workloads.

Each workload is a problem statement: number of sites, bond list, U and the
fillings n_up, n_dn (Sec. II.A).  Sizes follow from D = C(N, n_up) C(N, n_dn);
the figures quoted in the docstrings are for orientation only.
"""
from dataclasses import dataclass, field
from math import comb
from typing import List

import numpy as np

from .lattices import Bond, ring, torus, torus_nnn, single_bond


@dataclass
class Workload:
    name: str
    n_sites: int
    bonds: List[Bond]
    U: float
    n_up: int
    n_dn: int
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def D(self) -> int:
        return comb(self.n_sites, self.n_up) * comb(self.n_sites, self.n_dn)


def _mk():
    w = {}
    # ring of 8 sites at half filling: D = 70^2 = 4900
    w["ring8"] = Workload("ring8", 8, ring(8, 1.0), 4.0, 4, 4,
                          "1D ring L=8, periodic, 4+4, t=1, U=4")
    # 4x3 periodic cluster at half filling: D = 924^2 = 853,776
    w["torus4x3"] = Workload("torus4x3", 12, torus(4, 3, 1.0), 8.0, 6, 6,
                             "2D 4x3 periodic NN, 6+6, t=1, U=8")
    # 4x4 periodic cluster with t'=-0.3 at half filling: D = 12870^2 = 165,636,900
    w["torus4x4_nnn"] = Workload("torus4x4_nnn", 16, torus_nnn(4, 4, 1.0, -0.3), 6.0, 8, 8,
                                 "2D 4x4 periodic NN+NNN (t'=-0.3), 8+8, t=1, U=6")
    # 4x4 periodic NN cluster, 7+7: D = 11440^2 = 130,873,600
    w["torus4x4_n7"] = Workload("torus4x4_n7", 16, torus(4, 4, 1.0), 5.0, 7, 7,
                                "2D 4x4 periodic NN, 7+7, t=1, U=5")
    w["two_site"] = Workload("two_site", 2, single_bond(1.0), 4.0, 1, 1,
                             "two sites, one bond, 1+1")
    return w


WORKLOADS = _mk()


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def batched_workloads(count: int = 32, seed: int = 20170712) -> List[Workload]:
    """Mixed batch of 4x3 and 3x3 periodic clusters.

    Lattice chosen with probability 1/2 each, n_up and n_dn independently
    uniform on {3,4,5,6}, U uniform on [0, 8), t = 1.
    """
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        if rng.random() < 0.5:
            Lx, Ly = 4, 3
        else:
            Lx, Ly = 3, 3
        n_up = int(rng.integers(3, 7))
        n_dn = int(rng.integers(3, 7))
        U = float(rng.random() * 8.0)
        out.append(Workload(f"batch{k}_{Lx}x{Ly}_{n_up}_{n_dn}", Lx * Ly, torus(Lx, Ly, 1.0), U,
                            n_up, n_dn, f"{Lx}x{Ly} periodic NN, {n_up}+{n_dn}, U={U:.3f}"))
    return out
