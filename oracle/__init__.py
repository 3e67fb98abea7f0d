"""CPU FP64 oracle for the Hubbard H.v / Lanczos hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the CPU
baseline leg of bench.py may import, call, link or execute anything under
oracle/.  The product library never routes through it.

Everything here is the plain definition, written from the paper:

* the basis is the tensor product of per-spin sorted lists of occupation bit
  strings (Sec. II.A, the 4-site table), composite index
  idx = C(N, n_dn) * idx_up + idx_dn (Sec. III, after the forward-map example);
* an index is found by binary search over the stored sorted list, the
  "traditional" method of Sec. II.C, not by the perfect hash;
* H is Eq. (1), applied through explicit fermion operator algebra on the
  normal-ordered string of Sec. II.A (up operators left of down operators,
  site index increasing right to left), so every sign is counted, not derived;
* Lanczos is the textbook three-term recurrence (cited in Sec. I) with full
  re-orthogonalisation and LAPACK's tridiagonal eigensolver;
* the random start vector is SplitMix64 (Steele, Lea, Flood, OOPSLA 2014);
* fermion operators between sectors and the resolvent of the dynamical
  correlations are the operator algebra above and a spectral sum (dynamics.py);
* total-momentum sectors (Sec. IV.A) are sorted lists of (up, down) orbital
  strings and Eq. (4) applied term by term with the same algebra (momentum.py);
* inversion-parity subspaces (Sec. IV.B) are representatives in the decision
  tree's order and the projection B^T H B of the real-space H (inversion.py).

The oracle shares no code with the HIP path.  Its inputs come from synth/.
"""
from .fock import (sector_list, popcount, index_in_sorted, composite_keys, count_below,
                   apply_hop, apply_hop_vec, annihilate_sign, create_sign)
from .hamiltonian import (Problem, build_csr, hv_rows, diag_values, nnz_structural,
                          one_body_matrix)
from .lanczos import lanczos, LanczosResult
from .splitmix import splitmix64_mix, splitmix64_outputs, start_vector
from . import mlp
from . import dynamics
from . import momentum
from . import inversion

__all__ = [n for n in dir() if not n.startswith("_")]
