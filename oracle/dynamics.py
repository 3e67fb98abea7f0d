"""Fermion operators between sectors and the resolvent, from their definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Dynamical correlations (Sec. I cites the continued-fraction method built on
Lanczos) need the state c_{j,s}|psi> (one electron fewer) or c+_{j,s}|psi>
(one more) and the resolvent <phi|(w - H)^{-1}|phi> in the new sector.
Here both are the plain definitions:

* the operator is applied to every basis state of the source sector with the
  operator algebra of oracle.fock (normal-ordered strings, Sec. II.A), and
  the index of each result in the target sector is found by binary search
  over the target's sorted key list (Sec. II.C);
* the resolvent is the spectral (Lehmann) sum over the eigenpairs of the
  target sector's H from a dense symmetric eigensolver:
      R(w) = sum_n |<n|phi>|^2 / (w - E_n).
"""
import numpy as np

from .fock import sector_list, composite_keys, index_in_sorted, annihilate_sign, create_sign


def target_fillings(n_up, n_dn, spin, op):
    """(n_up, n_dn) after the operator: op 0 removes, op 1 adds an electron of `spin`."""
    d = -1 if op == 0 else 1
    return (n_up + d, n_dn) if spin == 0 else (n_up, n_dn + d)


def apply_fermion(N, n_up, n_dn, site, spin, op, psi):
    """c_{site,spin} psi (op 0) or c+_{site,spin} psi (op 1); psi in sector (n_up, n_dn).

    Returns the vector in the target sector (zeros when that sector is empty).
    """
    up, dn = sector_list(N, n_up), sector_list(N, n_dn)
    tu, td = target_fillings(n_up, n_dn, spin, op)
    out_up, out_dn = sector_list(N, tu), sector_list(N, td)
    out = np.zeros(len(out_up) * len(out_dn))
    if len(out) == 0 or len(up) * len(dn) == 0:
        return out
    phi_up = np.repeat(up, len(dn))
    phi_dn = np.tile(dn, len(up))
    psi = np.asarray(psi, dtype=np.float64)
    bit = np.uint64(1 << site)
    s = phi_up if spin == 0 else phi_dn
    if op == 0:
        ok = (s & bit) != 0
        count = annihilate_sign(phi_up, phi_dn, spin, site)   # on the state before the operator
        s2 = s & ~bit
    else:
        ok = (s & bit) == 0
        count = create_sign(phi_up, phi_dn, spin, site)
        s2 = s | bit
    u2, d2 = (s2, phi_dn) if spin == 0 else (phi_up, s2)
    sign = np.where(np.asarray(count) % 2 == 1, -1.0, 1.0)
    keys_out = composite_keys(out_up, out_dn, N)
    k = (u2[ok] << np.uint64(N)) | d2[ok]
    idx = index_in_sorted(keys_out, k)
    np.add.at(out, idx, sign[ok] * psi[ok])
    return out


def resolvent_exact(H, phi, w):
    """<phi|(w - H)^{-1}|phi> for complex w (array), by the spectral sum over a dense eigh of H."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    E, V = np.linalg.eigh(Hd)
    weight = (V.T @ np.asarray(phi, dtype=np.float64)) ** 2
    w = np.asarray(w, dtype=np.complex128)
    return (weight[None, :] / (w[:, None] - E[None, :])).sum(axis=1)
