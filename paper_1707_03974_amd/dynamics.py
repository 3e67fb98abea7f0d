"""Dynamical correlations by the Lanczos continued fraction (a driver over libpdz calls).

For a state psi0 of the sector (n_up, n_dn) and the operator O = c_{j,s} (op 0) or c+_{j,s}
(op 1), phi = O psi0 lies in the neighbouring sector; Lanczos on that sector's H started at
phi gives coefficients alpha, beta whose continued fraction is the resolvent
    R(w) = <phi|(w - H)^{-1}|phi>,
from which the removal (op 0) and addition (op 1) parts of the one-particle Green's function
follow, e.g. G_removal(omega) = -R(E0 - omega - i eta) for the electron-removal spectrum.  The
operator, the Lanczos run and the continued fraction all run in libpdz.
"""
from . import Problem, fermion_op, continued_fraction


def neighbour_problem(problem, spin, op):
    """The Problem on the same lattice with one electron of `spin` fewer (op 0) or more (op 1)."""
    d = -1 if op == 0 else 1
    nu = problem.n_up + (d if spin == 0 else 0)
    nd = problem.n_dn + (d if spin == 1 else 0)
    return Problem(problem.n_sites, problem.bonds, problem.U, nu, nd)


def resolvent(problem, psi0, site, spin, op, w, steps=200, storage="f64", target=None, reorth=0):
    """R(w) = <phi|(w - H)^{-1}|phi> with phi = c or c+ (op) on psi0, from `steps` Lanczos steps in the
    target sector (fewer when the Krylov space closes; reorth=1 re-orthogonalises each step locally, reorth=2 fully).
    Returns (R at the points w, Lanczos result)."""
    import torch
    tgt = target if target is not None else neighbour_problem(problem, spin, op)
    phi = fermion_op(problem, tgt, site, spin, op, psi0)
    want = torch.float64 if storage == "f64" else torch.float32
    if phi.dtype != want:
        phi = phi.to(want)
    r = tgt.lanczos(v0=phi, storage=storage, tol=0.0, max_iter=steps, coefficients=True, reorth=reorth)
    g = continued_fraction(r["alpha"], r["beta"], r["norm0"] ** 2, w)
    return g, r
