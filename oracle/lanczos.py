"""Textbook Lanczos for the lowest eigenvalue (the Krylov method cited in Sec. I).

Recurrence: w = H v_k - beta_k v_{k-1};  alpha_k = <v_k, w>;  w -= alpha_k v_k;
full re-orthogonalisation against every previous v (classical Gram-Schmidt,
applied twice);  beta_{k+1} = |w|;  v_{k+1} = w / beta_{k+1}.
The Ritz value is the lowest eigenvalue of the tridiagonal T_k (LAPACK via
scipy), and the pair is accepted when beta_{k+1} |s_k| <= tol |theta|, with s_k
the last component of the normalised eigenvector of T_k.  If beta_{k+1} is
zero the Krylov space is invariant and theta is exact.
"""
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
from scipy.linalg import eigh_tridiagonal


@dataclass
class LanczosResult:
    E0: float
    iters: int
    converged: bool
    resid_est: float
    alphas: List[float] = field(default_factory=list)
    betas: List[float] = field(default_factory=list)
    thetas: List[float] = field(default_factory=list)
    ritz: Optional[np.ndarray] = None


def _lowest(alphas, betas_off):
    a = np.asarray(alphas, dtype=np.float64)
    if len(a) == 1:
        return a[0], np.array([1.0])
    w, v = eigh_tridiagonal(a, np.asarray(betas_off, dtype=np.float64),
                            select="i", select_range=(0, 0))
    return w[0], v[:, 0]


def lanczos(matvec: Callable[[np.ndarray], np.ndarray], v0: np.ndarray, max_iter: int = 300,
            tol: float = 1e-12, reorth: bool = True, want_vector: bool = False) -> LanczosResult:
    v = np.array(v0, dtype=np.float64)
    nrm = np.linalg.norm(v)
    if not np.isfinite(nrm) or nrm == 0.0:
        raise ValueError("start vector has zero or non-finite norm")
    v /= nrm
    V = None
    nV = 0
    if reorth or want_vector:
        V = np.empty((max_iter + 1, len(v)), dtype=np.float64)
        V[0] = v
        nV = 1
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas, thetas = [], [], []
    theta, s = 0.0, np.array([1.0])
    converged, resid = False, np.inf
    k = 0
    for k in range(1, max_iter + 1):
        w = matvec(v) - beta * v_prev
        alpha = float(np.dot(v, w))
        w -= alpha * v
        if reorth:
            for _ in range(2):
                Q = V[:nV]
                w -= Q.T @ (Q @ w)
        alphas.append(alpha)
        beta_next = float(np.linalg.norm(w))
        theta, s = _lowest(alphas, betas)
        thetas.append(float(theta))
        resid = beta_next * abs(s[-1])
        if beta_next == 0.0 or resid <= tol * max(abs(theta), 1e-300):
            converged = True
            betas.append(beta_next)
            break
        betas.append(beta_next)
        v_prev, v = v, w / beta_next
        beta = beta_next
        if V is not None:
            V[nV] = v
            nV += 1
    ritz = None
    if want_vector and V is not None:
        m = len(alphas)
        ritz = V[:m].T @ s
    return LanczosResult(float(theta), k, converged, float(resid), alphas, betas[:len(alphas)], thetas, ritz)
