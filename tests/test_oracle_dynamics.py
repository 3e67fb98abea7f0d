"""Pins of the oracle's fermion operators between sectors and of its resolvent.

The operator is pinned by the canonical anticommutation relations, by
c+_a c_b reproducing the hopping term of the oracle's H (so the operator and
H use one sign convention), and by the density sum rule; the resolvent by a
direct linear solve and by its large-|w| moments.
"""
import numpy as np
import pytest

import oracle
from oracle import dynamics as dy

N, NU, ND = 6, 2, 3


def _psi(nu, nd, seed):
    D = len(oracle.sector_list(N, nu)) * len(oracle.sector_list(N, nd))
    return np.random.default_rng(seed).standard_normal(D)


def _op(site, spin, op, psi, nu, nd):
    return dy.apply_fermion(N, nu, nd, site, spin, op, psi), dy.target_fillings(nu, nd, spin, op)


@pytest.mark.parametrize("s1,s2", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_anticommutator_of_c_and_cdagger_is_delta(s1, s2):
    psi = _psi(NU, ND, 1)
    for i in range(N):
        for j in range(N):
            a, fa = _op(j, s2, 1, psi, NU, ND)            # c+_j psi
            ca, _ = _op(i, s1, 0, a, *fa)                 # c_i c+_j psi
            b, fb = _op(i, s1, 0, psi, NU, ND)            # c_i psi
            cb, _ = _op(j, s2, 1, b, *fb)                 # c+_j c_i psi
            expect = psi if (i == j and s1 == s2) else np.zeros_like(ca)
            assert np.allclose(ca + cb, expect, atol=1e-12), (i, j, s1, s2)


def test_annihilators_anticommute():
    psi = _psi(NU, ND, 2)
    for s1 in (0, 1):
        for s2 in (0, 1):
            for i in range(N):
                for j in range(N):
                    a, fa = _op(j, s2, 0, psi, NU, ND)
                    ab, _ = _op(i, s1, 0, a, *fa)
                    b, fb = _op(i, s1, 0, psi, NU, ND)
                    ba, _ = _op(j, s2, 0, b, *fb)
                    assert np.allclose(ab + ba, 0.0, atol=1e-12)


def test_cdagger_c_reproduces_the_hopping_term_of_H():
    bonds = [(0, 1, 1.0), (1, 2, 0.7), (2, 5, -0.4), (3, 4, 1.3), (0, 5, 0.9)]
    p = oracle.Problem(N, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds], 0.0, NU, ND)
    H = oracle.build_csr(p)
    psi = _psi(NU, ND, 3)
    out = np.zeros_like(psi)
    for i, j, t in bonds:
        for s in (0, 1):
            for a, b in ((i, j), (j, i)):
                x, fx = _op(b, s, 0, psi, NU, ND)
                y, _ = _op(a, s, 1, x, *fx)
                out -= t * y
    assert np.allclose(out, H @ psi, atol=1e-12)


def test_density_sum_rule():
    psi = _psi(NU, ND, 4)
    up, dn = oracle.sector_list(N, NU), oracle.sector_list(N, ND)
    phi_up, phi_dn = np.repeat(up, len(dn)), np.tile(dn, len(up))
    for s, bits in ((0, phi_up), (1, phi_dn)):
        for j in range(N):
            occ = ((bits >> np.uint64(j)) & np.uint64(1)).astype(np.float64)
            c, _ = _op(j, s, 0, psi, NU, ND)
            assert np.isclose(c @ c, (occ * psi ** 2).sum(), rtol=1e-13)


def test_full_and_empty_shells():
    # annihilating from an empty sector or creating into a full one gives nothing
    psi = _psi(0, ND, 5)
    assert dy.apply_fermion(N, 0, ND, 2, 0, 0, psi).size == 0
    psi = _psi(N, ND, 6)
    assert dy.apply_fermion(N, N, ND, 2, 0, 1, psi).size == 0


def test_resolvent_against_a_linear_solve_and_its_moments():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((40, 40))
    H = (A + A.T) / 2
    phi = rng.standard_normal(40)
    w = np.array([0.3 + 0.2j, -1.7 + 0.05j, 4.0 - 1.0j])
    got = dy.resolvent_exact(H, phi, w)
    for k, wk in enumerate(w):
        direct = phi @ np.linalg.solve(wk * np.eye(40) - H, phi.astype(np.complex128))
        assert abs(got[k] - direct) <= 1e-10 * abs(direct)
    big = np.array([1e6 + 0j])
    r = dy.resolvent_exact(H, phi, big)[0]
    assert abs(big[0] * r - phi @ phi) <= 1e-5 * (phi @ phi)
    first = (big[0] * (big[0] * r - phi @ phi)).real
    assert abs(first - phi @ H @ phi) <= 1e-3 * abs(phi @ H @ phi) + 1e-6


def test_planted_sign_mistake_is_caught(monkeypatch):
    """Counting the same-spin electrons below the site instead of above breaks the pins."""
    from oracle import fock

    def wrong(phi_up, phi_dn, spin, j):
        bits = np.asarray(phi_up if spin == 0 else phi_dn, dtype=np.uint64)
        below = np.bitwise_count(bits & np.uint64((1 << j) - 1)).astype(np.int64)
        return below + (0 if spin == 0 else np.bitwise_count(np.asarray(phi_up, np.uint64)).astype(np.int64))

    monkeypatch.setattr(dy, "annihilate_sign", wrong)
    bonds = [(0, 1, 1.0), (1, 2, 0.7), (2, 5, -0.4)]
    p = oracle.Problem(N, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds], 0.0, NU, ND)
    H = oracle.build_csr(p)
    psi = _psi(NU, ND, 8)
    out = np.zeros_like(psi)
    for i, j, t in bonds:
        for s in (0, 1):
            for a, b in ((i, j), (j, i)):
                x, fx = _op(b, s, 0, psi, NU, ND)
                y, _ = _op(a, s, 1, x, *fx)
                out -= t * y
    assert not np.allclose(out, H @ psi, atol=1e-6)
