"""Pins of the inversion-symmetric oracle (Sec. IV.B) against what the mathematics fixes.

* F (site i -> N-1-i, signs from the operator algebra) is an involution that
  commutes with H for mirror-symmetric bonds;
* the two parity subspaces partition the sector (D_+ + D_- = D) and the union
  of the spectra of H_+ and H_- is the spectrum of H from the real-space oracle;
* the basis vectors are orthonormal and B B^T is the projector (1 + P F)/2;
* the paper's counts S_i^m and its single-string forward map (in the reading
  of the design notes) reproduce the tree order of the definition;
* the reordering sign is (-1)^(n_up(n_up-1)/2 + n_dn(n_dn-1)/2), a constant
  per sector (what the device path uses);
* row-sampled H_P x agrees with B^T H B x; a planted sign mistake is caught.
"""
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import inversion as inv
from oracle.fock import sector_list


def _chain(N, t=1.0, tp=0.0, periodic=False):
    b = [(i, i + 1, t) for i in range(N - 1)]
    if periodic:
        b.append((N - 1, 0, t))
    if tp:
        b += [(i, i + 2, tp) for i in range(N - 2)]
    return b


def _open_rect(Lx, Ly, t=1.0, tp=0.0):
    b = []
    for y in range(Ly):
        for x in range(Lx):
            s = x + Lx * y
            if x + 1 < Lx:
                b.append((s, s + 1, t))
            if y + 1 < Ly:
                b.append((s, s + Lx, t))
            if tp and x + 1 < Lx and y + 1 < Ly:
                b.append((s, s + Lx + 1, tp))
            if tp and x >= 1 and y + 1 < Ly:
                b.append((s, s + Lx - 1, tp))
    return b


def _problem(N, bonds, U, nu, nd):
    return oracle.Problem(N, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds], U, nu, nd)


CASES = [
    (8, _chain(8), 4.0, 4, 4),
    (7, _chain(7, 1.0, 0.3), 3.0, 3, 2),
    (9, _open_rect(3, 3, 1.0, 0.2), 5.0, 3, 3),
    (8, _open_rect(4, 2), 6.0, 3, 4),
    (8, _chain(8, periodic=True), 2.0, 4, 3),
    (6, _chain(6), 3.0, 0, 3),
]
IDS = ["chain8", "chain7_nnn", "open3x3", "open4x2", "ring8", "nup0"]


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_parity_spectra_together_are_the_sector_spectrum(case):
    N, bonds, U, nu, nd = case
    p = _problem(N, bonds, U, nu, nd)
    assert inv.mirror_symmetric(N, p.bond_i, p.bond_j, p.bond_t)
    H = oracle.build_csr(p)
    F = inv.inversion_matrix(N, nu, nd)
    assert abs(F @ F - sp.identity(H.shape[0])).max() == 0.0
    assert abs(F @ H - H @ F).max() < 1e-14
    ev = []
    dims = 0
    for P in (1, -1):
        B = inv.basis_matrix(N, nu, nd, P)
        dims += B.shape[1]
        np.testing.assert_allclose((B.T @ B).toarray(), np.eye(B.shape[1]), atol=1e-14)
        proj = (sp.identity(H.shape[0]) + P * F) / 2
        assert abs(B @ B.T - proj).max() < 1e-14
        HP = inv.build_csr_P(p, P)
        assert abs(HP - HP.T).max() < 1e-13
        if HP.shape[0]:
            ev.append(np.linalg.eigvalsh(HP.toarray()))
    assert dims == H.shape[0]
    np.testing.assert_allclose(np.sort(np.concatenate(ev)), np.linalg.eigvalsh(H.toarray()), atol=1e-10)


@pytest.mark.parametrize("nu,nd", [(0, 0), (1, 2), (3, 3), (4, 5), (2, 7)])
def test_reordering_sign_is_constant_per_sector(nu, nd):
    N = 7
    want = (-1) ** (nu * (nu - 1) // 2 + nd * (nd - 1) // 2)
    for u in sector_list(N, nu):
        for d in sector_list(N, nd)[::3]:
            assert inv.reorder_sign(u, d, N) == want


@pytest.mark.parametrize("N,n", [(8, 4), (9, 4), (10, 3), (7, 0), (6, 6), (11, 5)])
def test_paper_counts_and_forward_map_give_the_tree_order(N, n):
    reps = inv.tree_order(N, n)
    S = inv.paper_counts(N, n)
    assert S[N][n] == len(reps)
    pal = sum(1 for r in reps if inv.classify(r, N)[0] == "P")
    assert 2 * len(reps) - pal == comb(N, n)          # every orbit once, pairs counted twice
    assert [inv.paper_forward_map_inversion(r, N, n) for r in reps] == list(range(len(reps)))


def test_full_rows_hold_every_down_string_in_ascending_order():
    """Behind a non-palindromic up representative the row is the whole down sector in its plain order."""
    for N, n in ((8, 4), (9, 4), (6, 3)):
        assert inv.full_row_order(N, n) == [int(s) for s in sector_list(N, n)]


def test_row_index_matches_the_basis_order():
    for (N, bonds, U, nu, nd) in CASES[:4]:
        for P in (1, -1):
            bu, bd, _ = inv.basis(N, nu, nd, P)
            ridx = inv.RowIndex(N, nu, nd, P)
            assert ridx.D == len(bu)
            assert [ridx.index(u, d) for u, d in zip(bu, bd)] == list(range(len(bu)))


@pytest.mark.parametrize("case", CASES[:4], ids=IDS[:4])
def test_sampled_rows_match_the_projected_matrix(case):
    N, bonds, U, nu, nd = case
    p = _problem(N, bonds, U, nu, nd)
    for P in (1, -1):
        HP = inv.build_csr_P(p, P)
        bu, bd, _ = inv.basis(N, nu, nd, P)
        x = np.random.default_rng(4).uniform(-1, 1, len(bu))
        rows = np.arange(0, len(bu), 11)
        ridx = inv.RowIndex(N, nu, nd, P)
        lookup = lambda uu, dd: x[[ridx.index(u, d) for u, d in zip(uu, dd)]]   # noqa: E731
        y, a, n = inv.hv_rows_P(p, P, lookup, bu[rows], bd[rows])
        np.testing.assert_allclose(y, (HP @ x)[rows], atol=1e-12)


def test_planted_sign_mistake_is_caught(monkeypatch):
    N, bonds, U, nu, nd = CASES[0]
    p = _problem(N, bonds, U, nu, nd)
    ev_r = np.linalg.eigvalsh(oracle.build_csr(p).toarray())
    monkeypatch.setattr(inv, "reorder_sign", lambda u, d, N: 1 if (int(u) + int(d)) % 3 else -1)
    ev = np.sort(np.concatenate([np.linalg.eigvalsh(inv.build_csr_P(p, P).toarray()) for P in (1, -1)]))
    assert len(ev) != len(ev_r) or np.max(np.abs(ev - ev_r)) > 1e-3
