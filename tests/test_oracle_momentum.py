"""Pins of the momentum-space oracle (Sec. IV.A) against what the mathematics fixes.

* the Fourier transform of the 4x4 NN + NNN bond list is the band quoted in Sec. IV.A;
* the spectra of all total-momentum sectors together are the real-space spectrum of
  Eq. (1) from the independently pinned real-space oracle;
* U = 0: H_K is diagonal with the band energies of the occupied orbitals;
* the paper's k-space forward maps (Eqs. 5-7, in the reading stated in
  oracle/momentum.py) reproduce the sorted-list positions exactly;
* a planted sign mistake in the operator algebra breaks the spectrum pin.
"""
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import momentum as mk
from synth.lattices import ring, torus, torus_nnn


def _bonds(blist):
    return [(b.i, b.j, b.t) for b in blist]


def test_square_band_is_the_fourier_transform_of_the_bonds():
    for L1, L2, t, tp in ((4, 4, 1.0, -0.3), (4, 3, 1.0, 0.25), (3, 3, 0.7, 0.0)):
        eps = mk.band_from_bonds(L1, L2, _bonds(torus_nnn(L1, L2, t, tp)))
        np.testing.assert_allclose(eps, mk.square_band(L1, L2, t, tp), atol=1e-13)
    eps = mk.band_from_bonds(8, 1, _bonds(ring(8, 1.0)))
    np.testing.assert_allclose(eps, -2.0 * np.cos(2 * np.pi * np.arange(8) / 8), atol=1e-14)
    with pytest.raises(ValueError):
        mk.band_from_bonds(4, 1, [(0, 1, 1.0)])


def test_momentum_arithmetic_is_a_group():
    L1, L2 = 4, 3
    N = L1 * L2
    for a in range(N):
        assert mk.k_add(a, 0, L1, L2) == a
        assert mk.k_add(a, mk.k_neg(a, L1, L2), L1, L2) == 0
        for b in range(N):
            assert mk.k_add(a, b, L1, L2) == mk.k_add(b, a, L1, L2)
            assert mk.k_sub(mk.k_add(a, b, L1, L2), b, L1, L2) == a


def test_sectors_partition_the_basis():
    L1, L2, nu, nd = 4, 4, 3, 2
    N = L1 * L2
    total = 0
    for K in range(N):
        keys = mk.sector_keys(L1, L2, nu, nd, K)
        up, dn = mk.split_keys(keys, N)
        for u, d in zip(up[::37], dn[::37]):
            assert mk.k_add(mk.string_momentum(u, L1, L2), mk.string_momentum(d, L1, L2), L1, L2) == K
            assert bin(int(u)).count("1") == nu and bin(int(d)).count("1") == nd
        total += len(keys)
    assert total == comb(N, nu) * comb(N, nd)


CASES = [
    # L1, L2, bonds, U, n_up, n_dn
    (6, 1, _bonds(ring(6, 1.0)), 4.0, 3, 3),
    (7, 1, _bonds(ring(7, 1.0)) + [(i, (i + 2) % 7, 0.4) for i in range(7)], 3.0, 3, 2),
    (3, 3, _bonds(torus(3, 3, 1.0)), 5.0, 2, 2),
    (4, 4, _bonds(torus_nnn(4, 4, 1.0, -0.3)), 6.0, 2, 1),
]


@pytest.mark.parametrize("case", CASES, ids=["ring6", "ring7_nnn", "torus3x3", "torus4x4_nnn_2+1"])
def test_union_of_momentum_spectra_is_the_real_space_spectrum(case):
    L1, L2, bonds, U, nu, nd = case
    N = L1 * L2
    eps = mk.band_from_bonds(L1, L2, bonds)
    ev_k = []
    for K in range(N):
        H = mk.build_csr_k(L1, L2, eps, U, nu, nd, K)
        if H.shape[0]:
            assert abs(H - H.T).max() == 0.0
            ev_k.append(np.linalg.eigvalsh(H.toarray()))
    ev_k = np.sort(np.concatenate(ev_k))
    p = oracle.Problem(N, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds], U, nu, nd)
    ev_r = np.linalg.eigvalsh(oracle.build_csr(p).toarray())
    assert len(ev_k) == len(ev_r)
    np.testing.assert_allclose(ev_k, ev_r, atol=1e-10)


def test_U0_sector_is_diagonal_with_band_sums():
    L1, L2 = 4, 3
    eps = mk.square_band(L1, L2, 1.0, 0.2)
    N = L1 * L2
    for K in (0, 5):
        H = mk.build_csr_k(L1, L2, eps, 0.0, 3, 2, K)
        keys = mk.sector_keys(L1, L2, 3, 2, K)
        up, dn = mk.split_keys(keys, N)
        off = H - sp.diags(H.diagonal())
        assert abs(off).max() == 0.0
        want = np.array([sum(eps[i] for i in range(N) if (int(u) >> i) & 1) +
                         sum(eps[i] for i in range(N) if (int(d) >> i) & 1) for u, d in zip(up, dn)])
        np.testing.assert_allclose(H.diagonal(), want, atol=1e-13)


def test_interaction_diagonal_is_U_over_N_times_nup_ndn():
    L1, L2, nu, nd, U = 3, 3, 2, 3, 2.5
    H = mk.build_csr_k(L1, L2, np.zeros(9), U, nu, nd, 4)
    np.testing.assert_allclose(H.diagonal(), U / 9 * nu * nd, atol=1e-14)


@pytest.mark.parametrize("L1,L2,nu,nd", [(4, 4, 3, 2), (6, 1, 3, 3), (4, 3, 2, 4)])
def test_paper_kspace_forward_maps_give_sorted_positions(L1, L2, nu, nd):
    N = L1 * L2
    C = mk.extended_counts(L1, L2, max(nu, nd))
    by_k = mk.strings_by_momentum(L1, L2, nd)
    for k in range(N):   # single spin: counts and ranks within each momentum
        assert C[N][nd][k] == len(by_k[k])
        for pos, phi in enumerate(by_k[k]):
            assert mk.forward_map_k(phi, C, L1, L2) == (pos, k)
    Ct = mk.spinful_counts(C, L1, L2, nd)
    for K in range(N):
        keys = mk.sector_keys(L1, L2, nu, nd, K)
        up, dn = mk.split_keys(keys, N)
        got = [mk.forward_map_k_spin(u, d, C, Ct, L1, L2) for u, d in zip(up, dn)]
        assert got == list(range(len(keys)))
        tot = sum(C[N][nu][ku] * C[N][nd][mk.k_sub(K, ku, L1, L2)] for ku in range(N))
        assert tot == len(keys)


def test_extended_counts_by_brute_force():
    L1, L2 = 3, 2
    N = L1 * L2
    C = mk.extended_counts(L1, L2, 3)
    for i in range(N + 1):
        for m in range(4):
            for k in range(N):
                brute = sum(1 for s in range(1 << i) if bin(s).count("1") == m and mk.string_momentum(s, L1, L2) == k)
                assert C[i][m][k] == brute


def test_hv_rows_match_the_explicit_matrix():
    L1, L2, U = 4, 4, 6.0
    eps = mk.square_band(L1, L2, 1.0, -0.3)
    keys = mk.sector_keys(L1, L2, 2, 2, 0)
    H = mk.build_csr_k(L1, L2, eps, U, 2, 2, 0)
    x = np.random.default_rng(3).uniform(-1, 1, len(keys))
    rows = np.arange(0, len(keys), 7)
    y, a, n = mk.hv_rows_k(L1, L2, eps, U, keys, x, rows)
    np.testing.assert_allclose(y, (H @ x)[rows], atol=1e-12)
    assert np.all(n >= 1)


def test_planted_sign_mistake_is_caught(monkeypatch):
    L1, L2, bonds, U, nu, nd = CASES[0]
    N = L1 * L2
    eps = mk.band_from_bonds(L1, L2, bonds)
    real = oracle.Problem(N, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds], U, nu, nd)
    ev_r = np.linalg.eigvalsh(oracle.build_csr(real).toarray())
    monkeypatch.setattr(mk, "create_sign", lambda up, dn, spin, i: 0 * up)
    ev_k = np.sort(np.concatenate([np.linalg.eigvalsh(mk.build_csr_k(L1, L2, eps, U, nu, nd, K).toarray())
                                   for K in range(N)]))
    assert np.max(np.abs(ev_k - ev_r)) > 1e-3
