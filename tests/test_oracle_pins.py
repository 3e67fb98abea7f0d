"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a
printed example of the paper (tests/golden/), a closed form, an independent
construction (Jordan-Wigner matrices, brute-force counting), or a library
routine (LAPACK dense eigensolver, ARPACK).
"""
import json
import math
import os
from itertools import permutations

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import (Problem, build_csr, hv_rows, lanczos, nnz_structural, sector_list,
                    index_in_sorted, start_vector, splitmix64_outputs, one_body_matrix)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _prob(n_sites, bonds, U, n_up, n_dn):
    return Problem(n_sites, [b[0] for b in bonds], [b[1] for b in bonds],
                   [float(b[2]) for b in bonds], float(U), n_up, n_dn)


def _E0_dense(p):
    H = build_csr(p).toarray()
    return float(np.linalg.eigvalsh(H)[0])


# ---------------------------------------------------------------- paper examples

def test_sector_tables_4site():
    g = _gold("paper_examples.json")["sector_tables_4site"]
    assert list(sector_list(4, 2)) == g["n2"]
    assert list(sector_list(4, 3)) == g["n3"]


def test_forward_map_example():
    g = _gold("paper_examples.json")["forward_map_example"]
    lst = sector_list(g["N"], g["n"])
    assert int(index_in_sorted(lst, [g["phi"]])[0]) == g["idx"]


def test_simple_neighbour_distance_example():
    g = _gold("paper_examples.json")["simple_neighbour_example"]
    lst = sector_list(g["N"], g["n"])
    p1 = sum(1 << b for b in g["phi1_bits"])
    p2 = sum(1 << b for b in g["phi2_bits"])
    i1, i2 = index_in_sorted(lst, [p1, p2])
    assert int(i2 - i1) == g["dist"]
    assert g["dist"] == math.comb(9, 4) - math.comb(6, 4)


def test_composite_index_and_dimension_example():
    g = _gold("paper_examples.json")["composite_index_example"]
    e = _gold("paper_examples.json")["basis_element_4site"]
    up, dn = sector_list(g["N"], g["n_up"]), sector_list(g["N"], g["n_dn"])
    assert len(up) * len(dn) == e["D"]
    keys = oracle.composite_keys(up, dn, g["N"])
    key = (g["phi_up"] << g["N"]) | g["phi_dn"]
    assert int(index_in_sorted(keys, [key])[0]) == g["idx"]


def test_up_hopping_example_signs():
    g = _gold("paper_examples.json")["up_hopping_example"]
    t = 1.0
    p = _prob(g["N"], [(a, b, t) for a, b in g["ring_bonds"]], 0.0, g["n_up"], g["n_dn"])
    H = build_csr(p).toarray()
    up, dn = p.up_list, p.dn_list
    Ddn = len(dn)
    iu = int(index_in_sorted(up, [g["source_up"]])[0])
    idn = int(index_in_sorted(dn, [g["source_dn"]])[0])
    src = iu * Ddn + idn
    expect = {}
    for tu, c in zip(g["targets_up"], g["coeff_over_minus_t"]):
        expect[int(index_in_sorted(up, [tu])[0]) * Ddn + idn] = -t * c
    # entries of column src whose down part is unchanged come from up hops only
    for r in range(p.D):
        if r % Ddn != idn or r == src:
            continue
        assert H[r, src] == expect.get(r, 0.0), r


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("N", [1, 3, 6, 9, 12])
def test_sector_list_is_every_popcount_state_ascending(N):
    allx = np.arange(1 << N, dtype=np.uint64)
    pc = np.bitwise_count(allx)
    for n in range(N + 1):
        lst = sector_list(N, n)
        assert np.array_equal(lst, allx[pc == n])
        assert len(lst) == math.comb(N, n)


@pytest.mark.parametrize("N", [5, 8, 11])
def test_index_equals_count_of_smaller_states(N):
    allx = np.arange(1 << N)
    pc = np.array([bin(v).count("1") for v in allx])
    for n in range(N + 1):
        lst = sector_list(N, n)
        idx = index_in_sorted(lst, lst)
        brute = [int(np.count_nonzero((allx < v) & (pc == n))) for v in lst]
        assert list(idx) == brute


@pytest.mark.parametrize("N", [4, 7, 10])
def test_count_below_matches_brute_force(N):
    for n in range(N + 1):
        for x in range(1 << N):
            assert oracle.count_below(x, n) == sum(1 for y in range(x) if bin(y).count("1") == n)


# ---------------------------------------------------------------- Jordan-Wigner

def _jw_ops(n_modes):
    a = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))   # annihilation on (|0>, |1>)
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    I = sp.identity(2, format="csr")
    ops = []
    for m in range(n_modes):
        mats = [Z] * m + [a] + [I] * (n_modes - m - 1)
        op = mats[0]
        for M in mats[1:]:
            op = sp.kron(op, M, format="csr")
        ops.append(op)
    return ops


def _jw_projected_H(n_sites, bonds, U, n_up, n_dn):
    """H of Eq. (1) built from Jordan-Wigner matrices, projected on the paper's basis.

    Mode index: up site i -> i, down site i -> n_sites + i.  Basis vectors are
    made by applying creation matrices to the vacuum in the order the paper
    writes them: up operators (descending site) left of down operators
    (descending site).
    """
    M = 2 * n_sites
    c = _jw_ops(M)
    cd = [op.T.tocsr() for op in c]
    n = [cd[m] @ c[m] for m in range(M)]
    dim = 1 << M
    H = sp.csr_matrix((dim, dim))
    for (i, j, t) in bonds:
        for s in (0, n_sites):
            H = H - t * (cd[i + s] @ c[j + s] + cd[j + s] @ c[i + s])
    for i in range(n_sites):
        H = H + U * (n[i] @ n[i + n_sites])
    vac = np.zeros(dim)
    vac[0] = 1.0
    up, dn = sector_list(n_sites, n_up), sector_list(n_sites, n_dn)
    vecs = []
    for pu in up:
        for pd in dn:
            v = vac.copy()
            # rightmost operator acts first: down block, ascending site, then up block ascending
            for i in range(n_sites):
                if (int(pd) >> i) & 1:
                    v = cd[i + n_sites] @ v
            for i in range(n_sites):
                if (int(pu) >> i) & 1:
                    v = cd[i] @ v
            vecs.append(v)
    B = np.array(vecs).T
    return B.T @ (H @ B)


@pytest.mark.parametrize("case", [
    (4, [(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (3, 0, 1.0)], 2.5, 2, 3),
    (4, [(0, 2, 0.7), (1, 3, -1.3), (0, 3, 0.4), (2, 1, 1.1)], 1.5, 2, 2),
    (5, [(0, 4, 1.0), (1, 3, 0.6), (2, 0, -0.9), (3, 4, 0.3), (1, 2, 0.8)], 3.0, 2, 3),
    (5, [(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (3, 4, 1.0), (4, 0, 1.0), (0, 2, -0.3)], 4.0, 3, 1),
])
def test_hamiltonian_equals_jordan_wigner(case):
    n_sites, bonds, U, n_up, n_dn = case
    p = _prob(n_sites, bonds, U, n_up, n_dn)
    H = build_csr(p).toarray()
    Hjw = _jw_projected_H(n_sites, bonds, U, n_up, n_dn)
    assert np.array_equal(H, Hjw)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("U,t", [(4.0, 1.0), (0.0, 1.0), (8.0, 0.5), (1.0, 2.0)])
def test_two_site_ground_state(U, t):
    p = _prob(2, [(0, 1, t)], U, 1, 1)
    E = (U - math.sqrt(U * U + 16 * t * t)) / 2
    assert abs(_E0_dense(p) - E) <= 1e-13 * max(1, abs(E))
    r = lanczos(lambda x: build_csr(p) @ x, start_vector(5, p.D))
    assert abs(r.E0 - E) <= 1e-12 * max(1, abs(E))


@pytest.mark.parametrize("n_up,n_dn", [(2, 2), (4, 3), (5, 5), (0, 6)])
def test_atomic_limit(n_up, n_dn):
    N, U = 6, 3.5
    p = _prob(N, [(i, (i + 1) % N, 0.0) for i in range(N)], U, n_up, n_dn)
    assert _E0_dense(p) == U * max(0, n_up + n_dn - N)


def test_U0_ring8_closed_form():
    w = synth.workload("ring8")
    p = Problem.from_workload(w)
    p.U = 0.0
    r = lanczos(lambda x, H=build_csr(p): H @ x, start_vector(1, p.D))
    assert abs(r.E0 - (-4 - 4 * math.sqrt(2))) < 1e-11


def _eps_k(Lx, Ly, t, tp):
    out = []
    for a in range(Lx):
        for b in range(Ly):
            kx, ky = 2 * math.pi * a / Lx, 2 * math.pi * b / Ly
            out.append(-2 * t * (math.cos(kx) + math.cos(ky)) - 4 * tp * math.cos(kx) * math.cos(ky))
    return sorted(out)


@pytest.mark.parametrize("Lx,Ly,tp", [(4, 4, -0.3), (4, 4, 0.0), (4, 3, 0.0), (3, 3, 0.2)])
def test_one_body_spectrum_is_band_structure(Lx, Ly, tp):
    """U = 0 single-particle levels are eps_k of Sec. IV.A (NNN term only when both Lx, Ly > 2)."""
    bonds = synth.torus_nnn(Lx, Ly, 1.0, tp) if tp != 0.0 else synth.torus(Lx, Ly, 1.0)
    p = _prob(Lx * Ly, [(b.i, b.j, b.t) for b in bonds], 0.0, 1, 0)
    ev = np.linalg.eigvalsh(one_body_matrix(p))
    assert np.allclose(sorted(ev), _eps_k(Lx, Ly, 1.0, tp), atol=1e-12)


def test_U0_torus4x3_many_body_is_sum_of_band_levels():
    w = synth.workload("torus4x3")
    p = Problem.from_workload(w)
    p.U = 0.0
    lev = _eps_k(4, 3, 1.0, 0.0)
    expect = sum(lev[:6]) * 2
    assert abs(expect - (-20.0)) < 1e-12
    H = build_csr(p)
    E = spla.eigsh(H, k=1, which="SA", tol=1e-12)[0][0]
    assert abs(E - expect) < 1e-9


def test_U0_small_open_shell_sum_of_levels():
    # 3x3 torus, 2+3 electrons, U=0, t'=0.2: E0 = lowest 2 + lowest 3 band levels
    bonds = synth.torus_nnn(3, 3, 1.0, 0.2)
    p = _prob(9, [(b.i, b.j, b.t) for b in bonds], 0.0, 2, 3)
    lev = _eps_k(3, 3, 1.0, 0.2)
    assert abs(_E0_dense(p) - (sum(lev[:2]) + sum(lev[:3]))) < 1e-11


@pytest.mark.parametrize("name", ["ring8", "torus4x3"])
def test_trace_frobenius_nnz_closed_forms(name):
    p = Problem.from_workload(synth.workload(name))
    N, nu, nd = p.n_sites, p.n_up, p.n_dn
    Du, Dd = math.comb(N, nu), math.comb(N, nd)
    H = build_csr(p)
    B = len(p.bond_i)
    assert H.nnz == nnz_structural(p) == Du * Dd + 2 * B * math.comb(N - 2, nu - 1) * Dd + 2 * B * math.comb(N - 2, nd - 1) * Du
    assert abs(H.diagonal().sum() - p.U * N * math.comb(N - 1, nu - 1) * math.comb(N - 1, nd - 1)) < 1e-6
    off = H - sp.diags(H.diagonal())
    fro2 = 2 * sum(t * t for t in p.bond_t) * (math.comb(N - 2, nu - 1) * Dd + math.comb(N - 2, nd - 1) * Du)
    assert abs(off.multiply(off).sum() - fro2) < 1e-6
    assert (H - H.T).count_nonzero() == 0


# ---------------------------------------------------------------- identities

def test_particle_hole_and_spin_swap():
    bonds = [(b.i, b.j, b.t) for b in synth.torus_nnn(3, 3, 1.0, -0.3)]
    neg = [(i, j, -t) for i, j, t in bonds]
    N, U = 9, 2.7
    for nu, nd in [(2, 3), (4, 1), (3, 3)]:
        E = _E0_dense(_prob(N, bonds, U, nu, nd))
        Eh = _E0_dense(_prob(N, neg, U, N - nu, N - nd))
        assert abs(Eh - (E + U * (N - nu - nd))) < 1e-10
        assert abs(_E0_dense(_prob(N, bonds, U, nd, nu)) - E) < 1e-10


def test_site_relabelling_invariance():
    bonds = [(0, 1, 1.0), (1, 2, 0.5), (2, 3, 1.0), (3, 4, -0.7), (4, 0, 1.0), (1, 3, 0.3)]
    E = _E0_dense(_prob(5, bonds, 3.0, 2, 2))
    for perm in list(permutations(range(5)))[::17]:
        pb = [(perm[i], perm[j], t) for i, j, t in bonds]
        assert abs(_E0_dense(_prob(5, pb, 3.0, 2, 2)) - E) < 1e-11


# ---------------------------------------------------------------- eigensolvers

def test_lanczos_matches_dense_eigensolver_ring8():
    p = Problem.from_workload(synth.workload("ring8"))
    H = build_csr(p)
    E = float(np.linalg.eigvalsh(H.toarray())[0])
    r = lanczos(lambda x: H @ x, start_vector(1, p.D), tol=1e-13)
    assert r.converged and abs(r.E0 - E) <= 1e-12 * abs(E)


def test_lanczos_tridiagonal_solver_matches_dense():
    p = Problem.from_workload(synth.workload("ring8"))
    H = build_csr(p)
    r = lanczos(lambda x: H @ x, start_vector(2, p.D), max_iter=30, tol=0.0)
    T = np.diag(r.alphas) + np.diag(r.betas[:-1], 1) + np.diag(r.betas[:-1], -1)
    assert abs(np.linalg.eigvalsh(T)[0] - r.thetas[-1]) < 1e-12


def test_lanczos_matches_arpack_torus4x3():
    p = Problem.from_workload(synth.workload("torus4x3"))
    H = build_csr(p)
    Ea = float(spla.eigsh(H, k=1, which="SA", tol=1e-13)[0][0])
    r = lanczos(lambda x: H @ x, start_vector(1, p.D), max_iter=300, tol=1e-12)
    assert r.converged and abs(r.E0 - Ea) <= 1e-9 * abs(Ea)


def test_lanczos_breakdown_is_exact():
    # diagonal H (t = 0) and a unit start vector: invariant Krylov space of size 1
    p = _prob(4, [(0, 1, 0.0), (1, 2, 0.0)], 2.0, 2, 2)
    H = build_csr(p)
    v0 = np.zeros(p.D)
    v0[7] = 1.0
    r = lanczos(lambda x: H @ x, v0)
    assert r.converged and r.iters == 1 and r.E0 == H[7, 7]


# ---------------------------------------------------------------- matrix-free paths

def test_row_oracle_and_c_oracle_match_csr():
    from oracle.cmf import MatrixFree
    for name in ["ring8", "torus4x3"]:
        p = Problem.from_workload(synth.workload(name))
        H = build_csr(p)
        x = synth.random_vector(p.D, 11)
        y = H @ x
        rows = np.unique(np.random.default_rng(0).integers(0, p.D, 500))
        assert np.allclose(hv_rows(p, x, rows), y[rows], rtol=0, atol=1e-12)
        assert np.allclose(MatrixFree(p)(x), y, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- SplitMix64

def test_splitmix64_published_outputs():
    g = _gold("splitmix64.json")
    assert [hex(v) for v in splitmix64_outputs(g["seed"], 3)] == [hex(int(h, 16)) for h in g["outputs_hex"]]


def test_start_vector_is_counter_form_of_sequence():
    seq = splitmix64_outputs(12345, 40)
    v = start_vector(12345, 40)
    for k, z in enumerate(seq):
        assert v[k] == 2.0 * ((z >> 11) * 2.0 ** -53) - 1.0


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_planted_sign_mistake(monkeypatch):
    """Dropping the cross-spin operator count must break the Jordan-Wigner pin."""
    import oracle.fock as fk
    orig = fk.annihilate_sign

    def wrong(phi_up, phi_dn, spin, j):
        c = orig(phi_up, phi_dn, spin, j)
        return c + (1 if spin == 1 else 0)     # extra sign on every down annihilation
    monkeypatch.setattr(fk, "annihilate_sign", wrong)
    case = (4, [(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (3, 0, 1.0)], 2.5, 2, 3)
    p = _prob(case[0], case[1], case[2], case[3], case[4])
    assert not np.array_equal(build_csr(p).toarray(), _jw_projected_H(*case))


def test_pins_catch_planted_missing_annihilation_sign(monkeypatch):
    """Forgetting the operators passed by the annihilator must break the paper's hop example.

    (Counting from the other end of the string instead would not be a mistake:
    for a same-spin pair the two counts have the same parity.)
    """
    import oracle.fock as fk
    monkeypatch.setattr(fk, "annihilate_sign", lambda phi_up, phi_dn, spin, j: 0)
    with pytest.raises(AssertionError):
        test_up_hopping_example_signs()


def test_pins_catch_planted_index_transpose():
    """Composite index with the spins swapped must break the paper's example."""
    g = _gold("paper_examples.json")["composite_index_example"]
    up, dn = sector_list(g["N"], g["n_up"]), sector_list(g["N"], g["n_dn"])
    iu = int(index_in_sorted(up, [g["phi_up"]])[0])
    idn = int(index_in_sorted(dn, [g["phi_dn"]])[0])
    assert len(dn) * iu + idn == g["idx"]
    assert len(up) * idn + iu != g["idx"]
