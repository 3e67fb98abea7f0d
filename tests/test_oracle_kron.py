"""The oracle's tensor-product H.v (oracle.kron, used for the stored full-size
energies) against the element-wise oracle (explicit CSR, binary search per
nonzero) and the matrix-free C oracle.

* equal to the CSR product (within FP64 rounding) on the named small
  workloads, random bond lists (repeated pairs, empty sectors, full sectors);
* the per-spin matrices do not depend on the other spin's string that is held
  fixed while they are assembled (the reading that no hop carries a sign from
  the other spin, checked, not assumed);
* whole rows at full size (4x4 NN+NNN, 8+8) equal the C oracle's rows;
* a planted sign mistake in the operator algebra is caught.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import fock
from oracle.kron import KronH, spin_matrix


def _rand_problem(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 9))
    bonds = []
    for _ in range(int(rng.integers(0, 2 * N + 1))):
        i, j = rng.choice(N, 2, replace=False)
        bonds.append((int(i), int(j), float(np.round(rng.uniform(-1.5, 1.5), 3))))
    if bonds and rng.random() < 0.5:
        bonds.append(bonds[0])
    return oracle.Problem(N, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds],
                          float(np.round(rng.uniform(-2, 8), 3)), int(rng.integers(0, N + 1)),
                          int(rng.integers(0, N + 1)))


@pytest.mark.parametrize("name", ["two_site", "ring8", "torus4x3"])
def test_kron_equals_csr_on_named_workloads(name):
    p = oracle.Problem.from_workload(synth.workload(name))
    H = oracle.build_csr(p)
    x = synth.random_vector(p.D, 3)
    y = KronH(p, nthreads=4)(x)
    assert np.max(np.abs(y - H @ x)) <= 1e-12 * max(1.0, np.max(np.abs(H @ x)))


@pytest.mark.parametrize("seed", range(12))
def test_kron_equals_csr_on_random_problems(seed):
    p = _rand_problem(seed)
    H = oracle.build_csr(p)
    x = synth.random_vector(p.D, seed)
    y = KronH(p, nthreads=2)(x)
    assert np.max(np.abs(y - H @ x), initial=0.0) <= 1e-12


@pytest.mark.parametrize("nu,nd", [(3, 2), (2, 4), (4, 4)])
def test_spin_matrices_do_not_depend_on_the_other_spin(nu, nd):
    w = synth.workload("ring8")
    p = oracle.Problem(8, [b.i for b in w.bonds], [b.j for b in w.bonds], [b.t for b in w.bonds], 4.0, nu, nd)
    for spin, other in ((0, p.dn_list), (1, p.up_list)):
        ref = spin_matrix(p, spin, int(other[0])).toarray()
        for partner in other[1::7]:
            assert np.array_equal(spin_matrix(p, spin, int(partner)).toarray(), ref)


def test_full_size_rows_equal_the_c_oracle():
    from oracle.cmf import MatrixFree
    p = oracle.Problem.from_workload(synth.workload("torus4x4_nnn"))
    K = KronH(p, nthreads=4)
    x = np.random.default_rng(11).uniform(-1.0, 1.0, p.D)
    X = x.reshape(K.Du, K.Dd)
    mf = MatrixFree(p)
    for u0 in (0, 4321, K.Du - 1):
        yk = K.rows(X, u0, u0 + 1).reshape(-1)
        ye = mf.rows(x, u0 * K.Dd, (u0 + 1) * K.Dd)
        assert np.max(np.abs(yk - ye)) <= 1e-12


def test_planted_sign_mistake_is_caught(monkeypatch):
    p = oracle.Problem.from_workload(synth.workload("ring8"))
    H = oracle.build_csr(p)
    x = synth.random_vector(p.D, 5)
    real = fock.create_sign
    monkeypatch.setattr(fock, "create_sign", lambda u, d, s, i: real(u, d, s, i) + (1 if i == 3 else 0))
    import oracle.kron as kr
    monkeypatch.setattr(kr, "apply_hop_vec", fock.apply_hop_vec)
    y = KronH(p, nthreads=2)(x)
    assert np.max(np.abs(y - H @ x)) > 1e-3
