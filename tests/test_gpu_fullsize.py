"""Full-size checks of the device Lanczos where no CPU eigensolve finishes in test time.

At U = 0 the many-body ground energy is the sum of the lowest n_up and n_dn
one-particle levels of h_ij = -t_ij (the oracle's one-body matrix, LAPACK
eigvalsh): an exact pin for the benchmark lattices at D = 1.66e8 and 1.31e8.
At U != 0 the particle-hole identity E0(N - n_up, N - n_dn; t) =
E0(n_up, n_dn; -t) + U (N - n_up - n_dn) relates two independent device
solves of the same size.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _device(w, U=None, n=None, flip=False):
    import paper_1707_03974_amd as pdz
    bonds = [synth.Bond(b.i, b.j, -b.t if flip else b.t) for b in w.bonds]
    nu, nd = (n, n) if n is not None else (w.n_up, w.n_dn)
    return pdz.Problem(w.n_sites, bonds, w.U if U is None else U, nu, nd)


def _band_sum(w):
    po = oracle.Problem.from_workload(w)
    lev = np.linalg.eigvalsh(oracle.one_body_matrix(po))
    return float(lev[:w.n_up].sum() + lev[:w.n_dn].sum())


@pytest.mark.parametrize("name,expect", [("torus4x4_nnn", -26.4), ("torus4x4_n7", -24.0)])
def test_full_size_U0_energy_is_the_band_sum(name, expect):
    w = synth.workload(name)
    E = _band_sum(w)
    assert abs(E - expect) < 1e-12
    r = _device(w, U=0.0).lanczos(tol=1e-12, max_iter=600)
    assert r["converged"] == 1
    assert abs(r["E0"] - E) <= 1e-9 * abs(E), (r, E)


def test_full_size_particle_hole_identity():
    w = synth.workload("torus4x4_n7")
    N, U = w.n_sites, w.U
    a = _device(w, n=N - w.n_up).lanczos(tol=1e-12, max_iter=800)
    b = _device(w, flip=True).lanczos(tol=1e-12, max_iter=800)
    assert a["converged"] == 1 and b["converged"] == 1
    expect = b["E0"] + U * (N - w.n_up - w.n_dn)
    assert abs(a["E0"] - expect) <= 1e-9 * abs(expect), (a, b)
