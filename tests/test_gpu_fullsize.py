"""Full-size checks of the device Lanczos (D = 1.66e8 and 1.31e8).

* At U != 0 the ground-state energies of the 4x4 NN+NNN 8+8 (U = 6) and 4x4 NN
  7+7 (U = 5) clusters against the oracle's stored values
  (tests/golden/energies_fullsize.json, written by
  tests/golden/make_energies_fullsize.py from the oracle only): FP64 within
  1e-9 relative, FP32 storage with the self-checking FP64 refinement within
  1e-8, under the launch plan the benchmark's tuning procedure selects.
* At U = 0 the many-body ground energy is the sum of the lowest n_up and n_dn
  one-particle levels of h_ij = -t_ij (the oracle's one-body matrix, LAPACK
  eigvalsh), also under the selected plan.
* The particle-hole identity E0(N - n_up, N - n_dn; t) = E0(n_up, n_dn; -t) +
  U (N - n_up - n_dn) relates two independent device solves of the same size.
"""
import json
import os

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


GOLD = os.path.join(os.path.dirname(__file__), "golden", "energies_fullsize.json")


def _golden(name):
    if not os.path.exists(GOLD):
        pytest.skip("no oracle energies stored yet (tests/golden/make_energies_fullsize.py)")
    with open(GOLD) as f:
        rec = json.load(f)
    if name not in rec:
        pytest.skip(f"no oracle energy stored for {name}")
    return rec[name]["E0"]


def _tuned(g, dtype_name):
    """The plan the benchmark selects: every H.v plan timed, the fastest few timed as Lanczos steps."""
    best, _, _ = g.tune_lanczos(dtype_name, top=3)
    return best


@pytest.mark.parametrize("name", ["torus4x4_nnn", "torus4x4_n7"])
def test_full_size_energy_matches_the_oracle(name):
    w = synth.workload(name)
    E = _golden(name)
    g = _device(w)
    _tuned(g, "f64")
    r = g.lanczos(storage="f64", tol=1e-12, max_iter=600)
    assert r["converged"] == 1
    assert abs(r["E0"] - E) <= 1e-9 * abs(E), (r["E0"], E)
    _tuned(g, "f32")
    r = g.lanczos(storage="f32", tol=1e-7, max_iter=200, refine=2, keep_basis=1)   # kept basis: 201 x 0.66 GB
    assert abs(r["E0_refined"] - E) <= 1e-8 * abs(E), (r, E)


@pytest.mark.parametrize("name,expect", [("torus4x4_nnn", -26.4), ("torus4x4_n7", -24.0)])
def test_full_size_U0_band_sum_under_the_selected_plans(name, expect):
    """The fused Lanczos step (recurrence riding on the down pass) under the tuned plans, FP64 and FP32
    storage with refinement."""
    w = synth.workload(name)
    E = _band_sum(w)
    g = _device(w, U=0.0)
    _tuned(g, "f64")
    r = g.lanczos(storage="f64", tol=1e-12, max_iter=600)
    assert abs(r["E0"] - E) <= 1e-9 * abs(E), (r, E)
    _tuned(g, "f32")
    r = g.lanczos(storage="f32", tol=1e-7, max_iter=200, refine=2, keep_basis=1)   # kept basis: 201 x 0.66 GB
    assert abs(r["E0_refined"] - E) <= 1e-8 * abs(E), (r, E)
