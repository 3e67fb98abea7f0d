"""Host-side checks of the momentum-space entry points (no GPU): the band
energies of pdz_kspace_band against the oracle's Fourier transform and the
square-lattice closed form, and argument validation before any device work."""
import ctypes

import numpy as np
import pytest

import paper_1707_03974_amd as pdz
from paper_1707_03974_amd import _lib
from oracle import momentum as mk
from synth.lattices import ring, torus, torus_nnn


@pytest.mark.parametrize("L1,L2,bonds", [
    (4, 4, torus_nnn(4, 4, 1.0, -0.3)),
    (4, 3, torus(4, 3, 1.0)),
    (8, 1, ring(8, 1.0)),
    (3, 3, torus_nnn(3, 3, 0.8, 0.35)),
])
def test_band_matches_the_oracle(L1, L2, bonds):
    got = np.array(pdz.kspace_band(L1, L2, bonds))
    want = mk.band_from_bonds(L1, L2, [(b.i, b.j, b.t) for b in bonds])
    np.testing.assert_allclose(got, want, atol=1e-13)


def test_band_of_the_square_lattice_is_the_closed_form():
    got = np.array(pdz.kspace_band(4, 4, torus_nnn(4, 4, 1.0, -0.3)))
    np.testing.assert_allclose(got, mk.square_band(4, 4, 1.0, -0.3), atol=1e-13)


def test_band_rejects_a_lattice_without_translation_symmetry():
    with pytest.raises(_lib.PdzError):
        pdz.kspace_band(4, 1, [(0, 1, 1.0)])
    with pytest.raises(_lib.PdzError):
        pdz.kspace_band(4, 1, [(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (3, 0, 0.5)])


def test_create_validates_before_touching_a_device():
    lib = _lib.load()
    h = ctypes.c_void_p()
    eps = (ctypes.c_double * 16)(*([0.0] * 16))
    assert lib.pdz_kspace_problem_create(4, 4, None, 1.0, 2, 2, 0, ctypes.byref(h)) == _lib.PDZ_EINVAL
    assert lib.pdz_kspace_problem_create(0, 4, eps, 1.0, 2, 2, 0, ctypes.byref(h)) == _lib.PDZ_ERANGE
    assert lib.pdz_kspace_problem_create(8, 8, eps, 1.0, 2, 2, 0, ctypes.byref(h)) == _lib.PDZ_ERANGE
    assert lib.pdz_kspace_problem_create(4, 4, eps, 1.0, 17, 2, 0, ctypes.byref(h)) == _lib.PDZ_EINVAL
    assert lib.pdz_kspace_problem_create(4, 4, eps, 1.0, 2, 2, 16, ctypes.byref(h)) == _lib.PDZ_EINVAL
    assert lib.pdz_kspace_problem_create(4, 4, eps, float("nan"), 2, 2, 0, ctypes.byref(h)) == _lib.PDZ_EINVAL
    bad = (ctypes.c_double * 16)(*([0.0] * 15 + [float("inf")]))
    assert lib.pdz_kspace_problem_create(4, 4, bad, 1.0, 2, 2, 0, ctypes.byref(h)) == _lib.PDZ_EINVAL
    assert lib.pdz_kspace_rank(None, None, None, 0, None, None) == _lib.PDZ_EINVAL
    assert lib.pdz_kspace_unrank(None, None, 0, None, None, None) == _lib.PDZ_EINVAL
    assert lib.pdz_kspace_info(None, None, None, None, None, None, None) == _lib.PDZ_EINVAL
