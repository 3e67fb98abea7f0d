"""Host side of the dynamical correlations: the continued fraction (libpdz host code) against a
direct solve with the tridiagonal matrix it encodes; argument checks that need no GPU."""
import ctypes

import numpy as np
import pytest

import paper_1707_03974_amd as pdz
from paper_1707_03974_amd import _lib


def test_continued_fraction_equals_the_tridiagonal_resolvent():
    rng = np.random.default_rng(3)
    n = 25
    alpha = rng.normal(0.0, 2.0, n)
    beta = np.concatenate([[0.0], np.abs(rng.normal(1.0, 0.3, n))])   # beta[0] unused, beta[n] not part of T
    T = np.diag(alpha) + np.diag(beta[1:n], 1) + np.diag(beta[1:n], -1)
    w = np.array([0.5 + 0.1j, -3.0 + 0.02j, 7.5 - 0.4j, 1e3 + 0j])
    norm2 = 2.7
    got = pdz.continued_fraction(alpha, beta, norm2, w)
    e0 = np.zeros(n)
    e0[0] = 1.0
    for k, wk in enumerate(w):
        direct = norm2 * np.linalg.solve(wk * np.eye(n) - T, e0.astype(np.complex128))[0]
        assert abs(got[k] - direct) <= 1e-11 * abs(direct), (wk, got[k], direct)


def test_single_level_fraction():
    g = pdz.continued_fraction([1.5], [0.0, 9.9], 2.0, [4.0 + 0j])
    assert np.allclose(g, 2.0 / 2.5)


def test_argument_checks_without_a_gpu():
    L = _lib.load()
    d = (ctypes.c_double * 2)()
    assert L.pdz_continued_fraction(d, d, 0, 1.0, d, d, 1, d, d) == _lib.PDZ_EINVAL
    assert L.pdz_continued_fraction(None, d, 1, 1.0, d, d, 1, d, d) == _lib.PDZ_EINVAL
    assert L.pdz_fermion_op(None, None, 0, 0, 0, 0, None, None, None) == _lib.PDZ_EINVAL
