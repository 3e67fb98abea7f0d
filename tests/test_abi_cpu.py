"""C-ABI checks that need no GPU: the library loads, exports every declared
entry point, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_1707_03974_amd as pdz
from paper_1707_03974_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pdz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdz_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_expected_calls():
    names = _declared()
    for n in ["pdz_problem_create", "pdz_problem_destroy", "pdz_problem_info", "pdz_rank", "pdz_unrank",
              "pdz_hv", "pdz_lanczos", "pdz_lanczos_workspace_size", "pdz_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) <= set(_lib.exported_symbols()) | {"pdz_version"}


def test_version():
    assert _lib.load().pdz_version() == 100


def _create(n_sites, bonds, U, n_up, n_dn):
    lib = _lib.load()
    arr = (_lib.Bond * max(1, len(bonds)))(*[_lib.Bond(i, j, t) for i, j, t in bonds])
    h = ctypes.c_void_p()
    st = lib.pdz_problem_create(n_sites, arr if bonds else None, len(bonds), U, n_up, n_dn, ctypes.byref(h))
    return st, lib.pdz_last_error().decode()


@pytest.mark.parametrize("args,code,words", [
    ((0, [], 1.0, 0, 0), _lib.PDZ_ERANGE, "n_sites"),
    ((33, [], 1.0, 1, 1), _lib.PDZ_ERANGE, "n_sites"),
    ((4, [(0, 1, 1.0)], 1.0, 5, 1), _lib.PDZ_EINVAL, "n_up"),
    ((4, [(0, 1, 1.0)], 1.0, 1, -1), _lib.PDZ_EINVAL, "n_up"),
    ((4, [(0, 0, 1.0)], 1.0, 1, 1), _lib.PDZ_EINVAL, "itself"),
    ((4, [(0, 4, 1.0)], 1.0, 1, 1), _lib.PDZ_EINVAL, "outside"),
    ((4, [(-1, 2, 1.0)], 1.0, 1, 1), _lib.PDZ_EINVAL, "outside"),
    ((4, [(0, 1, float("nan"))], 1.0, 1, 1), _lib.PDZ_EINVAL, "non-finite"),
    ((4, [(0, 1, 1.0)], float("inf"), 1, 1), _lib.PDZ_EINVAL, "U"),
])
def test_problem_create_rejects_invalid_input(args, code, words):
    st, msg = _create(*args)
    assert st == code
    assert words in msg


def test_null_arguments_are_rejected():
    lib = _lib.load()
    assert lib.pdz_problem_info(None, None) == _lib.PDZ_EINVAL
    assert lib.pdz_hv(None, 0, None, None, None) == _lib.PDZ_EINVAL
    assert lib.pdz_problem_destroy(None) == _lib.PDZ_OK
    assert lib.pdz_rank(0, 0, None, 0, None, None) == _lib.PDZ_ERANGE
    assert lib.pdz_unrank(8, 9, None, 0, None, None) == _lib.PDZ_EINVAL
    assert lib.pdz_rank(8, 2, None, 5, None, None) == _lib.PDZ_EINVAL
    n = ctypes.c_size_t()
    assert lib.pdz_lanczos_workspace_size(None, None, ctypes.byref(n)) == _lib.PDZ_EINVAL


def test_lanczos_default_options_and_validation():
    lib = _lib.load()
    o = _lib.LanczosOpts()
    assert lib.pdz_lanczos_default_opts(ctypes.byref(o)) == 0
    assert (o.max_iter, o.tol, o.storage, o.reorth, o.seed, o.check_every, o.use_graph, o.refine) == \
        (300, 1e-12, 0, 0, 1, 10, 1, 0)
    res = _lib.LanczosResult()
    # a NULL problem is rejected before the options or any device work
    assert lib.pdz_lanczos(None, ctypes.byref(o), None, None, 0, None, ctypes.byref(res), None) == _lib.PDZ_EINVAL


def test_batch_calls_reject_null_arguments_without_a_device():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.pdz_batch_create(None, 0, ctypes.byref(h)) == _lib.PDZ_EINVAL
    assert lib.pdz_batch_create(None, 2, None) == _lib.PDZ_EINVAL
    assert lib.pdz_batch_destroy(None) == _lib.PDZ_OK
    offs = (ctypes.c_uint64 * 2)()
    assert lib.pdz_batch_offsets(None, offs) == _lib.PDZ_EINVAL
    assert lib.pdz_batch_hv(None, 0, None, None, None) == _lib.PDZ_EINVAL
    pl = _lib.BatchPlan()
    assert lib.pdz_batch_get_plan(None, ctypes.byref(pl)) == _lib.PDZ_EINVAL
    assert lib.pdz_batch_set_plan(None, ctypes.byref(pl)) == _lib.PDZ_EINVAL
    o = _lib.LanczosOpts()
    lib.pdz_lanczos_default_opts(ctypes.byref(o))
    n = ctypes.c_size_t()
    assert lib.pdz_batch_lanczos_workspace_size(None, ctypes.byref(o), ctypes.byref(n)) == _lib.PDZ_EINVAL
    res = (_lib.LanczosResult * 1)()
    assert lib.pdz_batch_lanczos(None, ctypes.byref(o), None, 0, res, None) == _lib.PDZ_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    """No CPU fallback: without the built HIP library the binding raises."""
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError, match="no fallback"):
        _lib.load(os.path.join(ROOT, "does_not_exist", "libpdz.so"))


def _decide(alpha, beta, E, resid):
    lib = _lib.load()
    k = len(alpha)
    a = (ctypes.c_double * k)(*alpha)
    b = (ctypes.c_double * (k + 1))(*beta)
    rs = ctypes.c_int32()
    gap = ctypes.c_double()
    assert lib.pdz_refine_decision(a, b, k, E, resid, ctypes.byref(rs), ctypes.byref(gap)) == _lib.PDZ_OK
    return rs.value, gap.value


def test_refine_decision_skips_copies_of_the_lowest_ritz_value():
    """A duplicated lowest Ritz value (a ghost or a degenerate level) must not read as a zero gap."""
    # T_k = diag(-2, -2, 1, 3) with tiny couplings: theta_1 = -2 twice, next distinct value 1
    alpha = [-2.0, -2.0, 1.0, 3.0]
    beta = [0.0, 1e-13, 1e-13, 1e-13, 0.5]
    restart, gap = _decide(alpha, beta, -2.0, 1e-6)
    assert abs(gap - 0.3) < 1e-9          # (1 - (-2)) / 10
    assert restart == 0                    # 1e-12 / 0.3 < 1e-8 * 2
    restart, _ = _decide(alpha, beta, -2.0, 1e-3)
    assert restart == 1                    # 1e-6 / 0.3 > 2e-8


def test_refine_decision_restarts_when_the_gap_is_unknown():
    # every Ritz value in one cluster: no distinct second value
    restart, gap = _decide([-1.0, -1.0], [0.0, 0.0, 0.0], -1.0, 1e-12)
    assert restart == 1 and gap == 0.0
    # a single step
    restart, gap = _decide([-1.0], [0.0, 0.1], -1.0, 1e-12)
    assert restart == 1


def test_refine_decision_matches_the_bound_on_a_clear_gap():
    # T = [[0, 1], [1, 0]]: Ritz values -1, 1; gap estimate 0.2
    restart, gap = _decide([0.0, 0.0], [0.0, 1.0, 0.0], -1.0, 1e-5)
    assert abs(gap - 0.2) < 1e-9 and restart == 0          # 1e-10 / 0.2 <= 1e-8
    restart, _ = _decide([0.0, 0.0], [0.0, 1.0, 0.0], -1.0, 1e-4)
    assert restart == 1                                      # 1e-8 / 0.2 > 1e-8
    with pytest.raises(AssertionError):
        _decide([], [0.0], -1.0, 0.0)
