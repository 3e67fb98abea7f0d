"""pdz_dot_noalloc (partial sums in the library's fixed device array, result in
device memory) against pdz_dot, the entry point it is a variant of: two calls
in a row, the second on a smaller input, each bitwise equal to pdz_dot's
result on the same inputs (same kernels, same fixed reduction order), and
within FP64 rounding of the plain sum."""
import ctypes

import numpy as np
import pytest

from tests._gpu import torch_cuda, to_dev

pytestmark = pytest.mark.gpu


def _dot(lib, code, a, b, n):
    r = ctypes.c_double()
    from paper_1707_03974_amd import _lib
    _lib.check(lib.pdz_dot(code, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, ctypes.byref(r),
                           None))
    return r.value


def _dot_noalloc(torch, lib, code, a, b, n):
    from paper_1707_03974_amd import _lib
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    _lib.check(lib.pdz_dot_noalloc(code, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n,
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream)))
    torch.cuda.synchronize()
    return float(out.cpu()[0])


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_dot_noalloc_equals_pdz_dot_on_two_calls(dtype_name):
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    lib = pdz.lib()
    code = pdz.PDZ_F64 if dtype_name == "f64" else pdz.PDZ_F32
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    rng = np.random.default_rng(17)
    for n in (3_000_017, 777):          # the second call is smaller: no stale partial sum may leak in
        a = rng.uniform(-1, 1, n)
        b = rng.uniform(-1, 1, n)
        if dtype_name == "f32":
            a, b = a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
        ad, bd = to_dev(a, dt), to_dev(b, dt)
        ref = _dot(lib, code, ad, bd, n)
        got = _dot_noalloc(torch, lib, code, ad, bd, n)
        assert got == ref, (n, got, ref)
        exact = float(np.dot(a, b))
        assert abs(got - exact) <= n * 2.0 ** -52 * float(np.dot(np.abs(a), np.abs(b))), (n, got, exact)


def test_dot_noalloc_rejects_bad_arguments():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    from paper_1707_03974_amd import _lib
    lib = pdz.lib()
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert lib.pdz_dot_noalloc(pdz.PDZ_F64, None, ctypes.c_void_p(x.data_ptr()), 4, ctypes.c_void_p(x.data_ptr()),
                               None) == _lib.PDZ_EINVAL
    assert lib.pdz_dot_noalloc(7, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 4,
                               ctypes.c_void_p(x.data_ptr()), None) == _lib.PDZ_EINVAL
