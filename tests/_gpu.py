"""Helpers for the GPU parity tests (device transfers, tolerance bounds)."""
import numpy as np

EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("these tests need a HIP device")
    return torch


def to_dev(a, dtype):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    return t.detach().cpu().numpy()


def hv_error_bound(H, x, eps):
    """Per-row bound for a floating-point sum of the row's terms in any order.

    |fl(sum) - sum| <= (n + 2) eps sum|a_k x_k|: n - 1 roundings of the
    running sum, one per product, one for rounding x to the working
    precision, one for the coefficient (t' is not exact in FP32).  The FP64
    oracle's own error (n eps64 sum|.|) is added.
    """
    import scipy.sparse as sp
    A = abs(H)
    s = A @ abs(x)
    n = np.diff(H.indptr)
    return (n + 2) * eps * s + n * EPS64 * s


def rows_error_bound(terms_abs_sum, nterms, eps):
    return (nterms + 2) * eps * terms_abs_sum + nterms * EPS64 * terms_abs_sum
