"""ctypes wrapper of the plain-C matrix-free oracle (oracle/c/hv_bsearch.c).

Used where the explicit sparse H would not fit in host memory, and for the
CPU baseline timing.  Built with gcc/OpenMP by oracle.build.
"""
import ctypes
import os

import numpy as np

from .build import build_oracle, library_path

_lib = None


def load(build_if_missing: bool = True):
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        if not build_if_missing:
            raise FileNotFoundError(path)
        build_oracle()
    lib = ctypes.CDLL(path)
    f = lib.oracle_hv_rows
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    _lib = lib
    return lib


class MatrixFree:
    """Row-range H.v of one problem, sector lists held as uint32 arrays."""

    def __init__(self, p, nthreads: int = 0):
        self.p = p
        self.bi = np.ascontiguousarray(p.bond_i, dtype=np.int32)
        self.bj = np.ascontiguousarray(p.bond_j, dtype=np.int32)
        self.bt = np.ascontiguousarray(p.bond_t, dtype=np.float64)
        self.up = np.ascontiguousarray(p.up_list.astype(np.uint32))
        self.dn = np.ascontiguousarray(p.dn_list.astype(np.uint32))
        self.D = len(self.up) * len(self.dn)
        self.nthreads = nthreads or (os.cpu_count() or 1)
        self.lib = load()

    def rows(self, x: np.ndarray, r0: int, r1: int) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.D,) and 0 <= r0 <= r1 <= self.D
        y = np.empty(r1 - r0, dtype=np.float64)
        rc = self.lib.oracle_hv_rows(len(self.bi), self.bi.ctypes.data, self.bj.ctypes.data,
                                     self.bt.ctypes.data, float(self.p.U),
                                     self.up.ctypes.data, len(self.up), self.dn.ctypes.data, len(self.dn),
                                     x.ctypes.data, y.ctypes.data, r0, r1, self.nthreads)
        if rc != 0:
            raise RuntimeError("oracle matrix-free H.v found an inconsistent state")
        return y

    def __call__(self, x: np.ndarray) -> np.ndarray:
        return self.rows(x, 0, self.D)
