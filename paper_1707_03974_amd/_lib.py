"""ctypes binding of libpdz.so: argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts
Python arguments and torch device tensors into the pointers and sizes of the
C ABI declared in include/pdz.h, and turns failing status codes into
PdzError.  It refuses to run without the compiled library.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdz.so")

PDZ_OK = 0
PDZ_EINVAL = -1
PDZ_ERANGE = -2
PDZ_ENOMEM = -3
PDZ_EHIP = -4
PDZ_ENOCONV = -5
PDZ_EDEVICE = -6
STATUS_NAMES = {0: "PDZ_OK", -1: "PDZ_EINVAL", -2: "PDZ_ERANGE", -3: "PDZ_ENOMEM", -4: "PDZ_EHIP",
                -5: "PDZ_ENOCONV", -6: "PDZ_EDEVICE"}

PDZ_F64 = 0
PDZ_F32 = 1


class PdzError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class Bond(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32), ("t", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("D", ctypes.c_uint64), ("D_up", ctypes.c_uint64), ("D_dn", ctypes.c_uint64),
                ("nnz", ctypes.c_uint64), ("hops_up", ctypes.c_uint64), ("hops_dn", ctypes.c_uint64),
                ("n_sites", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
                ("n_bonds", ctypes.c_int32), ("max_hops_up", ctypes.c_int32), ("max_hops_dn", ctypes.c_int32),
                ("device", ctypes.c_int32), ("hv_path", ctypes.c_int32)]


class LanczosOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("storage", ctypes.c_int32),
                ("reorth", ctypes.c_int32), ("seed", ctypes.c_uint64), ("check_every", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("refine", ctypes.c_int32), ("keep_basis", ctypes.c_int32)]


class LanczosResult(ctypes.Structure):
    _fields_ = [("E0", ctypes.c_double), ("resid_est", ctypes.c_double), ("E0_refined", ctypes.c_double),
                ("resid_refined", ctypes.c_double), ("seconds", ctypes.c_double), ("iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("restart_iters", ctypes.c_int32)]


class HvPlan(ctypes.Structure):
    _fields_ = [("down", ctypes.c_int32), ("up_cw", ctypes.c_int32), ("up", ctypes.c_int32), ("map", ctypes.c_int32)]


class HvTrial(ctypes.Structure):
    _fields_ = [("plan", HvPlan), ("ms", ctypes.c_double)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("tile_elems", ctypes.c_int32), ("block", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32)]


class BatchTrial(ctypes.Structure):
    _fields_ = [("plan", BatchPlan), ("ms", ctypes.c_double)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "pdz_problem_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(Bond), ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "pdz_problem_destroy": (ctypes.c_int32, [_P]),
    "pdz_problem_info": (ctypes.c_int32, [_P, ctypes.POINTER(Info)]),
    "pdz_rank": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_uint64, _P, _P]),
    "pdz_unrank": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_uint64, _P, _P]),
    "pdz_device_errors": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_uint32)]),
    "pdz_hv": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, _P]),
    "pdz_hv_pitched": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, ctypes.c_uint64, _P]),
    "pdz_hv_get_plan": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(HvPlan)]),
    "pdz_hv_set_plan": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(HvPlan)]),
    "pdz_hv_tune": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.POINTER(HvTrial),
                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(HvPlan), _P]),
    "pdz_hv_kernel_times": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_double), _P]),
    "pdz_lanczos_default_opts": (ctypes.c_int32, [ctypes.POINTER(LanczosOpts)]),
    "pdz_refine_decision": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "pdz_lanczos_workspace_size": (ctypes.c_int32, [_P, ctypes.POINTER(LanczosOpts), ctypes.POINTER(ctypes.c_size_t)]),
    "pdz_lanczos": (ctypes.c_int32, [_P, ctypes.POINTER(LanczosOpts), _P, _P, ctypes.c_size_t, _P,
                                     ctypes.POINTER(LanczosResult), _P]),
    "pdz_lanczos_kernel_times": (ctypes.c_int32, [_P, ctypes.POINTER(LanczosOpts), _P, ctypes.c_size_t, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), _P]),
    "pdz_lanczos_coefficients": (ctypes.c_int32, [_P, ctypes.POINTER(LanczosOpts), _P, ctypes.c_size_t, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "pdz_fermion_op": (ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                        _P]),
    "pdz_continued_fraction": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                                ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pdz_kspace_band": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Bond), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_double)]),
    "pdz_kspace_problem_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                   ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.POINTER(_P)]),
    "pdz_parity_problem_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(Bond), ctypes.c_int32,
                                                   ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.POINTER(_P)]),
    "pdz_parity_rank": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint64, _P, _P]),
    "pdz_parity_unrank": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P, _P, _P]),
    "pdz_kspace_rank": (ctypes.c_int32, [_P, _P, _P, ctypes.c_uint64, _P, _P]),
    "pdz_kspace_unrank": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P, _P, _P]),
    "pdz_kspace_info": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "pdz_lanczos_history": (ctypes.c_int32, [_P, ctypes.POINTER(LanczosOpts), _P, ctypes.c_size_t, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "pdz_batch_create": (ctypes.c_int32, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P)]),
    "pdz_batch_destroy": (ctypes.c_int32, [_P]),
    "pdz_batch_offsets": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    "pdz_batch_hv": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, _P]),
    "pdz_batch_get_plan": (ctypes.c_int32, [_P, ctypes.POINTER(BatchPlan)]),
    "pdz_batch_set_plan": (ctypes.c_int32, [_P, ctypes.POINTER(BatchPlan)]),
    "pdz_batch_tune": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.POINTER(BatchTrial),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(BatchPlan),
                                        _P]),
    "pdz_batch_lanczos_workspace_size": (ctypes.c_int32, [_P, ctypes.POINTER(LanczosOpts),
                                                          ctypes.POINTER(ctypes.c_size_t)]),
    "pdz_batch_lanczos": (ctypes.c_int32, [_P, ctypes.POINTER(LanczosOpts), _P, ctypes.c_size_t,
                                           ctypes.POINTER(LanczosResult), _P]),
    "pdz_mlp_param_count": (ctypes.c_int32, []),
    "pdz_mlp_init": (ctypes.c_int32, [_P, _P, ctypes.c_uint64]),
    "pdz_mlp_to_bf16": (ctypes.c_int32, [_P, _P, _P]),
    "pdz_mlp_forward": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P, _P, _P]),
    "pdz_mlp_workspace_size": (ctypes.c_int32, [ctypes.c_uint64, ctypes.POINTER(ctypes.c_size_t)]),
    "pdz_mlp_loss": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P, _P, _P, ctypes.c_size_t, _P]),
    "pdz_mlp_backward": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "pdz_adam_step": (ctypes.c_int32, [_P, _P, _P, _P, _P, ctypes.c_uint64, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_int32, _P]),
    "pdz_sampler_workspace_size": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "pdz_sampler_prepare": (ctypes.c_int32, [_P, _P, _P, ctypes.c_size_t, _P]),
    "pdz_sample": (ctypes.c_int32, [_P, _P, _P, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_double, _P, _P, _P, _P]),
    "pdz_start_vector": (ctypes.c_int32, [_P, _P, ctypes.c_int32, _P, _P]),
    "pdz_dot": (ctypes.c_int32, [ctypes.c_int32, _P, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), _P]),
    "pdz_dot_noalloc": (ctypes.c_int32, [ctypes.c_int32, _P, _P, ctypes.c_uint64, _P, _P]),
    "pdz_last_error": (ctypes.c_char_p, []),
    "pdz_version": (ctypes.c_int32, []),
}

_lib = None


def exported_symbols():
    return list(_SIGNATURES)


def load(path: str = LIB_PATH):
    """Load libpdz.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1707_03974_amd.build` "
                          "(the HIP library is required; there is no fallback)")
    # torch provides the device memory and streams, so its HIP runtime must be the
    # process's runtime: load it before libpdz resolves libamdhip64.so.7.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, allow=()):
    if status != PDZ_OK and status not in allow:
        msg = load().pdz_last_error()
        raise PdzError(status, msg.decode() if msg else "")
    return status
