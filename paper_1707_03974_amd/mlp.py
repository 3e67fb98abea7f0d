"""Learned Lanczos start vector: thin Python front end of the MLP kernels in libpdz.

Every computation (forward, loss, backward, Adam, |psi|^2 sampling, start
vector over the basis) runs in the HIP library; this module allocates the
device buffers with torch and passes pointers.
"""
import ctypes

from . import _lib
from ._lib import PDZ_F64, PDZ_F32


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _s(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def param_count():
    return _lib.load().pdz_mlp_param_count()


class Net:
    """FP32 master weights, their BF16 copy and the Adam moments, all on the device."""

    def __init__(self, seed=1, params=None):
        import torch
        n = param_count()
        self.w = torch.empty(n, dtype=torch.float32, device="cuda")
        self.wb = torch.empty(n, dtype=torch.int16, device="cuda")
        self.m = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.v = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.step = 0
        if params is None:
            _lib.check(_lib.load().pdz_mlp_init(_p(self.w), _p(self.wb), int(seed)))
        else:
            self.w.copy_(params.to(device="cuda", dtype=torch.float32))
            _lib.check(_lib.load().pdz_mlp_to_bf16(_p(self.w), _p(self.wb), _s()))

    def forward(self, occ, out=None, act=None, stream=None):
        """Outputs (n x 2 FP32) for occupation pairs occ (n x 2 int32: up bits, down bits)."""
        import torch
        n = occ.shape[0]
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        _lib.check(_lib.load().pdz_mlp_forward(_p(self.wb), _p(occ), n, _p(out), _p(act), _s(stream)))
        return out

    def adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        _lib.check(_lib.load().pdz_adam_step(_p(self.w), _p(self.wb), _p(grad), _p(self.m), _p(self.v),
                                             self.w.numel(), float(lr), float(beta1), float(beta2), float(eps),
                                             self.step, _s(stream)))


class Trainer:
    """Buffers of one training batch size (n a multiple of 32)."""

    def __init__(self, net, n):
        import torch
        if n % 32:
            raise ValueError("the batch size must be a multiple of 32")
        self.net, self.n = net, n
        self.occ = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        self.target = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        self.out = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        self.dout = torch.empty_like(self.out)
        self.act = torch.empty(n * 384, dtype=torch.int16, device="cuda")
        self.grad = torch.empty(param_count(), dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        nb = ctypes.c_size_t()
        _lib.check(_lib.load().pdz_mlp_workspace_size(n, ctypes.byref(nb)))
        self.ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")

    def gradient(self, stream=None):
        """Forward with saved activations, loss, backward on the current batch (occ, target)."""
        L = _lib.load()
        s = _s(stream)
        n = self.n
        _lib.check(L.pdz_mlp_forward(_p(self.net.wb), _p(self.occ), n, _p(self.out), _p(self.act), s))
        _lib.check(L.pdz_mlp_loss(_p(self.out), _p(self.target), n, _p(self.dout), _p(self.loss), _p(self.ws),
                                  self.ws.numel(), s))
        _lib.check(L.pdz_mlp_backward(_p(self.net.wb), _p(self.occ), n, _p(self.act), _p(self.dout),
                                      _p(self.grad), _p(self.ws), self.ws.numel(), s))
        return self.grad


class Sampler:
    """|psi|^2 sampling of basis states of one problem (exact integer prefix sums)."""

    def __init__(self, problem, psi, gauge=1.0, stream=None):
        import torch
        L = _lib.load()
        self.problem, self.psi, self.gauge = problem, psi, float(gauge)
        nb = ctypes.c_size_t()
        _lib.check(L.pdz_sampler_workspace_size(problem.handle, ctypes.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        _lib.check(L.pdz_sampler_prepare(problem.handle, _p(psi), _p(self.ws), self.ws.numel(), _s(stream)))

    def draw(self, seed, first, occ, target, idx=None, stream=None):
        n = occ.shape[0]
        _lib.check(_lib.load().pdz_sample(self.problem.handle, _p(self.psi), _p(self.ws), self.ws.numel(),
                                          int(seed), int(first), n, self.gauge, _p(occ), _p(target), _p(idx),
                                          _s(stream)))


def start_vector(problem, net, dtype, out=None, stream=None):
    """Unnormalised learned start vector over the problem's basis (N <= 16)."""
    import torch
    tdt = torch.float64 if dtype in (torch.float64, "f64", PDZ_F64) else torch.float32
    if out is None:
        out = torch.empty(problem.D, dtype=tdt, device="cuda")
    code = PDZ_F64 if tdt == torch.float64 else PDZ_F32
    _lib.check(_lib.load().pdz_start_vector(problem.handle, _p(net.wb), code, _p(out), _s(stream)))
    return out


def dot(a, b, stream=None):
    """FP64-accumulated dot product of two device vectors (synchronous)."""
    import torch
    r = ctypes.c_double()
    code = PDZ_F64 if a.dtype == torch.float64 else PDZ_F32
    _lib.check(_lib.load().pdz_dot(code, _p(a), _p(b), a.numel(), ctypes.byref(r), _s(stream)))
    return r.value
