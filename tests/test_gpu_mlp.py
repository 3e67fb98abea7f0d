"""MLP kernels of the learned start (libpdz) against the FP64 reference in oracle/mlp.py.

The device multiplies BF16 operands with FP32 accumulation and stores BF16
activations; the reference rounds the same quantities (round_bf16=True) and
does everything else in FP64.  Bounds: outputs and gradients within 1e-2
relative (FP32 accumulation, BF16 storage of activations and of the
backward's intermediate products); loss, dout and Adam within FP32 rounding;
sampled indices exact (integer weights, exact prefix sums).
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as ref
import synth
from tests._gpu import torch_cuda, to_dev, to_host

pytestmark = pytest.mark.gpu


def _net(seed, scale=1.0):
    from paper_1707_03974_amd import mlp
    torch = torch_cuda()
    theta = ref.init_params(seed) * scale
    rng = np.random.default_rng(seed + 1)
    p = ref.unpack(theta)
    for b in ("b1", "b2", "b3"):
        p[b][...] = rng.normal(0.0, 0.3, p[b].shape)
    theta32 = theta.astype(np.float32)
    return mlp.Net(params=torch.from_numpy(theta32)), theta32.astype(np.float64)


def _states(rng, n):
    up = rng.integers(0, 1 << 16, n).astype(np.uint32)
    dn = rng.integers(0, 1 << 16, n).astype(np.uint32)
    return up, dn


def _occ(up, dn):
    torch = torch_cuda()
    o = np.stack([up, dn], axis=1).astype(np.uint32).view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(o)).cuda()


def test_bf16_copy_of_the_weights_is_round_to_nearest_even():
    torch = torch_cuda()
    net, theta = _net(3)
    wb = to_host(net.wb).astype(np.uint16).astype(np.uint32) << 16
    got = wb.view(np.float32).astype(np.float64)
    assert np.array_equal(got, ref.bf16_round(theta))


@pytest.mark.parametrize("n", [1, 16, 77, 1000, 4096])
def test_forward_matches_reference(n):
    net, theta = _net(5)
    rng = np.random.default_rng(n)
    up, dn = _states(rng, n)
    out = to_host(net.forward(_occ(up, dn))).astype(np.float64)
    expect, _ = ref.forward(theta, up, dn, round_bf16=True)
    err = np.abs(out - expect)
    assert np.all(err <= 1e-2 * np.maximum(1.0, np.abs(expect))), float(err.max())
    # typical agreement is far tighter than the bound
    assert np.median(err) < 1e-3


def test_saved_activations_match_reference():
    torch = torch_cuda()
    net, theta = _net(9)
    n = 256
    rng = np.random.default_rng(2)
    up, dn = _states(rng, n)
    act = torch.empty(n * 384, dtype=torch.int16, device="cuda")
    net.forward(_occ(up, dn), act=act)
    a = (to_host(act).astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    h1, h1t, h2 = a[:n * 128].reshape(n, 128), a[n * 128:2 * n * 128].reshape(128, n), a[2 * n * 128:].reshape(n, 128)
    _, cache = ref.forward(theta, up, dn, round_bf16=True)
    assert np.array_equal(h1, h1t.T)
    # one BF16 ulp (2^-8 relative, values within [-1, 1]) covers FP32-vs-FP64 rounding flips
    assert np.max(np.abs(h1 - cache["h1"])) <= 2.0 ** -7
    assert np.max(np.abs(h2 - cache["h2"])) <= 2.0 ** -6
    assert np.mean(h1 == cache["h1"]) > 0.95


def test_loss_and_output_gradient_match_reference():
    torch = torch_cuda()
    from paper_1707_03974_amd import mlp
    net, _ = _net(4)
    n = 1024
    tr = mlp.Trainer(net, n)
    rng = np.random.default_rng(8)
    out = rng.normal(0.0, 2.0, (n, 2)).astype(np.float32)
    tgt = np.stack([rng.normal(-5, 1, n), rng.choice([-1.0, 1.0], n)], axis=1).astype(np.float32)
    tr.out.copy_(torch.from_numpy(out))
    tr.target.copy_(torch.from_numpy(tgt))
    from paper_1707_03974_amd import _lib
    import ctypes
    L = _lib.load()
    _lib.check(L.pdz_mlp_loss(ctypes.c_void_p(tr.out.data_ptr()), ctypes.c_void_p(tr.target.data_ptr()), n,
                              ctypes.c_void_p(tr.dout.data_ptr()), ctypes.c_void_p(tr.loss.data_ptr()),
                              ctypes.c_void_p(tr.ws.data_ptr()), tr.ws.numel(), None))
    torch.cuda.synchronize()
    loss, dout = ref.loss_and_dout(out.astype(np.float64), tgt[:, 0].astype(np.float64), tgt[:, 1])
    assert abs(tr.loss.item() - loss) <= 1e-6 * abs(loss)
    assert np.allclose(to_host(tr.dout), dout, rtol=1e-5, atol=1e-9)


def _gradient_case(n, seed):
    torch = torch_cuda()
    from paper_1707_03974_amd import mlp
    net, theta = _net(seed, scale=1.5)
    rng = np.random.default_rng(seed)
    up, dn = _states(rng, n)
    tr = mlp.Trainer(net, n)
    tr.occ.copy_(_occ(up, dn))
    la = rng.normal(-4.0, 1.5, n)
    sg = rng.choice([-1.0, 1.0], n)
    tr.target.copy_(torch.from_numpy(np.stack([la, sg], 1).astype(np.float32)))
    g = to_host(tr.gradient()).astype(np.float64)
    out, cache = ref.forward(theta, up, dn, round_bf16=True)
    _, dout = ref.loss_and_dout(out, la.astype(np.float32).astype(np.float64), sg)
    return g, ref.backward(cache, dout)


@pytest.mark.parametrize("n,seed", [(32, 1), (512, 2), (4096, 3), (1056, 4)])
def test_backward_matches_reference(n, seed):
    g, e = _gradient_case(n, seed)
    for name, part in ref.unpack(np.arange(ref.N_PARAMS)).items():
        k = part.ravel()
        rel = np.linalg.norm(g[k] - e[k]) / max(np.linalg.norm(e[k]), 1e-30)
        assert rel <= 1e-2, (name, rel)


def test_adam_matches_reference():
    torch = torch_cuda()
    from paper_1707_03974_amd import mlp
    net, theta = _net(6)
    rng = np.random.default_rng(6)
    m = np.zeros(ref.N_PARAMS)
    v = np.zeros(ref.N_PARAMS)
    th = theta.copy()
    for step in range(1, 6):
        g = rng.normal(0.0, 0.1, ref.N_PARAMS).astype(np.float32)
        net.adam(torch.from_numpy(g).cuda(), lr=1e-3)
        th, m, v = ref.adam_step(th, g.astype(np.float64), m, v, step, lr=1e-3)
    w = to_host(net.w).astype(np.float64)
    assert np.max(np.abs(w - th)) <= 1e-6 * np.max(np.abs(th)) + 1e-7
    wb = (to_host(net.wb).astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.array_equal(wb, ref.bf16_round(to_host(net.w)))


def _ground_state(name):
    from scipy.sparse.linalg import eigsh
    w = synth.workload(name)
    po = oracle.Problem.from_workload(w)
    H = oracle.build_csr(po)
    vals, vecs = eigsh(H, k=1, which="SA", v0=np.ones(H.shape[0]), tol=1e-12)
    return w, po, vecs[:, 0]


@pytest.mark.parametrize("gauge", [1.0, -1.0])
def test_sampler_draws_exactly_the_reference_indices(gauge):
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    from paper_1707_03974_amd import mlp
    w, po, psi = _ground_state("ring8")
    g = pdz.Problem.from_workload(w)
    psi_d = to_dev(psi, torch.float64)
    s = mlp.Sampler(g, psi_d, gauge=gauge)
    n = 3000
    occ = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    tgt = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    s.draw(21, 1000, occ, tgt, idx)
    got = to_host(idx).astype(np.int64)
    assert np.array_equal(got, ref.sample_indices(psi, 21, 1000, n))
    Ddn = len(po.dn_list)
    o = to_host(occ).view(np.uint32)
    assert np.array_equal(o[:, 0], po.up_list[got // Ddn]) and np.array_equal(o[:, 1], po.dn_list[got % Ddn])
    t = to_host(tgt)
    assert np.allclose(t[:, 0], np.log(np.abs(psi[got])), rtol=0, atol=1e-5)
    assert np.array_equal(t[:, 1], np.where(psi[got] * gauge > 0, 1.0, -1.0).astype(np.float32))


def test_sampler_prefix_is_exact_at_a_ragged_size():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    from paper_1707_03974_amd import mlp
    g = pdz.Problem(10, [synth.Bond(i, (i + 1) % 10, 1.0) for i in range(10)], 3.0, 4, 3)   # D = 210 * 120
    psi = synth.random_vector(g.D, 4) ** 3
    s = mlp.Sampler(g, to_dev(psi, torch.float64))
    n = 20000
    occ = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    tgt = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    s.draw(3, 0, occ, tgt, idx)
    assert np.array_equal(to_host(idx).astype(np.int64), ref.sample_indices(psi, 3, 0, n))


def test_start_vector_matches_reference_over_the_basis():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    from paper_1707_03974_amd import mlp
    net, theta = _net(12, scale=0.7)
    w = synth.workload("ring8")
    po = oracle.Problem.from_workload(w)
    g = pdz.Problem.from_workload(w)
    for dt in (torch.float64, torch.float32):
        v = to_host(mlp.start_vector(g, net, dt)).astype(np.float64)
        up = np.repeat(po.up_list, len(po.dn_list))
        dn = np.tile(po.dn_list, len(po.up_list))
        out, _ = ref.forward(theta, up, dn, round_bf16=True)
        e = ref.start_vector(theta, po.up_list, po.dn_list, round_bf16=True)
        sure = np.abs(out[:, 1]) > 0.05          # sign decisions away from the logit's zero
        assert np.array_equal(np.sign(v[sure]), np.sign(e[sure]))
        assert np.allclose(np.abs(v), np.abs(e), rtol=2e-2, atol=0)


def test_dot_matches_numpy():
    torch = torch_cuda()
    from paper_1707_03974_amd import mlp
    a = synth.random_vector(100003, 1)
    b = synth.random_vector(100003, 2)
    assert mlp.dot(to_dev(a, torch.float64), to_dev(b, torch.float64)) == pytest.approx(float(a @ b), rel=1e-12)


def test_training_steps_reduce_the_loss_on_a_ground_state():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    from paper_1707_03974_amd import mlp
    w, po, psi = _ground_state("ring8")
    g = pdz.Problem.from_workload(w)
    s = mlp.Sampler(g, to_dev(psi, torch.float64))
    net = mlp.Net(seed=3)
    tr = mlp.Trainer(net, 1024)
    losses = []
    for it in range(400):
        s.draw(17, it * 1024, tr.occ, tr.target)
        tr.gradient()
        net.adam(tr.grad, lr=3e-3)
        if it % 50 == 0 or it == 399:
            losses.append(tr.loss.item())
    assert losses[-1] < 0.5 * losses[0], losses
