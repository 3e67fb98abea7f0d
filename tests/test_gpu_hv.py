"""GPU H.v (libpdz) against the CPU oracle, element by element.

Tolerance: the GPU sums each row's terms in FP64 (or FP32) in its own order;
the bound (n+2) eps sum|terms| follows from the arithmetic (tests/_gpu.py).
Ranks and signs are exact: a wrong target or sign shows up as an error of the
size of a whole term, far above the bound.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from tests._gpu import torch_cuda, to_dev, to_host, hv_error_bound, EPS64, EPS32

pytestmark = pytest.mark.gpu


def _gpu_problem(w_or_args, fly=False):
    import paper_1707_03974_amd as pdz
    old = os.environ.get("PDZ_HV_ONTHEFLY")
    if fly:
        os.environ["PDZ_HV_ONTHEFLY"] = "1"
    try:
        if hasattr(w_or_args, "bonds"):
            return pdz.Problem.from_workload(w_or_args)
        return pdz.Problem(*w_or_args)
    finally:
        if fly:
            if old is None:
                del os.environ["PDZ_HV_ONTHEFLY"]
            else:
                os.environ["PDZ_HV_ONTHEFLY"] = old


def _oracle_problem(n_sites, bonds, U, n_up, n_dn):
    return oracle.Problem(n_sites, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds],
                          U, n_up, n_dn)


def _random_case(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 9))
    nb = int(rng.integers(0, 2 * N + 1))
    bonds = []
    for _ in range(nb):
        i, j = rng.choice(N, 2, replace=False)
        bonds.append((int(i), int(j), float(np.round(rng.uniform(-1.5, 1.5), 3))))
    if nb and rng.random() < 0.5:
        bonds.append(bonds[0])          # repeated pair: amplitudes add
    U = float(np.round(rng.uniform(-2, 8), 3))
    return N, bonds, U, int(rng.integers(0, N + 1)), int(rng.integers(0, N + 1))


NAMED = ["two_site", "ring8", "torus4x3"]
EDGE = [
    (4, [], 3.0, 2, 2),                        # no bonds: diagonal only
    (5, [(0, 1, 1.0), (3, 4, 1.0)], 2.0, 0, 0),  # D = 1
    (5, [(0, 1, 1.0), (1, 4, -0.5)], 2.0, 5, 2),  # full up sector
    (6, [(0, 5, 1.0), (2, 3, 0.7)], 1.0, 3, 0),   # D_dn = 1
    (1, [], 5.0, 1, 1),                        # one site, doubly occupied
    (7, [(i, (i + 1) % 7, 1.0) for i in range(7)], 4.0, 3, 5),  # ragged rows
]


def _check(args, dtype_name, fly=False, seed=7):
    torch = torch_cuda()
    N, bonds, U, nu, nd = args
    po = _oracle_problem(N, bonds, U, nu, nd)
    H = oracle.build_csr(po)
    x = synth.random_vector(po.D, seed)
    y_ref = H @ x
    g = _gpu_problem((N, [synth.Bond(i, j, t) for i, j, t in bonds], U, nu, nd), fly=fly)
    # structural count keeps one entry per bond term, so repeated pairs count twice
    assert g.D == po.D and g.nnz == oracle.nnz_structural(po)
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    y = to_host(g.hv(to_dev(x, dt))).astype(np.float64)
    bound = hv_error_bound(H, x, EPS64 if dtype_name == "f64" else EPS32)
    err = np.abs(y - y_ref)
    assert np.all(err <= bound), (args, float(np.max(err - bound)))
    return g, x, y


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("name", NAMED)
def test_hv_named_workloads(name, dtype_name):
    w = synth.workload(name)
    _check((w.n_sites, [(b.i, b.j, b.t) for b in w.bonds], w.U, w.n_up, w.n_dn), dtype_name)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(16))
def test_hv_random_small_problems(seed, dtype_name):
    _check(_random_case(seed), dtype_name, seed=seed)


@pytest.mark.parametrize("args", EDGE)
def test_hv_edge_cases(args):
    _check(args, "f64")
    _check(args, "f32")


@pytest.mark.parametrize("seed", [3, 5, 11])
def test_onthefly_path_is_bitwise_equal_to_table_path(seed):
    torch = torch_cuda()
    N, bonds, U, nu, nd = _random_case(seed)
    for dt in (torch.float64, torch.float32):
        gt = _gpu_problem((N, [synth.Bond(*b) for b in bonds], U, nu, nd))
        gf = _gpu_problem((N, [synth.Bond(*b) for b in bonds], U, nu, nd), fly=True)
        assert gt.info["hv_path"] == 0 and gf.info["hv_path"] == 1
        x = to_dev(synth.random_vector(gt.D, seed), dt)
        assert torch.equal(gt.hv(x), gf.hv(x))


def test_onthefly_path_matches_oracle():
    w = synth.workload("torus4x3")
    args = (w.n_sites, [(b.i, b.j, b.t) for b in w.bonds], w.U, w.n_up, w.n_dn)
    _check(args, "f64", fly=True)


def test_hv_is_deterministic():
    torch = torch_cuda()
    g = _gpu_problem(synth.workload("torus4x3"))
    x = to_dev(synth.random_vector(g.D, 1), torch.float64)
    assert torch.equal(g.hv(x), g.hv(x))


def test_hv_rejects_bad_arguments():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    from paper_1707_03974_amd import _lib
    import ctypes
    g = _gpu_problem(synth.workload("ring8"))
    x = torch.zeros(g.D, dtype=torch.float64, device="cuda")
    lib = pdz.lib()
    assert lib.pdz_hv(g.handle, 0, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr() + 8), None) == \
        _lib.PDZ_EINVAL
    assert lib.pdz_hv(g.handle, 7, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), None) == \
        _lib.PDZ_EINVAL


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("name", ["torus4x4_nnn", "torus4x4_n7"])
def test_hv_full_size_sampled_rows_every_plan(name, dtype_name):
    """Full 4x4 clusters (D ~ 1.3e8 - 1.7e8) under every launch plan the autotuner may pick (so the
    plan the benchmark selects is among them): sampled rows against the oracle with each row's own
    bound (n + 2) eps sum|terms| (and, in FP32, the 2e-6 sum|terms| tolerance proposed for FP32
    accumulation), and every plan bitwise equal to the first."""
    torch = torch_cuda()
    w = synth.workload(name)
    po = oracle.Problem.from_workload(w)
    g = _gpu_problem(w)
    D = g.D
    x = synth.random_vector(D, 2024)
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    if dtype_name == "f32":
        x = x.astype(np.float32).astype(np.float64)      # the oracle sees the FP32 inputs exactly
    xd = to_dev(x, dt)
    rng = np.random.default_rng(5)
    Ddn = g.info["D_dn"]
    rows = np.unique(np.concatenate([rng.integers(0, D, 4000), [0, 1, Ddn - 1, Ddn, D // 2, D - Ddn, D - 2, D - 1]]))
    rows_d = torch.from_numpy(rows).cuda()
    y_ref, asum, nterm = oracle.hv_rows(po, x, rows, with_abs=True)
    eps = EPS64 if dtype_name == "f64" else EPS32
    bound = (nterm + 2) * eps * asum + nterm * EPS64 * asum
    ref = None
    keys = ("down", "up_cw", "up", "map")
    _, trials = g.tune(dt, reps=1, x=xd, y=torch.empty_like(xd))
    assert len(trials) >= 2
    worst = 0.0
    for t in trials:
        g.set_plan(dt, *[t[k] for k in keys])
        yd = g.hv(xd)
        y = to_host(yd[rows_d]).astype(np.float64)
        err = np.abs(y - y_ref)
        assert np.all(err <= bound), (t, float(np.max(err - bound)))
        worst = max(worst, float(np.max(err / asum)))
        if ref is None:
            ref = yd
        else:
            assert torch.equal(yd, ref), (name, dtype_name, t)
        del yd
    if dtype_name == "f32":
        assert worst <= 2e-6, worst
    del xd, ref


@pytest.mark.parametrize("name", ["ring8", "torus4x3", "torus4x4_n7", "torus4x4_nnn"])
def test_every_plan_gives_identical_results(name):
    """All launch plans the autotuner may pick sum each element in the same order."""
    torch = torch_cuda()
    g = _gpu_problem(synth.workload(name))
    for dt in (torch.float64, torch.float32):
        x = to_dev(synth.random_vector(g.D, 5), dt)
        ref = g.hv(x)
        best, trials = g.tune(dt, reps=1, x=x, y=torch.empty_like(x))
        keys = ("down", "up_cw", "up", "map")
        assert len(trials) >= 1 and best in [{k: t[k] for k in keys} for t in trials]
        for t in trials:
            g.set_plan(dt, *[t[k] for k in keys])
            assert g.get_plan(dt) == {k: t[k] for k in keys}
            assert torch.equal(g.hv(x), ref), (name, dt, t)


def test_invalid_plan_is_rejected():
    import paper_1707_03974_amd as pdz
    g = _gpu_problem(synth.workload("torus4x3"))
    with pytest.raises(pdz.PdzError):
        g.set_plan("f32", 1, 7)


def test_problem_plan_cache_round_trip(tmp_path):
    from paper_1707_03974_amd import tuning
    g = _gpu_problem(synth.workload("torus4x3"))
    path = str(tmp_path / "plans.json")
    e1, t1 = tuning.tuned_plan(g, "f64", reps=1, path=path)
    assert t1 and e1["ms"] > 0
    g.set_plan("f64", 0, 0, 0, 0)
    e2, t2 = tuning.tuned_plan(g, "f64", reps=1, path=path)
    assert t2 is None and e2 == e1
    assert g.get_plan("f64") == {k: e1[k] for k in ("down", "up_cw", "up", "map")}


def _ring14(amps):
    """14-site ring, 2 up and 7 down electrons (down rows of 3432 states: the wide down pass),
    bond b carrying amplitude amps[b % len(amps)]."""
    bonds = [(i, (i + 1) % 14, float(amps[i % len(amps)])) for i in range(14)]
    return 14, bonds, 1.5, 2, 7


@pytest.mark.parametrize("amps,scheduled", [((1.0, -0.45), True), ((1.0, 0.7, -0.4), False)])
def test_down_families_on_rows_with_and_without_a_gather_schedule(amps, scheduled):
    """A down sector with at most two hop magnitudes gets the bank-conflict-free gather schedule
    (plans 5-7 by default); one with three keeps the looped family (plans 1-4).  Either way each
    element equals the oracle within its own rounding bound; the looped family, set explicitly on the
    scheduled problem, does too."""
    torch = torch_cuda()
    args = _ring14(amps)
    g = _gpu_problem(args)
    po = _oracle_problem(*args)
    x = synth.random_vector(g.D, 17)
    rows = np.unique(np.random.default_rng(3).integers(0, g.D, 3000))
    ref, asum, nterm = oracle.hv_rows(po, x, rows, with_abs=True)
    rows_d = torch.from_numpy(rows).cuda()
    for dt, eps in ((torch.float64, EPS64), (torch.float32, EPS32)):
        name = "f64" if dt == torch.float64 else "f32"
        down = g.get_plan(name)["down"]
        assert (5 <= down <= 7) if scheduled else (1 <= down <= 4), (amps, name, down)
        plans = [0] + ([2] if scheduled else [])
        for pl in plans:
            g.set_plan(name, pl, 0, 0, 0)
            y = to_host(g.hv(to_dev(x, dt))[rows_d])
            bound = (nterm + 2) * eps * asum + nterm * EPS64 * asum
            err = np.abs(y - ref)
            assert np.all(err <= bound), (amps, name, pl, float(np.max(err / np.maximum(bound, 1e-300))))
        g.set_plan(name, 0, 0, 0, 0)


def _ring_nnn(N, nu, nd, U=2.5):
    """N-site ring with first (t = 1) and second (t' = -0.35) neighbour bonds."""
    bonds = [(i, (i + 1) % N, 1.0) for i in range(N)] + [(i, (i + 2) % N, -0.35) for i in range(N)]
    return N, bonds, U, nu, nd


@pytest.mark.parametrize("args", [_ring_nnn(17, 1, 8), _ring_nnn(18, 1, 9)], ids=["dn24310", "dn48620"])
def test_down_rows_longer_than_the_gather_schedule_plane(args):
    """Down sectors of 24,310 and 48,620 states: past the gather schedule's plane (13,280 states), so
    the looped wide pass (rows staged in LDS) or the narrow pass (rows too long for LDS) runs; every
    plan the autotuner offers, on sampled rows, within each row's own rounding bound."""
    torch = torch_cuda()
    g = _gpu_problem(args)
    po = _oracle_problem(*args)
    assert g.info["D_dn"] in (24310, 48620)
    x = synth.random_vector(g.D, 23)
    rng = np.random.default_rng(8)
    Ddn = g.info["D_dn"]
    rows = np.unique(np.concatenate([rng.integers(0, g.D, 2500), [0, Ddn - 1, Ddn, g.D - 1]]))
    ref, asum, nterm = oracle.hv_rows(po, x, rows, with_abs=True)
    rows_d = torch.from_numpy(rows).cuda()
    for dt, eps in ((torch.float64, EPS64), (torch.float32, EPS32)):
        name = "f64" if dt == torch.float64 else "f32"
        xd = to_dev(x, dt)
        _, trials = g.tune(dt, reps=1, x=xd, y=torch.empty_like(xd))
        assert all(not (5 <= t["down"] <= 7) for t in trials), trials   # no schedule for these rows
        bound = (nterm + 2) * eps * asum + nterm * EPS64 * asum
        for t in trials:
            g.set_plan(name, t["down"], t["up_cw"], t["up"], t["map"])
            y = to_host(g.hv(xd)[rows_d])
            err = np.abs(y - ref)
            assert np.all(err <= bound), (args[:1], name, t, float(np.max(err / np.maximum(bound, 1e-300))))
        g.set_plan(name, 0, 0, 0, 0)


@pytest.mark.parametrize("name", ["torus4x3", "torus4x4_nnn"])
def test_pitched_rows_give_the_plain_result_bitwise(name):
    """pdz_hv_pitched on rows padded to a multiple of 32 elements (and to one element more than a row):
    every element bitwise equal to pdz_hv's, the padding columns of y untouched, x's never read."""
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    g = _gpu_problem(synth.workload(name))
    Dup, Ddn = g.info["D_up"], g.info["D_dn"]
    for dt in (torch.float64, torch.float32):
        x = to_dev(synth.random_vector(g.D, 31), dt)
        ref = g.hv(x)
        for pitch in ((Ddn + 31) // 32 * 32 + (32 if Ddn % 32 == 0 else 0), Ddn + 1):
            xp = torch.full((Dup, pitch), float("nan"), dtype=dt, device="cuda")   # padding never read
            xp[:, :Ddn] = x.view(Dup, Ddn)
            yp = torch.full((Dup, pitch), 7.0, dtype=dt, device="cuda")
            g.hv_pitched(xp.view(-1), pitch, y=yp.view(-1))
            assert torch.equal(yp[:, :Ddn].reshape(-1), ref), (name, dt, pitch)
            assert bool(torch.all(yp[:, Ddn:] == 7.0)), (name, dt, pitch)
            del xp, yp
        del x, ref
    with pytest.raises(pdz.PdzError):
        g.hv_pitched(torch.zeros(Dup * (Ddn - 1), device="cuda"), Ddn - 1)
