"""Device-resident Lanczos (libpdz) against the oracle's ground-state energies."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests._gpu import torch_cuda, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _energies():
    with open(os.path.join(GOLD, "energies.json")) as f:
        return json.load(f)


def _gpu(name):
    import paper_1707_03974_amd as pdz
    return pdz.Problem.from_workload(synth.workload(name))


@pytest.mark.parametrize("name", ["two_site", "ring8", "torus4x3"])
def test_fp64_energy_matches_oracle(name):
    E = _energies()[name]["E0"]
    g = _gpu(name)
    r = g.lanczos(tol=1e-12, max_iter=600)
    assert r["converged"] == 1
    assert abs(r["E0"] - E) <= 1e-9 * abs(E), (r, E)


def test_two_site_closed_form():
    U, t = 4.0, 1.0
    E = (U - np.sqrt(U * U + 16 * t * t)) / 2
    r = _gpu("two_site").lanczos(tol=1e-14)
    assert abs(r["E0"] - E) <= 1e-12


def test_graph_and_stream_paths_agree_bitwise():
    g = _gpu("ring8")
    a = g.lanczos(use_graph=1, check_every=6)
    b = g.lanczos(use_graph=0, check_every=6)
    c = g.lanczos(use_graph=1, check_every=30)
    assert a["E0"] == b["E0"] == c["E0"]
    assert a["iters"] == b["iters"] == c["iters"]


def test_seeded_start_equals_oracle_splitmix_vector():
    torch = torch_cuda()
    g = _gpu("ring8")
    v0 = to_dev(oracle.start_vector(77, g.D), torch.float64)
    a = g.lanczos(seed=77)
    b = g.lanczos(v0=v0)
    assert a["E0"] == b["E0"] and a["iters"] == b["iters"]


def test_fp32_storage_and_fp64_refinement():
    E = _energies()["torus4x3"]["E0"]
    g = _gpu("torus4x3")
    r = g.lanczos(storage="f32", tol=1e-7, max_iter=400, refine=1)
    assert abs(r["E0"] - E) <= 2e-6 * abs(E)
    assert abs(r["E0_refined"] - E) <= 1e-8 * abs(E), r
    assert r["resid_refined"] >= 0


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_kept_basis_refinement_equals_regenerating_refinement_bitwise(storage):
    """The refinement from kept Lanczos vectors forms the same sums, in the same order, over the same
    vectors as the one that regenerates them: identical Rayleigh quotient, residual and Ritz vector."""
    torch = torch_cuda()
    g = _gpu("torus4x3")
    ya = torch.empty(g.D, dtype=torch.float64, device="cuda")
    yb = torch.empty(g.D, dtype=torch.float64, device="cuda")
    a = g.lanczos(storage=storage, tol=1e-7, max_iter=400, ritz=ya)
    b = g.lanczos(storage=storage, tol=1e-7, max_iter=400, ritz=yb, keep_basis=1)
    for k in ("E0", "E0_refined", "resid_refined", "iters"):
        assert a[k] == b[k], (k, a, b)
    assert torch.equal(ya, yb)
    # a start vector given by the caller, and the plain stream path
    v0 = to_dev(synth.random_vector(g.D, 9), torch.float64 if storage == "f64" else torch.float32)
    c = g.lanczos(v0=v0, storage=storage, tol=1e-9, max_iter=400, refine=1, use_graph=0)
    d = g.lanczos(v0=v0, storage=storage, tol=1e-9, max_iter=400, refine=1, keep_basis=1)
    assert c["E0_refined"] == d["E0_refined"] and c["resid_refined"] == d["resid_refined"], (c, d)


# a problem whose rows are long enough for the wide down pass, where the update of each Lanczos step
# is carried out by the next step's down pass: 14-site ring, 2 + 7 electrons (D = 91 * 3432)
RING14 = dict(n_sites=14, U=3.0, n_up=2, n_dn=7)


def _ring14_bonds():
    return [synth.Bond(i, (i + 1) % 14, 1.0) for i in range(14)] + [synth.Bond(i, (i + 2) % 14, -0.3) for i in range(14)]


def _ring14():
    import paper_1707_03974_amd as pdz
    return pdz.Problem(RING14["n_sites"], _ring14_bonds(), RING14["U"], RING14["n_up"], RING14["n_dn"])


def _ring14_e0():
    from scipy.sparse.linalg import eigsh
    b = _ring14_bonds()
    po = oracle.Problem(14, [x.i for x in b], [x.j for x in b], [x.t for x in b], RING14["U"], RING14["n_up"],
                        RING14["n_dn"])
    H = oracle.build_csr(po)
    # a random start: a symmetric one (all ones) can miss the ground state's symmetry sector
    v0 = np.random.default_rng(14).standard_normal(H.shape[0])
    return float(eigsh(H, k=1, which="SA", tol=1e-13, v0=v0)[0][0])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_fused_recurrence_path_matches_oracle_and_unfused_path(storage):
    g = _ring14()
    assert g.info["D_dn"] >= 1024
    E = _ring14_e0()
    tol = 1e-12 if storage == "f64" else 1e-7
    # looped wide down pass (the update rides on it) against the up-front variant (separate update)
    g.set_plan(storage, 3, 0, 0, 0)
    a = g.lanczos(storage=storage, tol=tol, max_iter=600, refine=1)
    g.set_plan(storage, 1, 0, 0, 0)
    b = g.lanczos(storage=storage, tol=tol, max_iter=600, refine=1)
    g.set_plan(storage, 0, 0, 0, 0)
    bound = 1e-10 if storage == "f64" else 1e-8
    for r in (a, b):
        assert r["converged"] == 1
        assert abs(r["E0_refined"] - E) <= bound * abs(E), (r, E)
    assert abs(a["iters"] - b["iters"]) <= 2, (a, b)
    if storage == "f64":
        assert abs(a["E0"] - b["E0"]) <= 1e-12 * abs(E)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_fused_pass_forms_the_vectors_the_separate_update_regenerates(storage):
    """Kept vectors come from the fused down pass; the regenerating refinement re-forms them with the
    separate update kernel: equal Ritz vectors bit for bit only if every vector is equal bit for bit."""
    torch = torch_cuda()
    g = _ring14()
    g.set_plan(storage, 4 if storage == "f32" else 2, 0, 0, 0)
    ya = torch.empty(g.D, dtype=torch.float64, device="cuda")
    yb = torch.empty(g.D, dtype=torch.float64, device="cuda")
    a = g.lanczos(storage=storage, tol=1e-9, max_iter=400, ritz=ya)
    b = g.lanczos(storage=storage, tol=1e-9, max_iter=400, ritz=yb, keep_basis=1)
    g.set_plan(storage, 0, 0, 0, 0)
    for k in ("E0", "E0_refined", "resid_refined", "iters"):
        assert a[k] == b[k], (k, a, b)
    assert torch.equal(ya, yb)


@pytest.mark.parametrize("n_up", [0, 1])
def test_fused_path_with_one_or_few_rows(n_up):
    """Fused recurrence where the up sector has one state (no up hops: the up part is zero) or 14
    states (fewer rows than the work groups)."""
    import paper_1707_03974_amd as pdz
    from scipy.sparse.linalg import eigsh
    b = _ring14_bonds()
    g = pdz.Problem(14, b, 3.0, n_up, 7)
    po = oracle.Problem(14, [x.i for x in b], [x.j for x in b], [x.t for x in b], 3.0, n_up, 7)
    H = oracle.build_csr(po)
    v0 = np.random.default_rng(15).standard_normal(H.shape[0])
    E = float(eigsh(H, k=1, which="SA", tol=1e-13, v0=v0)[0][0])
    for dt in ("f64", "f32"):
        g.set_plan(dt, 2, 0, 0, 0)   # one-row looped down pass: the update rides on it
        t = g.lanczos_kernel_times(dt, steps=4)
        assert t["fused"], t
        r = g.lanczos(storage=dt, tol=1e-12 if dt == "f64" else 1e-7, max_iter=400, refine=1)
        bound = 1e-10 if dt == "f64" else 1e-8
        assert abs(r["E0_refined"] - E) <= bound * abs(E), (dt, r, E)


def test_fused_path_graph_and_stream_agree_bitwise():
    g = _ring14()
    a = g.lanczos(storage="f32", tol=1e-7, use_graph=1, check_every=4)
    b = g.lanczos(storage="f32", tol=1e-7, use_graph=0, check_every=4)
    c = g.lanczos(storage="f32", tol=1e-7, use_graph=1, check_every=7)
    assert a["E0"] == b["E0"] == c["E0"] and a["iters"] == b["iters"] == c["iters"]


def test_lanczos_step_timing_reports_each_launch_group():
    import paper_1707_03974_amd as pdz
    g = _ring14()
    for dt, plan, fused in (("f32", (4, 0, 0, 0), True), ("f32", (1, 0, 0, 0), False), ("f64", (2, 0, 0, 0), True)):
        g.set_plan(dt, *plan)
        t = g.lanczos_kernel_times(dt, steps=6)
        assert t["fused"] == fused, (dt, plan, t)
        assert t["down"] > 0 and t["up"] > 0 and t["scalars"] > 0
        assert (t["update"] > 0) == (not fused)
        assert t["step"] >= t["down"] + t["up"] + t["update"] - 1e-9
    g.set_plan("f32", 0, 0, 0, 0)
    g.set_plan("f64", 0, 0, 0, 0)
    with pytest.raises(pdz.PdzError):
        g.lanczos_kernel_times("f32", steps=0)


def test_fp32_run_with_fp64_restart_recovers_the_fp64_energy():
    """refine = 2: a loosely converged FP32 run whose Ritz vector does not bound the energy to 1e-8 is
    followed by FP64 Lanczos from that vector; the result is the FP64 ground-state energy."""
    torch = torch_cuda()
    E = _energies()["torus4x3"]["E0"]
    g = _gpu("torus4x3")
    y = torch.empty(g.D, dtype=torch.float64, device="cuda")
    r = g.lanczos(storage="f32", tol=1e-12, max_iter=25, refine=2, ritz=y)   # stopped early on purpose
    assert r["converged"] == 0 and r["restart_iters"] > 0, r
    assert abs(r["E0_refined"] - E) <= 1e-10 * abs(E), r
    assert abs(float(torch.linalg.norm(y)) - 1.0) < 1e-12
    # a converged FP64 run needs no restart; refine = 1 reports no restart either
    a = g.lanczos(storage="f64", tol=1e-12, max_iter=400, refine=2)
    assert a["restart_iters"] == 0 and abs(a["E0_refined"] - E) <= 1e-10 * abs(E), a
    b = g.lanczos(storage="f32", tol=1e-12, max_iter=25, refine=1)
    assert b["restart_iters"] == 0 and abs(b["E0_refined"] - E) > 1e-10 * abs(E), b
    # the restart's workspace is part of the refine = 2 size
    o1 = g.lanczos_opts(storage="f32", max_iter=100, refine=1)
    o2 = g.lanczos_opts(storage="f32", max_iter=100, refine=2)
    assert g.workspace_size(o2) > g.workspace_size(o1) + 3 * g.D * 8


def test_kept_basis_option_is_validated_and_sized():
    import paper_1707_03974_amd as pdz
    g = _gpu("ring8")
    o0 = g.lanczos_opts(storage="f32", max_iter=50)
    o1 = g.lanczos_opts(storage="f32", max_iter=50, keep_basis=1)
    vec = ((g.D * 4 + 255) // 256) * 256
    assert g.workspace_size(o1) - g.workspace_size(o0) == 51 * vec
    with pytest.raises(pdz.PdzError):
        g.lanczos(keep_basis=2)


def test_full_reorthogonalisation():
    E = _energies()["ring8"]["E0"]
    r = _gpu("ring8").lanczos(reorth=2, tol=1e-12)
    assert r["converged"] and abs(r["E0"] - E) <= 1e-10 * abs(E)


@pytest.mark.parametrize("name", ["ring8", "torus4x3"])
@pytest.mark.parametrize("reorth", [0, 1, 2])
def test_reorthogonalisation_modes_match_oracle(name, reorth):
    """0 none, 1 local (against v_(k-1), v_k), 2 full: FP64 E0 within 1e-9 of the oracle's."""
    E = _energies()[name]["E0"]
    r = _gpu(name).lanczos(reorth=reorth, tol=1e-12, max_iter=300)
    assert r["converged"] == 1
    assert abs(r["E0"] - E) <= 1e-9 * abs(E), (reorth, r, E)


def test_local_reorthogonalisation_fp32_storage_refined():
    """FP32 vectors with local re-orthogonalisation: the FP64 Rayleigh quotient of the Ritz vector
    (combined from the kept basis) is within 1e-8 of the oracle's E0."""
    E = _energies()["torus4x3"]["E0"]
    r = _gpu("torus4x3").lanczos(reorth=1, storage="f32", tol=1e-7, max_iter=300, refine=1)
    assert abs(r["E0_refined"] - E) <= 1e-8 * abs(E), (r, E)


def test_reorth_out_of_range_is_rejected():
    import paper_1707_03974_amd as pdz
    with pytest.raises(pdz.PdzError, match="reorth"):
        _gpu("ring8").lanczos(reorth=3)


def test_ritz_vector_is_an_eigenvector():
    torch = torch_cuda()
    w = synth.workload("ring8")
    g = _gpu("ring8")
    y = torch.empty(g.D, dtype=torch.float64, device="cuda")
    r = g.lanczos(ritz=y, tol=1e-12)
    H = oracle.build_csr(oracle.Problem.from_workload(w))
    yh = to_host(y)
    assert abs(np.linalg.norm(yh) - 1) < 1e-12
    assert np.linalg.norm(H @ yh - r["E0_refined"] * yh) < 1e-6
    assert abs(r["E0_refined"] - _energies()["ring8"]["E0"]) < 1e-11


def test_breakdown_gives_exact_eigenvalue():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    g = pdz.Problem(4, [synth.Bond(0, 1, 0.0)], 2.0, 2, 2)
    v0 = torch.zeros(g.D, dtype=torch.float64, device="cuda")
    v0[7] = 1.0
    r = g.lanczos(v0=v0)
    assert r["converged"] == 1 and r["iters"] == 1
    po = oracle.Problem(4, [0], [1], [0.0], 2.0, 2, 2)
    assert r["E0"] == oracle.build_csr(po)[7, 7]


def test_errors_and_noconv():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    g = _gpu("ring8")
    z = torch.zeros(g.D, dtype=torch.float64, device="cuda")
    with pytest.raises(pdz.PdzError) as e:
        g.lanczos(v0=z)
    assert e.value.status == -1
    nan = torch.full((g.D,), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(pdz.PdzError):
        g.lanczos(v0=nan)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(pdz.PdzError):
        g.lanczos(workspace=small)
    r = g.lanczos(max_iter=5, tol=1e-15)
    assert r["status"] == -5 and r["iters"] == 5 and r["converged"] == 0
    E = _energies()["ring8"]["E0"]
    assert r["E0"] > E


def test_padded_rows_keep_every_lanczos_path_exact():
    """Rows of 3,432 down strings are stored with a pitch of 3,456 inside Lanczos (aligned rows for the
    up pass): the seeded start equals the oracle's SplitMix64 vector given as v0, the Ritz vector comes
    back in the basis order as an eigenvector, and the restart, re-orthogonalisation and kept-basis
    paths reach the oracle's energy."""
    torch = torch_cuda()
    g = _ring14()
    assert g.info["D_dn"] == 3432
    E = _ring14_e0()
    v0 = to_dev(oracle.start_vector(77, g.D), torch.float64)
    a = g.lanczos(seed=77, tol=1e-12, max_iter=600)
    b = g.lanczos(v0=v0, tol=1e-12, max_iter=600)
    assert a["E0"] == b["E0"] and a["iters"] == b["iters"], (a, b)
    assert abs(a["E0"] - E) <= 1e-10 * abs(E), (a, E)
    y = torch.empty(g.D, dtype=torch.float64, device="cuda")
    r = g.lanczos(ritz=y, tol=1e-12, max_iter=600)
    assert abs(float(torch.linalg.norm(y)) - 1.0) < 1e-12
    hy = g.hv(y)
    assert float(torch.linalg.norm(hy - r["E0_refined"] * y)) < 1e-6, r
    assert abs(r["E0_refined"] - E) <= 1e-10 * abs(E), (r, E)
    # FP32 run stopped early, FP64 restart from its (padded) Ritz vector
    y2 = torch.empty(g.D, dtype=torch.float64, device="cuda")
    r2 = g.lanczos(storage="f32", tol=1e-12, max_iter=25, refine=2, ritz=y2)
    assert r2["restart_iters"] > 0 and abs(r2["E0_refined"] - E) <= 1e-10 * abs(E), r2
    assert float(torch.linalg.norm(g.hv(y2) - r2["E0_refined"] * y2)) < 1e-5, r2
    for reorth in (1, 2):
        rr = g.lanczos(reorth=reorth, tol=1e-12, max_iter=300)
        assert rr["converged"] == 1 and abs(rr["E0"] - E) <= 1e-9 * abs(E), (reorth, rr, E)
    ya = torch.empty(g.D, dtype=torch.float64, device="cuda")
    yb = torch.empty(g.D, dtype=torch.float64, device="cuda")
    ka = g.lanczos(storage="f32", tol=1e-9, max_iter=400, ritz=ya)
    kb = g.lanczos(storage="f32", tol=1e-9, max_iter=400, ritz=yb, keep_basis=1)
    assert ka["E0_refined"] == kb["E0_refined"] and torch.equal(ya, yb), (ka, kb)
    assert abs(ka["E0_refined"] - E) <= 1e-8 * abs(E), (ka, E)
