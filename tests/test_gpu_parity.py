"""Inversion-parity subspaces (Sec. IV.B) on the GPU against the CPU oracle.

* The device basis and the oracle's hold the same representative states; rows
  (up representatives) come in the decision tree's order on both sides, and a
  state's position inside its row is the layout's choice, so every comparison
  goes through the state a position holds (pdz_parity_unrank).  pdz_parity_rank
  inverts pdz_parity_unrank; states outside the basis are flagged.
* H.v element by element against B^T H B (small sectors) and on sampled rows of
  the 4x3 torus 6+6 and of the 4x4 NN+NNN 8+8 cluster (oracle rows from the
  real-space operator algebra), FP64 and FP32.  Tolerance: (n + 6) eps sum|terms|:
  each term is a product of up to five rounded factors (sqrt(2), 1/sqrt(2), the
  hop amplitude, x, and the sign P sigma, which is exact), and n - 1 roundings of
  the running sum.
* Lanczos on each parity: E0 against the oracle's H_P, and min over the two
  parities of the 4x4 NN+NNN 8+8 cluster equals the real-space ground-state
  energy from the real-space path.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
import synth
from oracle import inversion as inv
from tests._gpu import torch_cuda, to_dev, to_host, EPS64, EPS32

pytestmark = pytest.mark.gpu


def _chain(N, t=1.0, tp=0.0, periodic=False):
    b = [(i, i + 1, t) for i in range(N - 1)]
    if periodic:
        b.append((N - 1, 0, t))
    if tp:
        b += [(i, i + 2, tp) for i in range(N - 2)]
    return b


def _open_rect(Lx, Ly, t=1.0, tp=0.0):
    b = []
    for y in range(Ly):
        for x in range(Lx):
            s = x + Lx * y
            if x + 1 < Lx:
                b.append((s, s + 1, t))
            if y + 1 < Ly:
                b.append((s, s + Lx, t))
            if tp and x + 1 < Lx and y + 1 < Ly:
                b.append((s, s + Lx + 1, tp))
            if tp and x >= 1 and y + 1 < Ly:
                b.append((s, s + Lx - 1, tp))
    return b


SMALL = [
    (8, _chain(8), 4.0, 4, 4),
    (7, _chain(7, 1.0, 0.3), 3.0, 3, 2),
    (9, _open_rect(3, 3, 1.0, 0.2), 5.0, 3, 3),
    (8, _open_rect(4, 2), 6.0, 3, 4),
    (8, _chain(8, periodic=True), 2.0, 4, 3),
    (6, _chain(6), 3.0, 0, 3),
    (10, _open_rect(5, 2, 1.0, -0.25), 4.0, 5, 5),
]
IDS = ["chain8", "chain7nnn", "open3x3", "open4x2", "ring8", "nup0", "open5x2"]


def _oracle(N, bonds, U, nu, nd):
    return oracle.Problem(N, [b[0] for b in bonds], [b[1] for b in bonds], [b[2] for b in bonds], U, nu, nd)


def _gpu(N, bonds, U, nu, nd, P):
    import paper_1707_03974_amd as pdz
    return pdz.ParityProblem(N, bonds, U, nu, nd, P)


def _perm(g, N, nu, nd, P):
    """Oracle basis index of the state at every device position (asserted to be a bijection)."""
    torch = torch_cuda()
    bu, bd, _ = inv.basis(N, nu, nd, P)
    assert g.D == len(bu)
    gu, gd = g.unrank(torch.arange(g.D, dtype=torch.int64, device="cuda"))
    gu = to_host(gu).view(np.uint32).astype(np.uint64)
    gd = to_host(gd).view(np.uint32).astype(np.uint64)
    where = {(int(u), int(d)): k for k, (u, d) in enumerate(zip(bu, bd))}
    perm = np.array([where.get((int(u), int(d)), -1) for u, d in zip(gu, gd)], dtype=np.int64)
    assert np.all(perm >= 0) and len(np.unique(perm)) == len(perm), "device basis differs from the oracle's"
    return perm, gu, bu


@pytest.mark.parametrize("P", [1, -1])
@pytest.mark.parametrize("case", SMALL, ids=IDS)
def test_parity_maps_equal_the_oracle_basis(case, P):
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    N, bonds, U, nu, nd = case
    g = _gpu(N, bonds, U, nu, nd, P)
    perm, gu, bu = _perm(g, N, nu, nd, P)
    assert np.array_equal(gu, bu)          # rows: up representatives in tree order, equal lengths
    gu2, gd2 = g.unrank(torch.arange(g.D, dtype=torch.int64, device="cuda"))
    r = g.rank(gu2, gd2)
    assert torch.equal(r, torch.arange(g.D, dtype=torch.int64, device="cuda"))
    assert pdz.device_errors() == 0


def test_parity_rank_flags_states_outside_the_basis():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    g = _gpu(8, _chain(8), 4.0, 4, 4, 1)
    pdz.device_errors()
    up = np.array([0b00001111, 0b11110000, 0b00111100], np.uint32)   # A string, its image, a palindrome
    dn = np.array([0b01010101, 0b01010101, 0b00111100], np.uint32)   # ..., ..., palindrome: self-mapped
    r = to_host(g.rank(to_dev(up.view(np.int32), torch.int32), to_dev(dn.view(np.int32), torch.int32)))
    assert r[0] >= 0 and r[1] == -1
    sigma = (-1) ** (4 * 3 // 2 + 4 * 3 // 2)
    assert (r[2] >= 0) == (sigma == 1)
    assert pdz.device_errors() & 1
    gu, _ = g.unrank(torch.tensor([g.D], dtype=torch.int64, device="cuda"))
    assert to_host(gu)[0] == -1
    assert pdz.device_errors() & 2


def _bound(H, x, eps):
    A = abs(H)
    s = A @ abs(x)
    n = np.diff(H.indptr)
    return (n + 6) * eps * s + n * EPS64 * s


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("P", [1, -1])
@pytest.mark.parametrize("case", SMALL, ids=IDS)
def test_parity_hv_matches_the_oracle(case, P, dtype_name):
    torch = torch_cuda()
    N, bonds, U, nu, nd = case
    HP = inv.build_csr_P(_oracle(N, bonds, U, nu, nd), P)
    g = _gpu(N, bonds, U, nu, nd, P)
    dt, e = (torch.float64, EPS64) if dtype_name == "f64" else (torch.float32, EPS32)
    x = np.random.default_rng(12).uniform(-1, 1, g.D)
    if dtype_name == "f32":
        x = x.astype(np.float32).astype(np.float64)
    _check_hv(g, HP, x, dt, e, _perm(g, N, nu, nd, P)[0], (dtype_name, P))


def _check_hv(g, HP, x, dt, e, perm, what):
    """Device y = H x against B^T H B, each device position compared with the oracle row of its state."""
    xo = np.zeros_like(x)
    xo[perm] = x
    y = to_host(g.hv(to_dev(x, dt))).astype(np.float64)
    want = (HP @ xo)[perm]
    err = np.abs(y - want)
    assert np.all(err <= _bound(HP, xo, e)[perm] + 1e-300), (np.max(err), what)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("case", [SMALL[0], SMALL[3], SMALL[6]], ids=["chain8", "open4x2", "open5x2"])
def test_parity_one_pass_gather_kernel_matches_the_oracle(case, dtype_name, monkeypatch):
    """The one-pass kernel that serves rows too long for the two-pass form, forced on small rows."""
    torch = torch_cuda()
    N, bonds, U, nu, nd = case
    monkeypatch.setenv("PDZ_PARITY_GATHER", "1")
    for P in (1, -1):
        HP = inv.build_csr_P(_oracle(N, bonds, U, nu, nd), P)
        g = _gpu(N, bonds, U, nu, nd, P)
        dt, e = (torch.float64, EPS64) if dtype_name == "f64" else (torch.float32, EPS32)
        x = np.random.default_rng(21).uniform(-1, 1, g.D)
        if dtype_name == "f32":
            x = x.astype(np.float32).astype(np.float64)
        _check_hv(g, HP, x, dt, e, _perm(g, N, nu, nd, P)[0], (dtype_name, P))


@pytest.mark.parametrize("lanes", ["16", "32"])
@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("case", [SMALL[0], SMALL[1], SMALL[6]], ids=["chain8", "chain7nnn", "open5x2"])
def test_parity_up_pass_slab_widths_match_the_oracle(case, dtype_name, lanes, monkeypatch):
    """The up pass at 16 and 32 lanes per row (narrower slabs, several rows per wave) against B^T H B."""
    torch = torch_cuda()
    N, bonds, U, nu, nd = case
    monkeypatch.setenv("PDZ_PARITY_UP_LANES", lanes)
    for P in (1, -1):
        HP = inv.build_csr_P(_oracle(N, bonds, U, nu, nd), P)
        g = _gpu(N, bonds, U, nu, nd, P)
        dt, e = (torch.float64, EPS64) if dtype_name == "f64" else (torch.float32, EPS32)
        x = np.random.default_rng(23).uniform(-1, 1, g.D)
        if dtype_name == "f32":
            x = x.astype(np.float32).astype(np.float64)
        _check_hv(g, HP, x, dt, e, _perm(g, N, nu, nd, P)[0], (dtype_name, P, lanes))


def test_parity_up_pass_lanes_must_be_16_32_or_64(monkeypatch):
    torch_cuda()
    monkeypatch.setenv("PDZ_PARITY_UP_LANES", "48")
    with pytest.raises(Exception, match="PDZ_PARITY_UP_LANES"):
        _gpu(8, _chain(8), 4.0, 4, 4, 1)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("case", [SMALL[0], SMALL[1], SMALL[6]], ids=["chain8", "chain7nnn", "open5x2"])
def test_parity_down_pass_32bit_table_matches_the_oracle(case, dtype_name, monkeypatch):
    """The down pass on its 32-bit hop table (the form for sectors whose columns do not fit 16-bit entries)."""
    torch = torch_cuda()
    N, bonds, U, nu, nd = case
    monkeypatch.setenv("PDZ_PARITY_WIDE_TABLE", "1")
    for P in (1, -1):
        HP = inv.build_csr_P(_oracle(N, bonds, U, nu, nd), P)
        g = _gpu(N, bonds, U, nu, nd, P)
        dt, e = (torch.float64, EPS64) if dtype_name == "f64" else (torch.float32, EPS32)
        x = np.random.default_rng(29).uniform(-1, 1, g.D)
        if dtype_name == "f32":
            x = x.astype(np.float32).astype(np.float64)
        _check_hv(g, HP, x, dt, e, _perm(g, N, nu, nd, P)[0], (dtype_name, P))


def _sampled(w, P, nrows, seed, dtype_name):
    torch = torch_cuda()
    po = oracle.Problem.from_workload(w)
    g = _gpu(w.n_sites, [(b.i, b.j, b.t) for b in w.bonds], w.U, w.n_up, w.n_dn, P)
    ridx = inv.RowIndex(w.n_sites, w.n_up, w.n_dn, P)
    assert ridx.D == g.D
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, g.D)
    dt, e = (torch.float64, EPS64) if dtype_name == "f64" else (torch.float32, EPS32)
    if dtype_name == "f32":
        x = x.astype(np.float32).astype(np.float64)
    y = to_host(g.hv(to_dev(x, dt))).astype(np.float64)
    rows = np.unique(np.concatenate([rng.integers(0, g.D, nrows), [0, g.D - 1]]))
    gu, gd = g.unrank(to_dev(rows, torch.int64))
    ru, rd = to_host(gu).view(np.uint32), to_host(gd).view(np.uint32)
    assert all(inv.representative(u, d, w.n_sites)[:2] == (int(u), int(d)) for u, d in zip(ru, rd))

    def lookup(uu, dd):
        """x at the device position of each listed representative state (its rank)."""
        k = to_host(g.rank(to_dev(uu.astype(np.uint32).view(np.int32), torch.int32),
                           to_dev(dd.astype(np.uint32).view(np.int32), torch.int32)))
        assert np.all(k >= 0), "a source state is missing from the device basis"
        return x[k]

    want, a, n = inv.hv_rows_P(po, P, lookup, ru, rd)
    bound = (n + 6) * e * a + n * EPS64 * a
    err = np.abs(y[rows] - want)
    assert np.all(err <= bound), (np.max(err - bound), dtype_name, P)
    return g


@pytest.mark.parametrize("P", [1, -1])
def test_parity_hv_sampled_rows_torus4x3(P):
    _sampled(synth.workload("torus4x3"), P, 150, 3, "f64")


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_parity_hv_full_size_sampled_rows(dtype_name):
    g = _sampled(synth.workload("torus4x4_nnn"), 1, 60, 8, dtype_name)
    assert g.D > 80_000_000


@pytest.mark.parametrize("case", [SMALL[0], SMALL[2], SMALL[3], SMALL[6]], ids=["chain8", "open3x3", "open4x2", "open5x2"])
def test_parity_lanczos_E0_matches_the_oracle(case):
    N, bonds, U, nu, nd = case
    po = _oracle(N, bonds, U, nu, nd)
    for P in (1, -1):
        HP = inv.build_csr_P(po, P)
        v0 = np.random.default_rng(2).uniform(-1, 1, HP.shape[0])
        e0 = sla.eigsh(HP, k=1, which="SA", v0=v0, tol=1e-13)[0][0] if HP.shape[0] > 64 else \
            np.linalg.eigvalsh(HP.toarray())[0]
        g = _gpu(N, bonds, U, nu, nd, P)
        r = g.lanczos(storage="f64", tol=1e-12, max_iter=min(400, g.D + 2))
        assert abs(r["E0"] - e0) <= 1e-9 * max(1.0, abs(e0)), (P, r["E0"], e0)


@pytest.mark.parametrize("mode", ["f32_keep", "f32_regen", "f64_graph_off", "f64_reorth"])
def test_parity_lanczos_modes_match_the_oracle(mode):
    """The recurrence fused into the parity down pass (FP32 storage with kept or regenerated vectors for the
    FP64 refinement, FP64 without graphs) and the unfused step of full re-orthogonalisation, against the oracle."""
    N, bonds, U, nu, nd = SMALL[6]
    po = _oracle(N, bonds, U, nu, nd)
    kw = {"f32_keep": dict(storage="f32", tol=1e-7, refine=1, keep_basis=1),
          "f32_regen": dict(storage="f32", tol=1e-7, refine=1, keep_basis=0),
          "f64_graph_off": dict(storage="f64", tol=1e-12, use_graph=0),
          "f64_reorth": dict(storage="f64", tol=1e-12, reorth=2)}[mode]
    for P in (1, -1):
        HP = inv.build_csr_P(po, P)
        v0 = np.random.default_rng(2).uniform(-1, 1, HP.shape[0])
        e0 = sla.eigsh(HP, k=1, which="SA", v0=v0, tol=1e-13)[0][0]
        g = _gpu(N, bonds, U, nu, nd, P)
        r = g.lanczos(max_iter=300, **kw)
        e = r["E0_refined"] if mode.startswith("f32") else r["E0"]
        assert abs(e - e0) <= 1e-8 * max(1.0, abs(e0)), (mode, P, e, e0)


def test_parity_lanczos_on_the_one_pass_kernel_matches_the_oracle(monkeypatch):
    """Forced one-pass form: no x . y partials from the H.v, so alpha takes the separate dot kernel."""
    N, bonds, U, nu, nd = SMALL[6]
    monkeypatch.setenv("PDZ_PARITY_GATHER", "1")
    po = _oracle(N, bonds, U, nu, nd)
    for P in (1, -1):
        HP = inv.build_csr_P(po, P)
        v0 = np.random.default_rng(2).uniform(-1, 1, HP.shape[0])
        e0 = sla.eigsh(HP, k=1, which="SA", v0=v0, tol=1e-13)[0][0]
        g = _gpu(N, bonds, U, nu, nd, P)
        r = g.lanczos(storage="f64", tol=1e-12, max_iter=min(400, g.D + 2))
        assert abs(r["E0"] - e0) <= 1e-9 * max(1.0, abs(e0)), (P, r["E0"], e0)


def test_lowest_parity_is_the_real_space_ground_state():
    """4x4 NN+NNN torus (point inversion through the centre), 8+8, U = 6: the lower parity's E0 equals the
    real-space E0, and, in the parity the benchmark times (P = +1, the ground state), FP64 Lanczos and FP32
    Lanczos with the FP64 refinement (the recurrence fused into the scheduled down pass in both) reach the CPU
    oracle's stored E0 within 1e-9 and 1e-8."""
    import json
    import os
    torch_cuda()
    import paper_1707_03974_amd as pdz
    w = synth.workload("torus4x4_nnn")
    with open(os.path.join(os.path.dirname(__file__), "golden", "energies_fullsize.json")) as f:
        e_oracle = json.load(f)["torus4x4_nnn"]["E0"]
    real = pdz.Problem.from_workload(w)
    e_real = real.lanczos(storage="f64", tol=1e-11, max_iter=400)["E0"]
    real.close()
    e = []
    for P in (1, -1):
        g = pdz.ParityProblem.from_workload(w, P)
        e.append(g.lanczos(storage="f64", tol=1e-11, max_iter=400)["E0"])
        if P == 1:
            e32 = g.lanczos(storage="f32", tol=1e-7, max_iter=400, refine=1, keep_basis=1)["E0_refined"]
        g.close()
    assert abs(min(e) - e_real) <= 1e-8 * abs(e_real), (e, e_real)
    assert abs(e[0] - e_oracle) <= 1e-9 * abs(e_oracle), (e[0], e_oracle)
    assert abs(e32 - e_oracle) <= 1e-8 * abs(e_oracle), (e32, e_oracle)


def _chain14():
    """Open 14-site chain with NNN hops (two hop magnitudes), 7+7: full rows of C(14,7) = 3432 columns, long
    enough for the gather-scheduled down pass; palindromic rows split the full rows into runs of every length."""
    from synth.lattices import Bond
    from synth.workloads import Workload
    return Workload("chain14nnn", 14, [Bond(i, j, t) for i, j, t in _chain(14, 1.0, -0.35)], 5.0, 7, 7)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("P", [1, -1])
def test_parity_scheduled_down_pass_sampled_rows(P, dtype_name):
    _sampled(_chain14(), P, 200, 13, dtype_name)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_parity_scheduled_and_looped_down_passes_agree(dtype_name, monkeypatch):
    """The whole H.v from the scheduled down pass and from the looped one (PDZ_PARITY_LOOPED_DOWN=1) on every
    element: each is within (n + 6) eps sum|terms| of the exact value, so they are within twice that of each
    other; sum|terms| <= (U n_dn + sqrt(2) * 2 * (hops per string)) max|x| bounds every element's terms."""
    torch = torch_cuda()
    w = _chain14()
    bonds = [(b.i, b.j, b.t) for b in w.bonds]
    dt, e = (torch.float64, EPS64) if dtype_name == "f64" else (torch.float32, EPS32)
    for P in (1, -1):
        g = _gpu(w.n_sites, bonds, w.U, w.n_up, w.n_dn, P)
        x = np.random.default_rng(31).uniform(-1, 1, g.D)
        y1 = to_host(g.hv(to_dev(x, dt))).astype(np.float64)
        monkeypatch.setenv("PDZ_PARITY_LOOPED_DOWN", "1")
        g2 = _gpu(w.n_sites, bonds, w.U, w.n_up, w.n_dn, P)
        monkeypatch.delenv("PDZ_PARITY_LOOPED_DOWN")
        y2 = to_host(g2.hv(to_dev(x, dt))).astype(np.float64)
        hops = 2 * (2 * 13 + 2 * 12)   # bonds touching a string's electrons, both spins, at most
        n = 1 + hops
        a = (w.U * w.n_dn + np.sqrt(2.0) * hops) * np.max(np.abs(x))
        err = np.max(np.abs(y1 - y2))
        assert err <= 2 * (n + 6) * e * a, (P, dtype_name, err)
        assert err > 0.0 or dtype_name == "f64"   # FP32: the two summation orders differ somewhere
        g.close()
        g2.close()


def test_parity_scheduled_down_pass_lanczos_gives_the_real_space_ground_state(monkeypatch):
    """Lanczos with the recurrence fused into the scheduled parity down pass (FP64 storage, and FP32 storage with
    the FP64 refinement from regenerated or kept vectors): min over the parities is the real-space ground state, and each parity's E0 equals the
    looped down pass's."""
    torch_cuda()
    import paper_1707_03974_amd as pdz
    w = _chain14()
    bonds = [(b.i, b.j, b.t) for b in w.bonds]
    real = pdz.Problem(w.n_sites, bonds, w.U, w.n_up, w.n_dn)
    e_real = real.lanczos(storage="f64", tol=1e-11, max_iter=400)["E0"]
    real.close()
    es = []
    for P in (1, -1):
        g = _gpu(w.n_sites, bonds, w.U, w.n_up, w.n_dn, P)
        e64 = g.lanczos(storage="f64", tol=1e-11, max_iter=400)["E0"]
        e32 = g.lanczos(storage="f32", tol=1e-7, refine=1, keep_basis=0, max_iter=400)["E0_refined"]
        e32k = g.lanczos(storage="f32", tol=1e-7, refine=1, keep_basis=1, max_iter=400)["E0_refined"]
        g.close()
        monkeypatch.setenv("PDZ_PARITY_LOOPED_DOWN", "1")
        g2 = _gpu(w.n_sites, bonds, w.U, w.n_up, w.n_dn, P)
        monkeypatch.delenv("PDZ_PARITY_LOOPED_DOWN")
        e_loop = g2.lanczos(storage="f64", tol=1e-11, max_iter=400)["E0"]
        g2.close()
        assert abs(e64 - e_loop) <= 1e-9 * abs(e_loop), (P, e64, e_loop)
        assert abs(e32 - e64) <= 1e-8 * abs(e64), (P, e32, e64)
        assert abs(e32k - e64) <= 1e-8 * abs(e64), (P, e32k, e64)
        es.append(e64)
    assert abs(min(es) - e_real) <= 1e-9 * abs(e_real), (es, e_real)
