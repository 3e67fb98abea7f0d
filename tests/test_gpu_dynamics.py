"""Fermion operators between sectors and the continued-fraction resolvent (libpdz) against the oracle.

The operator is a signed map of one basis onto another: equal to the oracle's explicit operator
algebra bit for bit.  The resolvent from the Lanczos coefficients is compared with the oracle's
spectral sum over a dense eigendecomposition of the target sector's H.
"""
import numpy as np
import pytest

import oracle
from oracle import dynamics as ody
import synth
from tests._gpu import torch_cuda, to_dev, to_host

pytestmark = pytest.mark.gpu


def _problems(w, nu, nd):
    import paper_1707_03974_amd as pdz
    return pdz.Problem(w.n_sites, w.bonds, w.U, nu, nd)


@pytest.mark.parametrize("name", ["ring8", "torus4x3"])
@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_fermion_operators_equal_the_oracle_bit_for_bit(name, dtype_name):
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    w = synth.workload(name)
    src = pdz.Problem.from_workload(w)
    dt = torch.float64 if dtype_name == "f64" else torch.float32
    x = synth.random_vector(src.D, 11).astype(np.float32 if dtype_name == "f32" else np.float64)
    xd = to_dev(x, dt)
    sites = range(w.n_sites) if name == "ring8" else (0, 5, w.n_sites - 1)
    for spin in (0, 1):
        for op in (0, 1):
            tu = w.n_up + ((-1 if op == 0 else 1) if spin == 0 else 0)
            td = w.n_dn + ((-1 if op == 0 else 1) if spin == 1 else 0)
            dst = _problems(w, tu, td)
            for site in sites:
                y = to_host(pdz.fermion_op(src, dst, site, spin, op, xd))
                e = ody.apply_fermion(w.n_sites, w.n_up, w.n_dn, site, spin, op, x.astype(np.float64))
                assert y.shape == e.shape
                assert np.array_equal(y.astype(np.float64), e), (name, site, spin, op)


def test_fermion_operator_argument_checks():
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    w = synth.workload("ring8")
    src = pdz.Problem.from_workload(w)
    dst = _problems(w, w.n_up - 1, w.n_dn)
    x = torch.zeros(src.D, dtype=torch.float64, device="cuda")
    with pytest.raises(pdz.PdzError):
        pdz.fermion_op(src, dst, 0, 1, 0, x)          # dst is not the down-removal sector
    with pytest.raises(pdz.PdzError):
        pdz.fermion_op(src, dst, 8, 0, 0, x)          # site out of range
    with pytest.raises(pdz.PdzError):
        pdz.fermion_op(src, dst, 0, 0, 1, x)          # creation needs one electron more
    with pytest.raises(pdz.PdzError):
        pdz.fermion_op(src, dst, 0, 0, 0, x, y=x)     # overlap


@pytest.mark.parametrize("spin,op", [(0, 0), (1, 1)])
def test_continued_fraction_resolvent_matches_the_spectral_sum(spin, op):
    """Removal (c_up) and addition (c+_dn) parts on the 8-site ring from the library's ground state."""
    torch = torch_cuda()
    from paper_1707_03974_amd import dynamics
    w = synth.workload("ring8")
    g = _problems(w, w.n_up, w.n_dn)
    psi = torch.empty(g.D, dtype=torch.float64, device="cuda")
    r0 = g.lanczos(ritz=psi, tol=1e-12, max_iter=400)
    pts = np.linspace(-8.0, 8.0, 33) + 0.25j
    R, res = dynamics.resolvent(g, psi, 3, spin, op, pts, steps=300)   # converges geometrically: 8e-11 at 300
    po = oracle.Problem.from_workload(w)
    tu, td = ody.target_fillings(w.n_up, w.n_dn, spin, op)
    pt = oracle.Problem(po.n_sites, po.bond_i, po.bond_j, po.bond_t, po.U, tu, td)
    H = oracle.build_csr(pt)
    phi = ody.apply_fermion(w.n_sites, w.n_up, w.n_dn, 3, spin, op, to_host(psi))
    E = ody.resolvent_exact(H, phi, pts)
    assert abs(res["norm0"] ** 2 - phi @ phi) <= 1e-12
    err = np.abs(R - E) / np.abs(E)
    assert err.max() <= 1e-8, float(err.max())
    assert r0["converged"] == 1
