"""What the learned start gains: a network trained on ground states at neighbouring U
against seeded random starts, on a 4x4 periodic cluster with 3 + 3 electrons
(D = 313,600), and on the benchmark's own 7 + 7 cluster (D = 1.3e8, the last test).

Ground states at U in {2, 3, 4, 6, 7, 8} come from the library's own Lanczos;
the target is U = 5, which the network never saw.  The energy reference is an
FP64 Lanczos run to 1e-12, itself checked against the oracle's dense-free
Lanczos on the same problem.
"""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import torch_cuda, to_dev

pytestmark = pytest.mark.gpu

LX, LY, N_E = 4, 4, 3


def _make(U):
    import paper_1707_03974_amd as pdz
    return pdz.Problem(LX * LY, synth.torus(LX, LY, 1.0), U, N_E, N_E)


@pytest.fixture(scope="module")
def trained():
    torch_cuda()
    from paper_1707_03974_amd import learned
    states = learned.ground_states(_make, [2.0, 3.0, 4.0, 6.0, 7.0, 8.0], 4.0, tol=1e-10)
    net, losses, _ = learned.train(states, 4.0, steps=1500, batch=4096, lr=2e-3)
    return states, net, losses


def test_reference_energy_matches_oracle():
    p = _make(5.0)
    E = p.lanczos(tol=1e-12, max_iter=800)["E0"]
    bonds = synth.torus(LX, LY, 1.0)
    po = oracle.Problem(LX * LY, [b.i for b in bonds], [b.j for b in bonds], [b.t for b in bonds], 5.0, N_E, N_E)
    H = oracle.build_csr(po)
    r = oracle.lanczos(lambda x: H @ x, oracle.start_vector(1, po.D), max_iter=400, tol=1e-12, reorth=False)
    assert abs(E - r.E0) <= 1e-9 * abs(r.E0)


def test_training_loss_falls(trained):
    _, _, losses = trained
    assert losses[-1][1] < 0.1 * losses[0][1], losses


def test_learned_start_needs_fewer_lanczos_steps_than_random_starts(trained):
    torch = torch_cuda()
    from paper_1707_03974_amd import learned, mlp
    _, net, _ = trained
    p = _make(5.0)
    E = p.lanczos(tol=1e-12, max_iter=800)["E0"]
    res, v0 = learned.compare(p, net, E, seeds=(1, 2, 3, 4, 5))
    k_learned = res["learned"]["iters"]
    k_random = [r["iters"] for r in res["random"]]
    assert k_learned is not None and None not in k_random
    assert k_learned < min(k_random), res
    # the start vector itself: overlap with the U = 5 ground state
    y = torch.empty(p.D, dtype=torch.float64, device="cuda")
    p.lanczos(ritz=y, tol=1e-10, max_iter=800)
    ov_learned = abs(mlp.dot(v0, y)) / mlp.dot(v0, v0) ** 0.5
    rv = to_dev(synth.random_vector(p.D, 1), torch.float64)
    ov_random = abs(mlp.dot(rv, y)) / mlp.dot(rv, rv) ** 0.5
    assert ov_learned > 100 * ov_random, (ov_learned, ov_random)


def test_lanczos_from_the_learned_start_reaches_the_same_energy(trained):
    from paper_1707_03974_amd import mlp
    import torch
    _, net, _ = trained
    p = _make(5.0)
    E = p.lanczos(tol=1e-12, max_iter=800)["E0"]
    r = p.lanczos(v0=mlp.start_vector(p, net, torch.float64), tol=1e-12, max_iter=800)
    assert r["converged"] == 1 and abs(r["E0"] - E) <= 1e-10 * abs(E)


def test_learned_start_gain_on_the_full_size_7p7_cluster():
    """The benchmark's learned-start workload itself: 4x4 periodic NN, 7 + 7, U = 5 (D = 130,873,600), the
    network trained on ground states at U in {2, 3, 4, 6, 7, 8} as the benchmark trains it.  Fewer Lanczos
    steps to E0 within 1e-8 than every one of five seeded random starts, a start vector with more than 100x
    the random start's overlap with the U = 5 ground state, and the energy from the learned start equal to
    the CPU oracle's stored E0 within 1e-9."""
    import json
    import os
    torch = torch_cuda()
    import paper_1707_03974_amd as pdz
    from paper_1707_03974_amd import learned, mlp
    w = synth.workload("torus4x4_n7")

    def make(U):
        return pdz.Problem(w.n_sites, w.bonds, U, w.n_up, w.n_dn)

    with open(os.path.join(os.path.dirname(__file__), "golden", "energies_fullsize.json")) as f:
        E_oracle = json.load(f)["torus4x4_n7"]["E0"]
    states = learned.ground_states(make, [2.0, 3.0, 4.0, 6.0, 7.0, 8.0], 4.0, tol=1e-10)
    net, losses, _ = learned.train(states, 4.0, steps=3000, batch=4096, lr=2e-3)
    for q, _, _ in states.values():
        q.close()
    del states
    assert losses[-1][1] < 0.1 * losses[0][1], losses
    p = make(w.U)
    v0 = mlp.start_vector(p, net, torch.float64)
    k_learned = learned.iterations_to(p, E_oracle, 1e-8, v0=v0)
    k_random = [learned.iterations_to(p, E_oracle, 1e-8, seed=s) for s in (1, 2, 3, 4, 5)]
    assert k_learned is not None and None not in k_random
    assert k_learned < min(k_random), (k_learned, k_random)
    r = p.lanczos(v0=v0, tol=1e-11, max_iter=800)
    assert r["converged"] == 1 and abs(r["E0"] - E_oracle) <= 1e-9 * abs(E_oracle), (r["E0"], E_oracle)
    y = torch.empty(p.D, dtype=torch.float64, device="cuda")
    p.lanczos(ritz=y, tol=1e-10, max_iter=800)
    ov_learned = abs(mlp.dot(v0, y)) / mlp.dot(v0, v0) ** 0.5
    rv = to_dev(synth.random_vector(p.D, 1), torch.float64)
    ov_random = abs(mlp.dot(rv, y)) / mlp.dot(rv, rv) ** 0.5
    assert ov_learned > 100 * ov_random, (ov_learned, ov_random)
    p.close()
