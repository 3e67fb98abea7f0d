"""Write tests/golden/energies.json: ground-state energies computed by the oracle only.

Each entry records how it was obtained: dense LAPACK eigensolver for small D,
otherwise the oracle's Lanczos (full re-orthogonalisation, tol 1e-13)
cross-checked against ARPACK on the oracle's CSR matrix.
Run:  python tests/golden/make_energies.py
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402


def energy(w):
    p = oracle.Problem.from_workload(w)
    H = oracle.build_csr(p)
    if p.D <= 6000:
        E = float(np.linalg.eigvalsh(H.toarray())[0])
        return {"E0": E, "method": "dense LAPACK eigvalsh of the oracle CSR", "D": p.D}
    r = oracle.lanczos(lambda x: H @ x, oracle.start_vector(1, p.D), max_iter=600, tol=1e-13)
    Ea = float(spla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0])
    assert r.converged and abs(r.E0 - Ea) <= 1e-10 * abs(Ea), (w.name, r.E0, Ea)
    return {"E0": r.E0, "E0_arpack": Ea, "iters": r.iters,
            "method": "oracle Lanczos (full reorth, tol 1e-13), ARPACK cross-check", "D": p.D}


def main():
    out = {"_about": "Ground-state energies from the CPU oracle (tests/golden/make_energies.py)."}
    names = ["two_site", "ring8", "torus4x3"]
    for n in names:
        t = time.time()
        out[n] = energy(synth.workload(n))
        print(n, out[n], f"{time.time() - t:.1f}s", flush=True)
    batch = {}
    for w in synth.batched_workloads():
        t = time.time()
        batch[w.name] = energy(w)
        batch[w.name].update({"U": w.U, "n_up": w.n_up, "n_dn": w.n_dn, "n_sites": w.n_sites})
        print(w.name, batch[w.name]["E0"], f"{time.time() - t:.1f}s", flush=True)
    out["batched"] = batch
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "energies.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
