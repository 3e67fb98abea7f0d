"""Write tests/golden/energies_fullsize.json: ground-state energies of the two
full-size 4x4 problems, computed by the oracle only.

Workloads: the 4x4 periodic cluster with NN (t = 1) and NNN (t' = -0.3)
hopping at 8 + 8 electrons, U = 6 (D = 165,636,900), and the 4x4 periodic NN
cluster at 7 + 7, U = 5 (D = 130,873,600).

Method: the oracle's textbook Lanczos (oracle.lanczos, no re-orthogonalisation:
at this D the basis would not fit host memory) from the SplitMix64 start of
seed 1, stopped when beta_{k+1} |s_k| <= 1e-11 |theta|, on the oracle's
tensor-product H.v (oracle.kron: per-spin matrices assembled by operator
algebra and binary search).  Before the run, that product is compared with
the element-wise oracle (oracle.cmf, binary search per nonzero) on sampled
row blocks; the largest deviation relative to the row's sum of |terms| is
recorded.  CPU only; about 15 minutes per problem on 8 threads.

Run:  python tests/golden/make_energies_fullsize.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402
from oracle.cmf import MatrixFree  # noqa: E402
from oracle.kron import KronH      # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "energies_fullsize.json")
NAMES = ["torus4x4_nnn", "torus4x4_n7"]


def cross_check(p, K, blocks=6, rows=2000, seed=7):
    """Largest |kron - element-wise| / sum|terms| over sampled row blocks."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, p.D)
    xa = np.abs(x)
    mf = MatrixFree(p)
    Ka = KronH(p)
    Ka.Tup = abs(K.Tup)
    Ka.TdnT = abs(K.TdnT)
    Ka.p = oracle.Problem(p.n_sites, p.bond_i, p.bond_j, p.bond_t, abs(p.U), p.n_up, p.n_dn)
    X, XA = x.reshape(K.Du, K.Dd), xa.reshape(K.Du, K.Dd)
    worst = 0.0
    for r0 in rng.integers(0, K.Du - 1, blocks):
        u0 = int(r0)
        u1 = min(K.Du, u0 + max(1, rows // K.Dd))
        yk = K.rows(X, u0, u1).reshape(-1)
        ya = Ka.rows(XA, u0, u1).reshape(-1)
        ye = mf.rows(x, u0 * K.Dd, u1 * K.Dd)
        worst = max(worst, float(np.max(np.abs(yk - ye) / np.maximum(ya, 1e-300))))
    return worst


def main(names):
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    out["_about"] = ("Ground-state energies of the full-size 4x4 problems from the CPU oracle "
                     "(tests/golden/make_energies_fullsize.py).")
    for name in names:
        w = synth.workload(name)
        p = oracle.Problem.from_workload(w)
        K = KronH(p)
        dev = cross_check(p, K)
        print(f"{name}: D={p.D} tensor-product H.v vs element-wise oracle, max dev / sum|terms| = {dev:.2e}",
              flush=True)
        assert dev <= 1e-13, dev
        t0 = time.time()
        calls = [0]

        def hv(v):
            calls[0] += 1
            y = K(v)
            if calls[0] % 10 == 0:
                print(f"  {name}: {calls[0]} H.v, {time.time() - t0:.0f} s", flush=True)
            return y

        r = oracle.lanczos(hv, oracle.start_vector(1, p.D), max_iter=500, tol=1e-11, reorth=False)
        secs = time.time() - t0
        out[name] = {"E0": r.E0, "iters": r.iters, "converged": bool(r.converged), "resid_est": r.resid_est,
                     "thetas_last": r.thetas[-5:], "D": p.D, "U": w.U, "n_up": w.n_up, "n_dn": w.n_dn,
                     "seconds": secs, "threads": K.nthreads, "hv_crosscheck_max_rel_dev": dev,
                     "method": ("oracle Lanczos (no re-orthogonalisation, SplitMix64 seed 1, stop at "
                                "beta|s_k| <= 1e-11 |theta|) on the oracle tensor-product H.v, which was "
                                "checked against the element-wise binary-search oracle on sampled rows")}
        print(name, out[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or NAMES)
