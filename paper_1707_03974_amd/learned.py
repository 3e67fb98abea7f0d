"""Learned Lanczos start: ground states at neighbouring U, training, inference, comparison.

A driver over libpdz calls only: the Lanczos solves, the |psi|^2 sampler, the
network's forward/backward/Adam kernels and the start-vector inference all
run in the HIP library.

Recipe (the network and loss are defined in include/pdz.h):
  1. ground states psi_U at the training U values; psi at the reference U
     from the seeded random start, the others started from psi_ref, so that
     a degenerate ground space gives consistent vectors, and each psi_U
     gauge-fixed to <psi_U, psi_ref> > 0;
  2. Adam on minibatches drawn with probability |psi_U|^2, cycling over U;
  3. the start vector over the whole basis of the target problem.
"""
import time

from . import mlp


def ground_states(make_problem, Us, ref_U, tol=1e-10, max_iter=800, seed=1):
    """{U: (problem, psi (FP64 device), lanczos result)}; psi is normalised."""
    import torch
    out = {}
    p = make_problem(ref_U)
    y = torch.empty(p.D, dtype=torch.float64, device="cuda")
    out[ref_U] = (p, y, p.lanczos(ritz=y, tol=tol, max_iter=max_iter, seed=seed))
    for U in Us:
        if U == ref_U:
            continue
        q = make_problem(U)
        z = torch.empty(q.D, dtype=torch.float64, device="cuda")
        out[U] = (q, z, q.lanczos(v0=y, ritz=z, tol=tol, max_iter=max_iter))
    return out


def train(states, ref_U, steps=3000, batch=4096, lr=2e-3, lr_final=2e-4, seed=7, log_every=250):
    """Train a network on the ground states; returns (net, losses, seconds)."""
    import torch
    ref = states[ref_U][1]
    samplers = []
    for U, (p, psi, _) in sorted(states.items()):
        gauge = 1.0 if mlp.dot(psi, ref) >= 0.0 else -1.0
        samplers.append(mlp.Sampler(p, psi, gauge=gauge))
    net = mlp.Net(seed=seed)
    tr = mlp.Trainer(net, batch)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        s = samplers[it % len(samplers)]
        s.draw(seed, it * batch, tr.occ, tr.target)
        tr.gradient()
        frac = it / max(1, steps - 1)
        net.adam(tr.grad, lr * (lr_final / lr) ** frac)   # geometric decay
        if it % log_every == 0 or it == steps - 1:
            losses.append((it, tr.loss.item()))
    torch.cuda.synchronize()
    return net, losses, time.perf_counter() - t0


def iterations_to(problem, E_ref, rel, v0=None, seed=1, max_iter=800):
    """First Lanczos step whose Ritz value is within rel of E_ref (FP64 history), or None."""
    r = problem.lanczos(v0=v0, seed=seed, tol=0.0, max_iter=max_iter, history=True)
    return next((k + 1 for k, th in enumerate(r["thetas"]) if abs(th - E_ref) <= rel * abs(E_ref)), None)


def timed_solve(problem, k, v0=None, seed=1):
    """Wall time of exactly k FP64 Lanczos steps from v0 (or the seeded start)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = problem.lanczos(v0=v0, seed=seed, tol=0.0, max_iter=k)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def compare(problem, net, E_ref, seeds=(1, 2, 3, 4, 5), rel=1e-8, max_iter=800):
    """Learned start (inference included in its time) against seeded random starts."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v0 = mlp.start_vector(problem, net, torch.float64)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    k_l = iterations_to(problem, E_ref, rel, v0=v0, max_iter=max_iter)
    out = {"inference_s": t_inf, "learned": {"iters": k_l}}
    if k_l is not None:
        t, _ = timed_solve(problem, k_l, v0=v0)
        out["learned"]["solve_s"] = t
        out["learned"]["total_s"] = t + t_inf
    rnd = []
    for s in seeds:
        k = iterations_to(problem, E_ref, rel, seed=s, max_iter=max_iter)
        entry = {"seed": s, "iters": k}
        if k is not None:
            entry["solve_s"] = timed_solve(problem, k, seed=s)[0]
        rnd.append(entry)
    out["random"] = rnd
    return out, v0
