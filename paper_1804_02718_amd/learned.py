"""Learned-preconditioner workload: training pairs from the solver, training,
and flexible PCG against plain CG.  Host orchestration only: the solves,
sample packing, network passes, losses and Adam steps run in the HIP library
(``fl.Batch``, ``fl_unet_pack``, ``fl_unet_train``, ``fl_poisson_solve_ex``).

Workload (2D, (-1, 1)^2, N = 256, n = 255 interior points padded to a
256 x 256 network grid): alpha ~ U(0.3, 1.9), right-hand side a sum of eight
Gaussians (centres U(-0.5, 0.5)^2, widths U(0.05, 0.2)); training seeds
100000 + i, held-out seeds 900000 + i.  A training pair is (f, u) with
A u = f solved to 1e-8 by the batched mixed-precision solver.
"""
import time

import numpy as np

from . import fl, inputs


def _dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def make_pairs(net, N, count, seed0=100000, chunk=64, tol=1e-8, alpha_range=(0.3, 1.9)):
    """count (f, A^{-1} f) pairs from the batched solver, packed into network samples.
    Returns (x [count, H, H, 2], t [count, H, H], alphas, mean solver iterations)."""
    import torch
    H = net.H
    n = N - 1
    x = torch.zeros((count, H, H, 2), dtype=torch.float32, device="cuda:0")
    t = torch.zeros((count, H, H), dtype=torch.float32, device="cuda:0")
    alphas, iters = [], []
    for k in range(0, count, chunk):
        m = min(chunk, count - k)
        probs = [inputs.learned_problem(seed0 + k + j, N=N, alpha_range=alpha_range) for j in range(m)]
        al = [p[0] for p in probs]
        b = fl.Batch(2, [N] * m, al, [2.0 / N] * m)
        fs = [_dev(p[1], torch.float64) for p in probs]
        us, info = b.solve(fs, tol=tol)
        b.close()
        net.pack(fs, us, al, n, x[k:k + m], t[k:k + m])
        alphas += al
        iters += [i["iters"] for i in info]
    return x, t, alphas, float(np.mean(iters)) if iters else 0.0


def train(net, x, t, epochs, batch=16, lr=3e-4, lr_final=2e-5, seed=0):
    """Adam epochs with a cosine learning-rate decay over the whole run; mean loss per epoch."""
    return net.train(x, t, epochs=epochs, batch=batch, lr=lr, lr_final=lr_final, seed=seed)


def compare(net, N, seeds, tol=1e-8, reps=2):
    """Flexible PCG with the network against plain FP64 CG on held-out problems."""
    import torch
    out = []
    for sd in seeds:
        alpha, f = inputs.learned_problem(sd, N=N)
        op = fl.Operator(2, alpha, 2.0 / N, N)
        op.set_preconditioner(net)
        F = _dev(f, torch.float64)
        row = {"seed": sd, "alpha": alpha}
        for solver in ("fpcg", "cg64"):
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, info = op.poisson_solve(F, tol=tol, solver=solver)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
            row[solver] = {"iters": info["iters"], "relres": info["relres"], "fell_back": info["fell_back"],
                           "seconds": wall}
            row[solver + "_u"] = u
        row["rel_diff"] = float((row["fpcg_u"] - row["cg64_u"]).norm() / row["cg64_u"].norm())
        del row["fpcg_u"], row["cg64_u"]
        op.close()
        out.append(row)
    return out
