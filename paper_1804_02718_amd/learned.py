"""Learned-preconditioner workload: training pairs from the solver, training,
and flexible PCG against plain CG.  Host orchestration only: the solves,
sample packing, network passes, losses and Adam steps run in the HIP library
(``fl.Batch``, ``fl_unet_pack``, ``fl_unet_train``, ``fl_poisson_solve_ex``).

Workload (2D, (-1, 1)^2, N = 256, n = 255 interior points padded to a
256 x 256 network grid): alpha ~ U(0.3, 1.9), right-hand side a sum of eight
Gaussians (centres U(-0.5, 0.5)^2, widths U(0.05, 0.2)); training seeds
100000 + i, held-out seeds 900000 + i.  A training pair is (f, u) with
A u = f solved to 1e-8 by the batched mixed-precision solver.

Two recipes:
  * pairs: (f, u) pairs and the relative L2 loss ||y - u|| / ||u|| (the
    network learns A^{-1} on smooth right-hand sides only);
  * residual: target-free inputs (white noise, Gaussian sums, and the
    residuals f - A x_k of k plain-CG iterations) and the residual loss
    ||A y - x0||^2 / ||x0||^2, with each operator scaled to a unit diagonal
    (A(h) = h^-alpha A(1), so a mesh h_s gives -c a_0 = 1).  Flexible PCG is
    invariant to a constant factor on the preconditioner, so a network trained
    at unit diagonal serves every mesh of the same N and alpha.
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
    """Flexible PCG with the network against plain FP64 CG and the sine-transform preconditioned CG
    on held-out problems."""
    import torch
    out = []
    for sd in seeds:
        alpha, f = inputs.learned_problem(sd, N=N)
        op = fl.Operator(2, alpha, 2.0 / N, N)
        op.set_preconditioner(net)
        F = _dev(f, torch.float64)
        row = {"seed": sd, "alpha": alpha}
        for solver in ("fpcg", "cg64", "tau"):
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, info = op.poisson_solve(F, tol=tol, solver=solver)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
            row[solver] = {"iters": info["iters"], "relres": info["relres"], "fell_back": info["fell_back"],
                           "seconds": wall}
            row[solver + "_u"] = u
        uf, uc = row["fpcg_u"].cpu().numpy(), row["cg64_u"].cpu().numpy()
        row["rel_diff"] = float(np.linalg.norm(uf - uc) / np.linalg.norm(uc))
        del row["fpcg_u"], row["cg64_u"], row["tau_u"]
        op.close()
        out.append(row)
    return out


def unit_diagonal_operator(alpha, N, L=2.0):
    """The 2D operator of (alpha, N) scaled to a unit diagonal: A(h) = h^-alpha A(1), so the mesh
    h_s = h d^(1/alpha) with d = -c a_0 at h = L / N gives -c a_0 = 1."""
    o = fl.Operator(2, alpha, L / N, N)
    d0 = -o.c * o.a0
    o.close()
    return fl.Operator(2, alpha, (L / N) * d0 ** (1.0 / alpha), N)


def make_residual_samples(net, N, count, alphas=None, seed=7, max_cg=80, chunk=64):
    """Inputs for the residual loss, cycling through `alphas` (17 values over [0.3, 1.9] by default):
    sample i is white noise U(-1, 1) (seed 500000 + i) when i % 3 == 0, the Gaussian-sum right-hand
    side of seed 100000 + i when i % 3 == 1, and otherwise that right-hand side's residual
    f - A x_k after k ~ U{1, ..., max_cg} plain-CG iterations from 0.  Returns (x [count, H, H, 2],
    per-sample unit-diagonal operators, all operators to keep alive)."""
    import torch
    if alphas is None:
        alphas = np.linspace(0.3, 1.9, 17)
    H, n = net.H, N - 1
    rng = np.random.default_rng(seed)
    scaled = [unit_diagonal_operator(float(a), N) for a in alphas]
    plain = [fl.Operator(2, float(a), 2.0 / N, N) for a in alphas]
    x = torch.zeros((count, H, H, 2), dtype=torch.float32, device="cuda:0")
    ops = []
    for k0 in range(0, count, chunk):
        rs, al = [], []
        for i in range(k0, min(count, k0 + chunk)):
            j = i % len(alphas)
            if i % 3 == 0:
                r = _dev(inputs.uniform(n * n, seed=500000 + i), torch.float64)
            else:
                _, f = inputs.learned_problem(100000 + i, N=N)
                r = _dev(f, torch.float64)
                if i % 3 == 2:
                    kit = int(rng.integers(1, max_cg + 1))
                    u, _ = plain[j].poisson_solve(r, tol=1e-14, solver="cg64", max_iter=kit, raise_on_error=False)
                    r = plain[j].residual(r, u, r)
            rs.append(r)
            al.append(float(alphas[j]))
            ops.append(scaled[j])
        net.pack(rs, None, al, n, x[k0:k0 + len(rs)])
    return x, ops, scaled + plain


def train_residual(net, x, ops, epochs, batch=16, lr=1e-3, lr_final=2e-5, seed=3):
    """Adam epochs on the residual loss ||A y - x0||^2 / ||x0||^2; mean loss per epoch."""
    return net.train(x, None, epochs=epochs, batch=batch, lr=lr, lr_final=lr_final, seed=seed, ops=ops)
