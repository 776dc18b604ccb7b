#!/usr/bin/env python3
"""Benchmark of the FFT matvec of the FD integral fractional Laplacian on one MI355X.

Workload (timed "step"): one y = A u of the 2D operator with N = 1024 intervals
per axis (1023^2 = 1,046,529 unknowns, FFT length 2048 per axis), alpha = 1.5,
on the Gaussian u = exp(-|x|^2) sampled on (-4,4)^2, FP32 FFT path (the
path's arithmetic type), inputs resident in HBM.  value = unknowns * steps /
seconds (Gdof/s).

Also reported on the same JSON line:
  roofline      -- the dominant pass's algorithmic bytes over its average
                   duration (HIP events on the launch stream), against 8 TB/s;
                   `traffic` from committed rocprofv3 FETCH/WRITE counters when
                   they were taken on the current kernel source, else null.
  cpu_baseline  -- the FP64 oracle's explicit sum on a bounded sample of rows
                   of the same workload, on this host's cores.
  extra         -- FP64 matvec rate, per-pass times and the Poisson
                   time-to-1e-8 of the solvers; the 3D N=256 matvec; the batch
                   of 64 mixed Poisson solves; the learned-preconditioner
                   workload (training pairs, training, flexible PCG against
                   plain CG).  All outside the timed region.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2_fp32.json")
KERNEL_SOURCES = ["paper_1804_02718_amd/csrc/fl_fft.hip", "paper_1804_02718_amd/csrc/fl_internal.hpp",
                  "paper_1804_02718_amd/csrc/fl_wave2d.hpp", "paper_1804_02718_amd/csrc/fl_fourstep.hpp"]


def kernel_source_sha():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pass_bytes(d, n, Q, P, s):
    """Algorithmic bytes per pass (pass model: each pass reads its input once and
    writes its output once; lambda read once).  s = bytes per real."""
    if d == 2:
        # half spectra of real rows: P reals per row (DC and Nyquist packed)
        return [s * (n * n + P * n),                # X-fwd: u in, half spectra out
                s * (2 * P * n + Q * Q),            # Y fused: spectra in/out, lambda
                s * (P * n + n * n)]                # X-inv: spectra in, y out
    return [s * (n ** 3 + 2 * Q * n * n),           # X-fwd
            s * (2 * Q * n * n + 2 * Q * P * n),    # Y-fwd
            s * (4 * Q * P * n + Q ** 3),           # Z fused
            s * (2 * Q * P * n + 2 * Q * n * n),    # Y-inv
            s * (2 * Q * n * n + n ** 3)]           # X-inv


PASS_NAMES = {2: ["x_fwd", "y_fused", "x_inv"], 3: ["x_fwd", "y_fwd", "z_fused", "y_inv", "x_inv"]}


def kernel_instance(pass_name, T, P, var, d=2):
    """Template instance of the kernel that runs a pass for a variant (as rocprofv3 names it);
    the 2D path keeps packed DC/Nyquist columns (last template argument true)."""
    ex, ey, c, lpb = var["ex"], var["ey"], var["tile"], var["row_pairs"]
    if var.get("kind", 0) == 1:  # 2D, one wavefront per FFT line
        return {"x_fwd": "k_w2_xfwd<%s, %d, %d>" % (T, P, c),
                "y_fused": "k_w2_yfused<%s, %d, %d, true>" % (T, P, c),
                "x_inv": "k_w2_xinv<%s, %d, %d, false>" % (T, P, c)}[pass_name]
    pack = "true" if d == 2 else "false"
    if pass_name == "x_fwd":
        return "k_xfwd<%s, %d, %d, %d, %d, %s>" % (T, P, ex, c, lpb, pack)
    if pass_name == "x_inv":
        return "k_xinv<%s, %d, %d, %d, %d, false, %s>" % (T, P, ex, c, lpb, pack)
    mode = {"y_fused": 2, "z_fused": 2, "y_fwd": 0, "y_inv": 1}[pass_name]
    return "k_strided<%s, %d, %d, %d, %d, %s>" % (T, P, ey, c, mode, pack if mode == 2 else "false")


def time_matvec(op, u, y, steps, warmup, torch):
    for _ in range(warmup):
        op.apply(u, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        op.apply(u, y)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def traffic_entry(dominant_kernel):
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    if rec.get("source_sha") != kernel_source_sha():
        return None
    k = rec.get("kernels", {}).get(dominant_kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


def host_cpu():
    """The host CPU model (lscpu's "Model name", from /proc/cpuinfo) and thread settings."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_oracle_extra(inputs):
    """The oracle on the other workloads, on this host: the C1 grid (2D N=32, alpha=1.5) applied in full
    and solved by dense Cholesky (measured), and the 3D N=256 matvec timed on 4096 seeded rows and
    extrapolated to all 16.6M rows (labelled extrapolated)."""
    import numpy as np

    import oracle
    out = {}
    N, alpha = 32, 1.5
    h = 2.0 / N
    t0 = time.perf_counter()
    a = oracle.coeffs(2, alpha, h, N)
    t1 = time.perf_counter()
    y = oracle.apply(2, N, alpha, a, inputs.bump(2, N, alpha))
    t2 = time.perf_counter()
    A = oracle.dense(2, N, alpha, a)
    u = oracle.solve_dense(A, np.ones((N - 1) ** 2))
    t3 = time.perf_counter()
    out["c1"] = {"kind": "measured", "coeff_seconds": round(t1 - t0, 4), "apply_seconds": round(t2 - t1, 4),
                 "dense_solve_seconds": round(t3 - t2, 4), "u_max": float(u.max()), "y_centre": float(y[len(y) // 2])}
    N3, a3 = 256, 1.2
    h3 = 2.0 / N3
    M3 = (N3 - 1) ** 3
    t0 = time.perf_counter()
    c3 = oracle.coeffs(3, a3, h3, N3)
    t1 = time.perf_counter()
    rows = np.random.default_rng(12).choice(M3, size=4096, replace=False)
    oracle.apply_rows(3, N3, a3, c3, inputs.ac_initial(M3, seed=3), rows)
    t2 = time.perf_counter()
    per_row = (t2 - t1) / rows.size
    out["c3"] = {"kind": "extrapolated", "rows_timed": int(rows.size), "seconds_timed": round(t2 - t1, 2),
                 "coeff_seconds": round(t1 - t0, 2), "matvec_seconds_extrapolated": round(per_row * M3, 1),
                 "gdof_s_extrapolated": round(1.0 / per_row / 1e9, 9)}
    return out


def cpu_baseline(N, alpha, h, u_np, seconds, gpu_y=None):
    """The oracle's explicit FP64 sum on seeded random rows of the C2 matvec for about `seconds`,
    as rows per second.  gpu_y ({"fp64": y, "fp32": y} host arrays of the library's matvec of the
    same u, FP32 on u rounded to FP32): its sampled rows are compared with the oracle's, e_rel
    against |Au| and e_sc against the oracle's |A||u| on the first 1024 sampled rows."""
    import numpy as np

    import oracle
    a = oracle.coeffs(2, alpha, h, N)
    M = (N - 1) ** 2
    rng = np.random.default_rng(12345)
    order = rng.permutation(M)
    done = 0
    batch = 256
    refs = []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < M:
        rows = order[done:done + batch]
        refs.append(oracle.apply_rows(2, N, alpha, a, u_np, rows))
        done += rows.size
        batch = min(batch * 2, 8192)
    dt = time.perf_counter() - t0
    out = {"value": done / dt / 1e9, "unit": "Gdof/s", "cores": oracle.num_threads(), "kind": "oracle",
           "host": host_cpu(),
           "sample": "explicit O(M^2) FP64 sum (long-double accumulation) on %d seeded random rows of the "
                     "%d-row N=1024 matvec in %.1f s, rate = rows/s (coefficient setup excluded)"
                     % (done, M, dt)}
    if gpu_y is not None:
        rows = order[:done]
        ref = np.concatenate(refs)
        sub = rows[:1024]
        absref = oracle.apply_rows(2, N, alpha, a, u_np, sub, absmode=True)
        u32 = u_np.astype(np.float32).astype(np.float64)
        ref32 = oracle.apply_rows(2, N, alpha, a, u32, sub)
        par = {"rows": int(done), "abs_rows": int(sub.size)}
        for prec, y in gpu_y.items():
            d = y[rows] - ref
            ds = y[sub] - (ref[:sub.size] if prec == "fp64" else ref32)
            par[prec] = {"e_rel": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                         "e_sc": float(np.linalg.norm(ds) / np.linalg.norm(absref))}
        par["note"] = ("e_rel: ||y - A u|| / ||A u|| on all sampled rows (fp32 against the FP64 u); e_sc: "
                       "||y - A u|| / || |A||u| || on the first 1024 (fp32 against u rounded to FP32)")
        out["parity_on_sample"] = par
    return out


def c3_extra(torch, fl, inputs, autotune, N=256, alpha=1.2):
    """3D N=256 (255^3 unknowns, FFT length 512): matvec Gdof/s and per-pass times in FP32 and FP64,
    200 semi-implicit Allen--Cahn steps, and the Poisson problem by the preconditioned and plain CG."""
    import numpy as np
    h = 2.0 / N
    M = (N - 1) ** 3
    op = fl.Operator(3, alpha, h, N)
    out = {"workload": "3D N=256 (255^3 unknowns, 512^3 embedding), alpha=1.2, uniform u in [-0.9,0.9]"}
    u64 = torch.as_tensor(inputs.ac_initial(M, seed=3), device="cuda:0")
    for prec, dtype, s in (("fp32", torch.float32, 4), ("fp64", torch.float64, 8)):
        u = u64.to(dtype)
        y = torch.empty_like(u)
        if autotune:
            best, ms = op.autotune(prec, reps=10)
            out[prec + "_variant"] = {"chosen": best, "ms_per_variant": [round(m, 4) for m in ms]}
        steps = 60
        dt = time_matvec(op, u, y, steps, 5, torch)
        pm = fl.fl_apply_profiled(op.handle, u, y, reps=20)
        pb = pass_bytes(3, op.n, op.Q, op.P, s)
        out[prec] = {"gdof_s": round(M * steps / dt / 1e9, 3), "ms_per_step": round(dt / steps * 1e3, 4),
                     "chain_roofline_frac": round(sum(pb) / (dt / steps) / 1e9 / HBM_PEAK_GBS, 4),
                     "passes": {PASS_NAMES[3][i]: {"avg_ms": round(pm[i], 4),
                                                   "GB_per_s": round(pb[i] / (pm[i] * 1e-3) / 1e9, 1)}
                                for i in range(5)}}
    # the Allen--Cahn workload: 200 semi-implicit steps (theta = 1/2, eps = 0.05, tau = 1e-3), each solved
    # to an FP64 residual of 1e-8 with FP32 inner CG
    u = u64.clone()
    op.allen_cahn_step(u.clone(), 1e-3, 0.05)  # warm (workspaces)
    torch.cuda.synchronize()
    iters, outer = [], []
    t0 = time.perf_counter()
    for _ in range(200):
        info = op.allen_cahn_step(u, 1e-3, 0.05)
        iters.append(info["iters"])
        outer.append(info["outer_iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["allen_cahn"] = {"steps": 200, "seconds": round(dt, 3), "ms_per_step": round(dt / 200 * 1e3, 3),
                         "inner_iters_per_step": round(sum(iters) / 200, 2), "outer_per_step": round(sum(outer) / 200, 2),
                         "max_abs_u": round(float(u.abs().max()), 6), "tau": 1e-3, "eps": 0.05, "theta": 0.5,
                         "tol": 1e-8}
    # the Poisson problem on the same cube (f = 4 seeded Gaussians), to 1e-8: the default
    # sine-transform preconditioned CG against plain FP64 CG
    f = torch.as_tensor(inputs.gauss_sum(3, N, 4, seed=5), device="cuda:0")
    pois = {}
    for solver in ("auto", "tau", "cg64"):
        uu = torch.zeros_like(f)
        op.poisson_solve(f, tol=1e-8, u=uu, solver=solver)  # warm
        uu.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = op.poisson_solve(f, tol=1e-8, u=uu, solver=solver)
        torch.cuda.synchronize()
        pois[solver] = {"seconds": round(time.perf_counter() - t0, 4), "iters": info["iters"],
                        "relres": info["relres"]}
    out["poisson"] = {"workload": "3D N=%d alpha=%.1f, f = sum of 4 seeded Gaussians on (-1,1)^3, tol 1e-8"
                                  % (N, alpha), **pois}
    op.close()
    return out


def large_extra(torch, fl, inputs, N=8192, alpha=1.5, reps=20):
    """The fine operator of the paper's tables: 2D N = 8192 on (-1, 1)^2 (8191^2 unknowns, FFT length
    16384, the global-memory passes), one matvec in FP64 and in FP32 on u = ((1-x^2)(1-y^2))^2
    (3 warm applications, then `reps` back-to-back applications timed with HIP events on the stream
    they run on)."""
    out = {"workload": "2D N=%d (FFT length 16384), alpha=%g, u=((1-x^2)(1-y^2))^2" % (N, alpha)}
    t0 = time.perf_counter()
    op = fl.Operator(2, alpha, 2.0 / N, N)
    torch.cuda.synchronize()
    out["create_seconds"] = round(time.perf_counter() - t0, 3)
    u64 = torch.as_tensor(inputs.paper_family(2, N, 2.0), device="cuda:0")
    for name, u in (("fp64", u64), ("fp32", u64.float())):
        y = op.apply(u)
        for _ in range(2):
            op.apply(u, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op.apply(u, y)
        e1.record()
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) / 1e3 / reps
        # pass model: each of x forward, the fused y pass and x inverse reads its input and writes its
        # output once, lambda read once (s bytes per real; n^2 unknowns, n x Q half spectra)
        s = 8 if name == "fp64" else 4
        n, Q = N - 1, op.desc["Q"]
        model = 2 * s * n * n + 8 * s * n * Q + s * Q * Q
        out[name] = {"ms": round(dt * 1e3, 3), "gdof_s": round(op.M / dt / 1e9, 3),
                     "pass_model_GB": round(model / 1e9, 3), "GB_per_s": round(model / dt / 1e9, 1),
                     "roofline_frac": round(model / dt / 1e9 / HBM_PEAK_GBS, 4)}
    # the Poisson problem on this grid (f = 8 seeded Gaussians), to 1e-8, by the default
    # solver (the sine-transform preconditioned FP32 inner solves in FP64 refinement here)
    f = torch.as_tensor(inputs.gauss_sum(2, N, 8, seed=2), device="cuda:0")
    uu = torch.zeros_like(f)
    op.poisson_solve(f, tol=1e-8, u=uu)  # warm (workspaces, preconditioner symbol)
    uu.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = op.poisson_solve(f, tol=1e-8, u=uu)
    torch.cuda.synchronize()
    out["poisson"] = {"seconds": round(time.perf_counter() - t0, 4), "iters": info["iters"],
                      "outer": info["outer_iters"], "relres": info["relres"],
                      "workload": "f = 8 seeded Gaussians on (-1,1)^2, tol 1e-8, default solver"}
    op.close()
    return out


def c4_extra(torch, fl, inputs):
    """64 2D Poisson problems, N from {64,128,256,512}, alpha ~ U(0.2,1.95), tol 1e-8: one batched
    solve (every class here: FP32 CG preconditioned by the sine transform, inside FP64
    refinement) against the same problems solved one after another with the default solver (the
    preconditioned FP64 flexible CG) and with plain FP32-matvec refinement."""
    probs = inputs.batch_problems(64, seed=4)
    fs = [torch.as_tensor(p["f"], device="cuda:0") for p in probs]
    t0 = time.perf_counter()
    b = fl.Batch(2, [p["N"] for p in probs], [p["alpha"] for p in probs], [p["h"] for p in probs])
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    b.solve(fs, tol=1e-8)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    us, infos = b.solve(fs, tol=1e-8)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    bstats = b.stats()
    b.close()
    ops = [fl.Operator(2, p["alpha"], p["h"], p["N"]) for p in probs]
    seq = {}
    for solver in ("auto", "refine"):
        for op, f in zip(ops, fs):
            op.poisson_solve(f, tol=1e-8, solver=solver)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos_s = [op.poisson_solve(f, tol=1e-8, solver=solver)[1] for op, f in zip(ops, fs)]
        torch.cuda.synchronize()
        seq[solver] = (time.perf_counter() - t0, infos_s)
    for op in ops:
        op.close()
    dofs = sum((p["N"] - 1) ** 2 for p in probs)
    ts, seq_infos = seq["auto"]
    return {"workload": "64 problems, N in {64,128,256,512}, alpha~U(0.2,1.95), 4 Gaussians, tol 1e-8",
            "unknowns": dofs, "batched_seconds": round(tb, 4), "sequential_seconds": round(ts, 4),
            "speedup": round(ts / tb, 2), "setup_seconds": round(setup, 3),
            "host_waits_per_solve": bstats["host_waits"], "graph_replays_per_solve": bstats["graph_launches"],
            "class_variants": {"fp32": bstats["var32"], "fp64": bstats["var64"]},
            "max_outer_iters": max(i["outer_iters"] for i in infos),
            "max_relres": max(i["relres"] for i in infos),
            "max_inner_iters": max(i["iters"] for i in infos),
            "sequential_max_relres": max(i["relres"] for i in seq_infos),
            "sequential_refine_seconds": round(seq["refine"][0], 4),
            "sequential_refine_max_inner_iters": max(i["iters"] for i in seq["refine"][1])}


def poisson_shapes_extra(torch, fl, inputs, alphas=(1.0, 1.5, 1.9)):
    """Poisson solves to 1e-8 off the power-of-two squares (the restricted sine-transform
    preconditioner of the default solver) against plain FP64 CG: a 2D square of N = 700, a 2D box
    of 1024 x 300 intervals, a 3D cube of N = 200, and N = 1025 (2^k + 1, which keeps the plain
    solvers); right-hand sides U[-1, 1] from seed 1."""
    cases = [("2D N=700", 2, 700, None), ("2D box 1024x300", 2, 1024, [1024, 301]),
             ("3D N=200", 3, 200, None), ("2D N=1025", 2, 1025, None)]
    rows = []
    for name, d, N, Nk in cases:
        for alpha in alphas:
            h = 2.0 / N
            op = fl.Operator(d, alpha, h, N) if Nk is None else fl.Operator(d, alpha, h, None, Nk=Nk)
            f = torch.as_tensor(inputs.uniform(op.M, seed=1, lo=-1.0, hi=1.0), device="cuda:0")
            row = [name, alpha]
            for solver in ("auto", "cg64"):
                u = torch.zeros_like(f)
                op.poisson_solve(f, tol=1e-8, u=u, solver=solver)  # warm
                u.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = op.poisson_solve(f, tol=1e-8, u=u, solver=solver)
                torch.cuda.synchronize()
                row += [info["iters"], round((time.perf_counter() - t0) * 1e3, 2)]
            rows.append(row)
            op.close()
    return {"workload": "Poisson to 1e-8, f ~ U[-1,1] (seed 1): 2D N=700, 2D box 1024x300, 3D N=200, 2D N=1025",
            "rows": rows, "row_fields": ["case", "alpha", "default_iters", "default_ms", "cg64_iters", "cg64_ms"]}


def poisson_extra(torch, fl, inputs, N=1024, alpha=1.5, alphas=(0.5, 1.0, 1.5, 1.9),
                  solvers=("cg64", "refine", "tau", "tau32", "auto")):
    """Time-to-1e-8 relative residual for the 2D N=1024 Poisson problem, f = 8 Gaussians: plain FP64
    CG, FP32-matvec refinement, the sine-transform preconditioned CG in FP64 (tau) and as FP32 inner
    solves in FP64 refinement (tau32, what the default solver takes here) at `alpha`, and CG against
    the default solver over `alphas`."""
    h = 2.0 / N
    f = torch.as_tensor(inputs.gauss_sum(2, N, 8, seed=2), dtype=torch.float64, device="cuda:0")

    def timed(op, solver):
        u = torch.zeros_like(f)
        op.poisson_solve(f, tol=1e-8, u=u, solver=solver)  # warm (workspace, preconditioner symbol)
        torch.cuda.synchronize()
        u.zero_()
        t0 = time.perf_counter()
        _, info = op.poisson_solve(f, tol=1e-8, u=u, solver=solver)
        torch.cuda.synchronize()
        return {"seconds": time.perf_counter() - t0, "iters": info["iters"], "outer": info["outer_iters"],
                "relres": info["relres"], "fell_back": info["fell_back"]}

    op = fl.Operator(2, alpha, h, N)
    out = {solver: timed(op, solver) for solver in solvers}
    op.close()
    res = {"workload": "2D N=1024 alpha=%.2f, f = sum of 8 seeded Gaussians on (-1,1)^2, tol 1e-8" % alpha, **out}
    if "cg64" in out and "auto" in out:
        res["default_speedup_over_cg64"] = round(out["cg64"]["seconds"] / out["auto"]["seconds"], 1)
    sweep = []
    for a in alphas:
        op = fl.Operator(2, a, h, N)
        c, t = timed(op, "cg64"), timed(op, "auto")
        sweep.append([a, c["iters"], round(c["seconds"] * 1e3, 3), t["iters"], round(t["seconds"] * 1e3, 3),
                      round(c["seconds"] / t["seconds"], 1)])
        op.close()
    if sweep:
        res["by_alpha"] = sweep
        res["by_alpha_fields"] = ["alpha", "cg64_iters", "cg64_ms", "default_iters", "default_ms",
                                  "cg64_over_default"]
    return res


def c5_extra(torch, fl, pairs, epochs, N=256, res_samples=2048, res_epochs=10):
    """Learned preconditioner, two training recipes (solver pairs with the L2 loss; residual-like inputs
    with the residual loss), each then in flexible PCG against plain FP64 CG on 8 held-out problems
    (tol 1e-8)."""
    import numpy as np

    from paper_1804_02718_amd import learned
    t0 = time.perf_counter()
    net = fl.UNet(N, max_batch=16, seed=1)
    x, t, alphas, mean_it = learned.make_pairs(net, N, pairs)
    torch.cuda.synchronize()
    tgen = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses = learned.train(net, x, t, epochs)
    torch.cuda.synchronize()
    ttrain = time.perf_counter() - t0
    del x, t
    # one network application (3.66 GFLOP at 256^2: the norm of r and five launches) and one FP64
    # matvec, for scale; back-to-back applications on one stream, timed by events
    op = fl.Operator(2, 1.0, 2.0 / N, N)
    r = torch.randn((N - 1) ** 2, dtype=torch.float64, device="cuda:0")
    z = torch.empty_like(r)
    for _ in range(3):
        net.apply(r, N - 1, 1.0, z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        net.apply(r, N - 1, 1.0, z)
    e1.record()
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / 1e3 / 50
    y = torch.empty_like(r)
    for _ in range(3):
        op.apply(r, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        op.apply(r, y)
    torch.cuda.synchronize()
    t_mv = (time.perf_counter() - t0) / 100
    op.close()
    held = [900000 + j for j in range(64)]
    rows = learned.compare(net, N, held)
    net.close()
    # the residual recipe: unit-diagonal operators, target-free residual loss on noise, Gaussian
    # sums and plain-CG residuals
    t0 = time.perf_counter()
    net2 = fl.UNet(N, max_batch=16, seed=1)
    x2, ops2, keep = learned.make_residual_samples(net2, N, res_samples)
    torch.cuda.synchronize()
    tgen2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses2 = learned.train_residual(net2, x2, ops2, res_epochs)
    torch.cuda.synchronize()
    ttrain2 = time.perf_counter() - t0
    del x2
    for o in keep:
        o.close()
    rows2 = learned.compare(net2, N, held)
    net2.close()

    def summary(rs):
        """Iteration and time ratios CG / FPCG over the held-out problems, overall and by alpha band,
        and the compact per-problem rows."""
        out = {"fell_back": int(sum(r["fpcg"]["fell_back"] for r in rs)),
               "max_rel_diff_vs_cg": float(max(r["rel_diff"] for r in rs)),
               "tau_mean_iters": round(float(np.mean([r["tau"]["iters"] for r in rs])), 2),
               "fpcg_over_tau_seconds": round(float(np.mean([r["fpcg"]["seconds"] / r["tau"]["seconds"]
                                                             for r in rs])), 2)}
        for lo, hi in ((0.3, 1.0), (1.0, 1.5), (1.5, 1.91), (0.3, 1.91)):
            sel = [r for r in rs if lo <= r["alpha"] < hi]
            if not sel:
                continue
            key = "alpha_%.1f_%.1f" % (lo, min(hi, 1.9))
            out[key] = {"problems": len(sel),
                        "cg_over_fpcg_iters": round(float(np.mean([r["cg64"]["iters"] / max(1, r["fpcg"]["iters"])
                                                                   for r in sel])), 3),
                        "cg_over_fpcg_seconds": round(float(np.mean([r["cg64"]["seconds"] / r["fpcg"]["seconds"]
                                                                     for r in sel])), 3)}
        out["rows"] = [[round(r["alpha"], 4), r["fpcg"]["iters"], r["fpcg"]["fell_back"],
                        round(r["fpcg"]["seconds"] * 1e3, 3), r["cg64"]["iters"], round(r["cg64"]["seconds"] * 1e3, 3),
                        r["tau"]["iters"], round(r["tau"]["seconds"] * 1e3, 3)]
                       for r in rs]
        out["row_fields"] = ["alpha", "fpcg_iters", "fpcg_fell_back", "fpcg_ms", "cg64_iters", "cg64_ms",
                             "tau_iters", "tau_ms"]
        return out

    return {"workload": "2D N=256 (255^2 interior on a 256^2 network grid), alpha~U(0.3,1.9), f = 8 Gaussians; "
                        "held-out seeds 900000..900063, tol 1e-8",
            "pairs": {"recipe": "%d solver pairs (seeds 100000+i), relative L2 loss, %d epochs" % (pairs, epochs),
                      "pair_generation_seconds": round(tgen, 2), "pair_solver_mean_iters": round(mean_it, 1),
                      "training_seconds": round(ttrain, 2), "epoch_loss": [round(float(l), 4) for l in losses],
                      "held_out": summary(rows)},
            "residual": {"recipe": "%d inputs (noise, Gaussian sums, plain-CG residuals), unit-diagonal operators, "
                                   "residual loss, %d epochs" % (res_samples, res_epochs),
                         "sample_seconds": round(tgen2, 2), "training_seconds": round(ttrain2, 2),
                         "epoch_loss": [round(float(l), 4) for l in losses2],
                         "held_out": summary(rows2)},
            "net_apply_ms": round(t_apply * 1e3, 4), "net_apply_TFLOP_s": round(3.66e9 / t_apply / 1e12, 2),
            "fp64_matvec_ms": round(t_mv * 1e3, 4)}


# CPU seconds the paper reports for its two-bubble Allen--Cahn run to t = 0.015 (Sec. 5.3,
# table of CPU times; hardware, language and CG tolerance not stated), by alpha and N
PAPER_AC_SECONDS = {1.9: {1024: 25728, 512: 4497, 256: 456, 128: 86},
                    1.5: {1024: 4896, 512: 974, 256: 112, 128: 27},
                    1.0: {1024: 648, 512: 170, 256: 30, 128: 9},
                    0.7: {1024: 430, 512: 107, 256: 24, 128: 7}}


def paper_ac_extra(torch, fl, inputs, sizes=(128, 256, 512, 1024), alphas=(1.9, 1.5, 1.0, 0.7),
                   sizes3d=(128, 256)):
    """The paper's two kissing bubbles: u_t = -(-Delta)^{alpha/2} u - delta^-alpha u (u^2 - 1) on (0,1)^d,
    u = -1 outside, delta = 0.03, h = 1/N, tau = 5e-4, 30 Crank--Nicolson steps to t = 0.015 (stepped as
    ubar = u + 1), each solved to an FP64 residual of 1e-8 by the default solver (the sine-transform
    preconditioned CG on these grids) and, for comparison, by FP32-matvec CG in FP64 refinement.  The
    paper's CPU seconds (2D) are context."""
    delta, tau, steps = 0.03, 5e-4, 30
    out = {"workload": "two kissing bubbles on (0,1)^d, delta=0.03, tau=5e-4, 30 steps to t=0.015, tol 1e-8",
           "runs": []}

    def run(d, alpha, N, centres, solver):
        h = 1.0 / N
        op = fl.Operator(d, alpha, h, N)
        ub = torch.as_tensor(inputs.kissing_bubbles(N, delta, centres), device="cuda:0")
        gamma = delta ** -alpha
        op.allen_cahn_step_gen(ub.clone(), tau, 1.0, gamma, 1.0, solver=solver)  # warm (workspaces)
        torch.cuda.synchronize()
        iters = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            iters += op.allen_cahn_step_gen(ub, tau, 1.0, gamma, 1.0, solver=solver)["iters"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        op.close()
        return ub, dt, iters

    c2, c3 = ((0.4, 0.4), (0.6, 0.6)), ((0.4, 0.6, 0.5), (0.6, 0.4, 0.5))
    # the 3D run (alpha = 1.9): the paper states neither its 3D mesh nor a time for
    # it; h = 1/N at the sizes3d, same delta, tau and end time
    cases = [(2, a, N, c2) for a in alphas for N in sizes] + [(3, 1.9, N, c3) for N in sizes3d]
    for d, alpha, N, centres in cases:
        ub, dt, iters = run(d, alpha, N, centres, "auto")
        ur, dtr, itr = run(d, alpha, N, centres, "refine")
        mass = float((ub - 1.0).abs().sum()) * (1.0 / N) ** d  # integral of |u| over the box
        out["runs"].append({"d": d, "alpha": alpha, "N": N, "seconds": round(dt, 4), "iters": iters,
                            "refine_seconds": round(dtr, 4), "refine_inner_iters": itr,
                            "max_abs_diff_vs_refine": float((ub - ur).abs().max()),
                            "mass_in_box": round(mass, 6),
                            "paper_cpu_seconds": PAPER_AC_SECONDS[alpha][N] if d == 2 else None})
        del ub, ur
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner report (the timed matvec always uses the library's default "
                         "kernel variant, the fastest one measured for this size)")
    ap.add_argument("--poisson-solvers", default="cg64,refine,tau,tau32,auto",
                    help="solvers timed on the 2D N=1024 Poisson problem (comma list of cg64, refine, tau, "
                         "tau32, auto)")
    ap.add_argument("--no-poisson-sweep", action="store_true",
                    help="skip CG64 against tau-PCG over alpha in {0.5, 1, 1.5, 1.9}")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 3D N=256 workload (matvec in FP32 and FP64, 200 Allen--Cahn steps)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2D N=8192 operator (FFT length 16384) of the paper's reference grid")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the batch of 64 mixed-(N, alpha) Poisson solves, batched and one by one")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the learned-preconditioner workload (pairs, training, flexible PCG vs CG)")
    ap.add_argument("--no-paper-ac", action="store_true",
                    help="skip the paper's two-bubble Allen--Cahn run (timed against its CPU table as context)")
    ap.add_argument("--c5-pairs", type=int, default=20000,
                    help="training pairs for the learned preconditioner (solver pairs, seeds 100000+i)")
    ap.add_argument("--c5-epochs", type=int, default=2)
    ap.add_argument("--c5-res-samples", type=int, default=2048,
                    help="inputs for the residual-loss recipe of the learned preconditioner")
    ap.add_argument("--c5-res-epochs", type=int, default=10)
    ap.add_argument("--large-only", action="store_true",
                    help="run only the 2D N=8192 operator (FFT length 16384) leg and print its JSON (for profiling)")
    ap.add_argument("--net-apply-only", action="store_true",
                    help="only time 50 applications of the learned preconditioner at 256^2 (untrained weights; "
                         "for profiling the network's kernels)")
    ap.add_argument("--c5-only", action="store_true",
                    help="run only the learned-preconditioner workload and print its JSON (for profiling)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB three times (a plain copy kernel "
                         "whose known traffic calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(no sharding or inter-GPU collectives); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1804_02718_amd import fl, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.net_apply_only:
        N = 256
        net = fl.UNet(N, max_batch=1, seed=1)
        r = torch.as_tensor(inputs.gauss_sum(2, N, 8, 5), device="cuda:0")
        z = torch.empty_like(r)
        for _ in range(3):
            net.apply(r, N - 1, 1.2, z)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(50):
            net.apply(r, N - 1, 1.2, z)
        e1.record()
        torch.cuda.synchronize()
        print(json.dumps({"net_apply_ms": round(e0.elapsed_time(e1) / 50, 4)}), flush=True)
        net.close()
        return
    if args.large_only:
        print(json.dumps({"large_operator": large_extra(torch, fl, inputs)}), flush=True)
        return
    if args.c5_only:
        print(json.dumps({"c5_learned": c5_extra(torch, fl, args.c5_pairs, args.c5_epochs,
                                                 res_samples=args.c5_res_samples,
                                                 res_epochs=args.c5_res_epochs)}), flush=True)
        return
    d, N, alpha = 2, 1024, 1.5
    lo, hi = -4.0, 4.0
    h = (hi - lo) / N
    M = (N - 1) ** d
    op = fl.Operator(d, alpha, h, N)
    u_np = inputs.gaussian(d, N, lo, hi)
    u32 = torch.as_tensor(u_np, dtype=torch.float32, device="cuda:0")
    y32 = torch.empty_like(u32)
    print("bench: workload 2D N=%d fp32, %d warmup + %d timed steps" % (N, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb * 262144, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    dt = time_matvec(op, u32, y32, args.steps, args.warmup, torch)
    value = M * args.steps / dt / 1e9
    ms_per_step = dt / args.steps * 1e3

    # per-pass durations, HIP events on the stream the passes are launched on
    pass_ms = fl.fl_apply_profiled(op.handle, u32, y32, reps=max(50, min(args.steps, 500)))
    names = PASS_NAMES[d]
    pb = pass_bytes(d, op.n, op.Q, op.P, 4)
    dom = int(np.argmax(pass_ms))
    achieved = pb[dom] / (pass_ms[dom] * 1e-3) / 1e9
    var = op.variants("fp32")[0]
    dom_kernel = kernel_instance(names[dom], "float", op.P, var, d)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_entry(dom_kernel),
                "kernel": dom_kernel, "pass": names[dom], "algorithmic_bytes": pb[dom],
                "avg_ms": round(pass_ms[dom], 5)}

    # autotuner report: every variant timed, the fastest selected; the headline above used variant 0
    tune = {}
    if not args.no_autotune:
        best, ms = op.autotune("fp32", reps=50)
        tune["fp32"] = {"chosen": best, "variant": op.variants("fp32")[best],
                        "ms_per_variant": [round(m, 5) for m in ms]}
        best64, ms64 = op.autotune("fp64", reps=30)
        tune["fp64"] = {"chosen": best64, "variant": op.variants("fp64")[best64],
                        "ms_per_variant": [round(m, 5) for m in ms64]}
        op.select_variant("fp32", 0)
        op.select_variant("fp64", 0)
        torch.cuda.synchronize()

    extra = {"passes": {names[i]: {"avg_ms": round(pass_ms[i], 5), "algorithmic_bytes": pb[i],
                                   "GB_per_s": round(pb[i] / (pass_ms[i] * 1e-3) / 1e9, 1)}
                        for i in range(len(names))},
             "chain_model_bytes": sum(pb),
             "chain_GB_per_s": round(sum(pb) / (dt / args.steps) / 1e9, 1),
             "chain_roofline_frac": round(sum(pb) / (dt / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
             "autotune": tune}
    if not args.no_extra:
        u64 = u32.double()
        y64 = torch.empty_like(u64)
        dt64 = time_matvec(op, u64, y64, max(100, args.steps // 4), 10, torch)
        extra["fp64_gdof_s"] = round(M * max(100, args.steps // 4) / dt64 / 1e9, 3)
        print("bench: poisson solves", file=sys.stderr, flush=True)
        extra["poisson"] = poisson_extra(torch, fl, inputs, solvers=tuple(args.poisson_solvers.split(",")),
                                         alphas=() if args.no_poisson_sweep else (0.5, 1.0, 1.5, 1.9))
        if not args.no_poisson_sweep:
            extra["poisson_shapes"] = poisson_shapes_extra(torch, fl, inputs)
    gpu_y = None
    if not args.no_cpu_baseline:
        # the matvec the oracle's sample is compared with: FP64 on the unrounded u, FP32 on u rounded
        u64n = torch.as_tensor(u_np, dtype=torch.float64, device="cuda:0")
        y64n = torch.empty_like(u64n)
        op.apply(u64n, y64n)
        op.apply(u32, y32)
        gpu_y = {"fp64": y64n.cpu().numpy(), "fp32": y32.cpu().numpy().astype(np.float64)}
        del u64n, y64n
    op.close()
    if not args.no_extra and not args.no_c3:
        print("bench: 3D N=256 matvec", file=sys.stderr, flush=True)
        extra["c3_matvec"] = c3_extra(torch, fl, inputs, not args.no_autotune)
    if not args.no_extra and not args.no_large:
        print("bench: 2D N=8192 operator", file=sys.stderr, flush=True)
        extra["large_operator"] = large_extra(torch, fl, inputs)
    if not args.no_extra and not args.no_c4:
        print("bench: batched solves", file=sys.stderr, flush=True)
        extra["c4_batch"] = c4_extra(torch, fl, inputs)
    if not args.no_extra and not args.no_paper_ac:
        print("bench: paper Allen--Cahn workload", file=sys.stderr, flush=True)
        extra["paper_allen_cahn"] = paper_ac_extra(torch, fl, inputs)
    if not args.no_extra and not args.no_c5:
        print("bench: learned preconditioner", file=sys.stderr, flush=True)
        extra["c5_learned"] = c5_extra(torch, fl, args.c5_pairs, args.c5_epochs, res_samples=args.c5_res_samples,
                                       res_epochs=args.c5_res_epochs)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(N, alpha, h, u_np, args.cpu_seconds, gpu_y)
        if not args.no_extra:
            extra["cpu_oracle"] = cpu_oracle_extra(inputs)
        # the oracle's Poisson solve at C2, extrapolated (not measured): one full explicit
        # matvec at the measured row rate, times the GPU's plain-CG iteration count
        if "poisson" in extra and "cg64" in extra["poisson"] and cpu.get("value"):
            mv_s = M / (cpu["value"] * 1e9)
            extra["poisson"]["oracle_extrapolated"] = {
                "kind": "extrapolated", "oracle_matvec_seconds": round(mv_s, 1),
                "cg64_seconds": round(mv_s * extra["poisson"]["cg64"]["iters"], 1)}

    line = {"metric": "Toeplitz matvec Gdof/s", "value": round(value, 3), "unit": "Gdof/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "2D fractional Laplacian FFT matvec, N=1024 (1023^2 unknowns, 2048^2 "
                                   "embedding), alpha=1.5, Gaussian u on (-4,4)^2", "d": d, "N": N,
                       "unknowns": M, "precision": "fp32"},
            "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
