"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only samples test functions on grids and draws random numbers; it
holds none of the discretisation's arithmetic.  Layout of every grid vector:
the (N-1)^d interior nodes x_i = lo + i h, i in [1, N-1]^d, h = (hi - lo)/N,
flattened with the x index fastest (the ordering of the paper's matrix form).

Workloads (all synthetic; the paper's experiments use analytic functions):
  * ``gaussian``      -- exp(-|x|^2), the smooth test function whose image has
                         a closed form through 1F1.
  * ``bump``          -- (1 - |x|^2)_+^{alpha/2}, image constant on the unit ball.
  * ``paper_family``  -- prod_i (1 - x_i^2)^s on (-1,1)^d (the accuracy
                         family of Sec. 5.1 and Examples 5.2.1-5.2.2).
  * ``uniform``       -- i.i.d. U[lo, hi] values from a seed.
  * ``gauss_sum``     -- sum of seeded Gaussians exp(-|x-c_k|^2 / (2 w_k^2)),
                         centres U(-0.5, 0.5)^d, widths U(0.05, 0.2).
  * ``batch_problems`` -- the mixed (N, alpha) batch of Poisson problems.
"""
import numpy as np

__all__ = ["nodes_1d", "grid", "gaussian", "bump", "paper_family", "uniform",
           "gauss_sum", "ac_initial", "batch_problems", "learned_problem"]


def nodes_1d(N: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    h = (hi - lo) / N
    return lo + h * np.arange(1, N)


def grid(d: int, N: int, lo: float = -1.0, hi: float = 1.0):
    """Coordinate arrays (x_1, ..., x_d), each flattened over the interior, x fastest."""
    x = nodes_1d(N, lo, hi)
    g = np.meshgrid(*([x] * d), indexing="ij")  # g[k] varies along numpy axis k
    # numpy axis 0 is the slowest; the x index (coordinate 1) must be fastest
    return [g[d - 1 - k].ravel() for k in range(d)]


def _r2(d, N, lo, hi):
    return sum(c * c for c in grid(d, N, lo, hi))


def gaussian(d: int, N: int, lo: float = -4.0, hi: float = 4.0) -> np.ndarray:
    return np.exp(-_r2(d, N, lo, hi))


def bump(d: int, N: int, alpha: float, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.maximum(0.0, 1.0 - _r2(d, N, lo, hi)) ** (0.5 * alpha)


def paper_family(d: int, N: int, s: float, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    out = np.ones((N - 1) ** d)
    for c in grid(d, N, lo, hi):
        out *= np.maximum(0.0, 1.0 - c * c)
    return out ** s


def uniform(M: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, M)


def _gauss_params(rng, d, count, crange=0.5, wmin=0.05, wmax=0.2):
    params = []
    for _ in range(count):
        c = [rng.uniform(-crange, crange) for _ in range(d)]
        w = rng.uniform(wmin, wmax)
        params.append((c, w))
    return params


def _gauss_eval(d, N, params, lo, hi):
    coords = grid(d, N, lo, hi)
    f = np.zeros((N - 1) ** d)
    for c, w in params:
        r2 = sum((coords[k] - c[k]) ** 2 for k in range(d))
        f += np.exp(-r2 / (2.0 * w * w))
    return f


def gauss_sum(d: int, N: int, count: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Sum of ``count`` Gaussians; per Gaussian the draws are c_1, ..., c_d, then w."""
    rng = np.random.default_rng(seed)
    return _gauss_eval(d, N, _gauss_params(rng, d, count), lo, hi)


def ac_initial(M: int, seed: int = 3) -> np.ndarray:
    """Allen--Cahn initial state, i.i.d. U[-0.9, 0.9]."""
    return uniform(M, seed, -0.9, 0.9)


def batch_problems(count: int = 64, seed: int = 4, sizes=(64, 128, 256, 512),
                   alpha_range=(0.2, 1.95), gaussians: int = 4):
    """Mixed batch: per problem draw N, then alpha, then the Gaussians of its rhs.

    Returns a list of dicts {N, alpha, h, f} on (-1, 1)^2.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        N = int(sizes[int(rng.integers(0, len(sizes)))])
        alpha = float(rng.uniform(*alpha_range))
        params = _gauss_params(rng, 2, gaussians)
        f = _gauss_eval(2, N, params, -1.0, 1.0)
        out.append({"N": N, "alpha": alpha, "h": 2.0 / N, "f": f})
    return out


def learned_problem(seed: int, N: int = 256, alpha_range=(0.3, 1.9), gaussians: int = 8):
    """One (alpha, rhs) draw of the learned-preconditioner workload on (-1, 1)^2."""
    rng = np.random.default_rng(seed)
    alpha = float(rng.uniform(*alpha_range))
    params = _gauss_params(rng, 2, gaussians)
    return alpha, _gauss_eval(2, N, params, -1.0, 1.0)


def kissing_bubbles(N: int, delta: float = 0.03, centres=((0.4, 0.4), (0.6, 0.6)), radius: float = 0.12):
    """Two touching bubbles on (0, 1)^d (Sec. 5.3; d = len of a centre, 2 or 3): u0 = 1 - tanh(d1/delta)
    - tanh(d2/delta) with d_i = |x - x_i| - radius, at the interior nodes x = i/N, returned as
    ubar0 = u0 + 1 (the shifted field that is 0 outside the box, where u = -1).  The paper's 3D
    run takes the centres (0.4, 0.6, 0.5) and (0.6, 0.4, 0.5)."""
    d = len(centres[0])
    xs = grid(d, N, 0.0, 1.0)
    u = np.ones_like(xs[0])
    for c in centres:
        r = np.sqrt(sum((xs[k] - c[k]) ** 2 for k in range(d)))
        u -= np.tanh((r - radius) / delta)
    return u + 1.0
