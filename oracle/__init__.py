"""FP64 CPU oracle for the FD integral fractional Laplacian -- TEST INFRASTRUCTURE.

Duo & Zhang, "Accurate numerical methods for two and three dimensional
integral fractional Laplacian with applications" (arXiv:1804.02718).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path
and never imports the product package.

Contents (gamma = 2, the paper's default in Sec. 5):

* ``const(d, alpha)``          -- c_{d,alpha} of the hypersingular integral (Sec. 1).
* ``J(d, p)``, ``E0``, ``D2``  -- closed-form pieces of the element integrals
  (origin element, Sec. 2 proof of Thm 1 polar identity; tail region D2,
  Sec. 2 / Sec. 4).
* ``elements`` / ``coeffs``    -- element integrals and scheme coefficients
  a_v (Sec. 2 a_mn, a_00; Sec. 4 a_mns, a_000).
* ``apply`` / ``apply_rows``   -- the scheme as an explicit O(M^2) sum
  (Sec. 2 2D scheme, Sec. 4 3D scheme), long-double accumulated.
* ``dense``                    -- the symmetric multilevel Toeplitz matrix
  (Sec. 2 block-Toeplitz form, Sec. 4 three-level form).
* ``solve_dense`` / ``solve_cg`` -- fractional Poisson solve (Sec. 5.2):
  Cholesky, or plain conjugate gradients on the explicit sum.
* ``ac_step``                  -- one semi-implicit step of the fractional
  Allen--Cahn equation (Sec. 5.3: Crank--Nicolson on the linear term, the
  cubic term explicit at the old time level).

Parity of the GPU path is measured against these functions; the functions
themselves are pinned by ``tests/test_oracle_*.py`` against closed forms,
limits stated in the paper, high-precision quadrature and brute force.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_J.restype = ctypes.c_double
        lib.orc_J.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.orc_E0.restype = ctypes.c_double
        lib.orc_E0.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_D2.restype = ctypes.c_double
        lib.orc_D2.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_const.restype = ctypes.c_double
        lib.orc_const.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.orc_elements.restype = ctypes.c_int
        lib.orc_elements.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        lib.orc_coeffs.restype = ctypes.c_int
        lib.orc_coeffs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.orc_coeffs_g.restype = ctypes.c_int
        lib.orc_coeffs_g.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, dp, dp]
        lib.orc_apply_rows.restype = ctypes.c_int
        lib.orc_apply_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp,
                                       i64p, ctypes.c_int64, dp, ctypes.c_int]
        lib.orc_apply_rows_box.restype = ctypes.c_int
        lib.orc_apply_rows_box.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_double,
                                           dp, dp, i64p, ctypes.c_int64, dp, ctypes.c_int]
        lib.orc_gl_rule.restype = None
        lib.orc_gl_rule.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_lib().orc_num_threads())


def gl_rule(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    _lib().orc_gl_rule(n, _dp(x), _dp(w))
    return x, w


def const(d: int, alpha: float) -> float:
    """c_{d,alpha} = 2^{alpha-1} alpha Gamma((d+alpha)/2) / (pi^{d/2} Gamma(1-alpha/2)) (Sec. 1)."""
    return (2.0 ** (alpha - 1.0) * alpha * math.gamma(0.5 * (d + alpha))
            / (math.pi ** (0.5 * d) * math.gamma(1.0 - 0.5 * alpha)))


def J(d: int, p: float) -> float:
    """int_{[0,1]^{d-1}} (1+|s|^2)^{-p/2} ds."""
    return float(_lib().orc_J(d, p))


def E0(d: int, alpha: float, h: float) -> float:
    """Integral of |xi|^{-(d+alpha-2)} over the origin element [0,h]^d."""
    return float(_lib().orc_E0(d, d + alpha - 2.0, h))


def D2(d: int, alpha: float, L: float) -> float:
    """Integral of |xi|^{-(d+alpha)} over R^d_+ minus (0,L)^d (Sec. 2 / Sec. 4)."""
    return float(_lib().orc_D2(d, alpha, L))


def elements(d: int, alpha: float, h: float, N: int) -> np.ndarray:
    """E[e] = int_{I_e} |xi|^{gamma-(d+alpha)}, e in [0,N-1]^d; array index order (e_d,...,e_1)."""
    E = np.zeros(N ** d)
    rc = _lib().orc_elements(d, alpha, h, N, _dp(E))
    if rc:
        raise ValueError("orc_elements failed (%d)" % rc)
    return E.reshape((N,) * d)


def coeffs(d: int, alpha: float, h: float, N: int, return_elements: bool = False, gamma: float = 2.0):
    """Scheme coefficients a_v, v in [0,N]^d, numpy index order (v_d, ..., v_1); a[0,..,0] = a_0.

    Sec. 2: a_mn and a_00; Sec. 4: a_mns and a_000 (origin correction for
    (1,1,1) read as +1, the value the gamma = 2 limit rule implies); d = 1 is
    the one-dimensional case of the general-d scheme (Sec. 4, Theorems 3-4):
    a_m = (int_{T_m} w + floor(gamma/2) [m = 1] E_0) / (2 |xi_m|^gamma).  gamma is
    the splitting parameter of Sec. 2, in (alpha, 2]; for gamma < 2 the
    origin-element corrections vanish (their weight is floor(gamma/2)).
    """
    if d not in (1, 2, 3):
        raise ValueError("d must be 1, 2 or 3")
    if not (0.0 < alpha < 2.0) or N < 2 or not (h > 0) or not (alpha < gamma <= 2.0):
        raise ValueError("bad parameters")
    a = np.zeros((N + 1) ** d)
    E = np.zeros(N ** d)
    if gamma == 2.0:
        rc = _lib().orc_coeffs(d, alpha, h, N, _dp(a), _dp(E))
    else:
        rc = _lib().orc_coeffs_g(d, alpha, gamma, h, N, _dp(a), _dp(E))
    if rc:
        raise ValueError("orc_coeffs failed (%d)" % rc)
    a = a.reshape((N + 1,) * d)
    if return_elements:
        return a, E.reshape((N,) * d)
    return a


def apply_rows(d: int, N: int, alpha: float, a: np.ndarray, u: np.ndarray, rows=None,
               absmode: bool = False, shape=None) -> np.ndarray:
    """(A u)_i = -c sum_j a_{|i-j|} u_j for the interior rows i (Sec. 2 / Sec. 4 scheme).

    ``u`` has (N-1)^d entries, x index fastest, or on a box (``shape`` = interior
    nodes per axis, x first, each <= N-1; the coefficient table is the one of
    the square of side L = N h, the longest side).  ``rows`` are flat interior
    indices (all rows when None).  ``absmode`` gives c sum_j |a_{|i-j|} u_j|.
    """
    c = const(d, alpha)
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    nk = [N - 1] * d if shape is None else [int(x) for x in shape]
    if len(nk) != d or min(nk) < 1 or max(nk) > N - 1:
        raise ValueError("bad shape")
    M = int(np.prod(nk))
    if u.size != M or a.size != (N + 1) ** d:
        raise ValueError("size mismatch")
    nka = (ctypes.c_int * 3)(*(nk + [1] * (3 - d)))
    if rows is None:
        y = np.zeros(M)
        rc = _lib().orc_apply_rows_box(d, N, nka, c, _dp(a), _dp(u), None, 0, _dp(y), int(absmode))
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64).ravel()
        if r.size and (r.min() < 0 or r.max() >= M):
            raise ValueError("row index out of range")
        y = np.zeros(r.size)
        rc = _lib().orc_apply_rows_box(d, N, nka, c, _dp(a), _dp(u),
                                       r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       r.size, _dp(y), int(absmode))
    if rc:
        raise ValueError("orc_apply_rows_box failed (%d)" % rc)
    return y


def apply(d, N, alpha, a, u, absmode=False, shape=None):
    return apply_rows(d, N, alpha, a, u, None, absmode, shape)


def dense(d: int, N: int, alpha: float, a: np.ndarray, shape=None) -> np.ndarray:
    """Dense matrix A_{ij} = -c a_{|i-j|} (Sec. 2 block Toeplitz / Sec. 4 three-level Toeplitz),
    on the square grid or on a box of ``shape`` interior nodes per axis (x first)."""
    c = const(d, alpha)
    nk = [N - 1] * d if shape is None else [int(x) for x in shape]
    Ds = [np.abs(np.arange(m)[:, None] - np.arange(m)[None, :]) for m in nk]
    a = np.asarray(a)
    M = int(np.prod(nk))
    if d == 1:
        return -c * a[Ds[0]]
    if d == 2:
        # a is indexed [v1, v0]; row i = i1*n0 + i0, column j = j1*n0 + j0
        D0, D1 = Ds
        A = a[D1[:, None, :, None], D0[None, :, None, :]]  # [i1, i0, j1, j0]
    else:
        D0, D1, D2 = Ds
        A = a[D2[:, None, None, :, None, None], D1[None, :, None, None, :, None],
              D0[None, None, :, None, None, :]]  # [i2, i1, i0, j2, j1, j0]
    return -c * A.reshape(M, M)


def solve_dense(A: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Solve A u = f by Cholesky (A is symmetric positive definite, Sec. 2)."""
    Lc = np.linalg.cholesky(A)
    z = np.linalg.solve(Lc, f)
    return np.linalg.solve(Lc.T, z)


def solve_cg(matvec, f: np.ndarray, tol: float, x0=None, maxiter: int = 100000):
    """Plain conjugate gradients (Sec. 5.3 names CG for these systems).

    Stops when ||f - A x||_2 <= tol ||f||_2 on the recursively updated
    residual; returns (x, iterations).
    """
    x = np.zeros_like(f) if x0 is None else x0.astype(np.float64).copy()
    r = f - matvec(x) if x0 is not None else f.copy()
    p = r.copy()
    rr = float(r @ r)
    fn = float(np.linalg.norm(f))
    it = 0
    if fn == 0.0:
        return x, 0
    while math.sqrt(rr) > tol * fn and it < maxiter:
        Ap = matvec(p)
        alpha = rr / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def ac_step(d: int, N: int, alpha: float, a: np.ndarray, u: np.ndarray, tau: float,
            eps: float, theta: float = 0.5, A: np.ndarray = None,
            reaction: bool = True) -> np.ndarray:
    """One step of u_t = -eps^2 (-Delta)^{alpha/2} u + u - u^3, zero exterior.

    theta-scheme on the linear term (theta = 1/2 is Crank--Nicolson, Sec. 5.3),
    the cubic term explicit:
      (I + theta tau eps^2 A) u+ = u - (1-theta) tau eps^2 A u + tau (u - u^3).
    Dense Cholesky solve (small grids only).  ``reaction=False`` drops the
    u - u^3 term (used to pin the linear part).
    """
    return ac_step_gen(d, N, alpha, a, u, tau, eps * eps, 1.0 if reaction else 0.0, 0.0, theta, A)


def ac_step_gen(d: int, N: int, alpha: float, a: np.ndarray, u: np.ndarray, tau: float,
                kappa: float, gamma: float, shift: float, theta: float = 0.5,
                A: np.ndarray = None) -> np.ndarray:
    """One step of u_t = -kappa (-Delta)^{alpha/2} u + gamma (w - w^3), w = u - shift,
    zero exterior, with the theta-scheme on the linear term and the reaction explicit:
      (I + theta tau kappa A) u+ = u - (1-theta) tau kappa A u + tau gamma (w - w^3).
    Sec. 5.3's equation (u = -1 outside (0,1)^d, reaction -delta^{-alpha} u (u^2 - 1))
    is this form for ubar = u + 1: kappa = 1, gamma = delta^{-alpha}, shift = 1.
    """
    if A is None:
        A = dense(d, N, alpha, a)
    u = np.asarray(u, dtype=np.float64)
    s = tau * kappa
    w = u - shift
    b = u - (1.0 - theta) * s * (A @ u) + tau * gamma * (w - w ** 3)
    K = np.eye(A.shape[0]) + theta * s * A
    return solve_dense(K, b)
