"""FP64 CPU oracle of the sine-transform (tau) preconditioner -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU path.

The preconditioner is not part of the paper's scheme: it is a preconditioner
for the CG solves of its Poisson problem (Sec. 5.2) and of the linear systems
of its semi-implicit Allen--Cahn steps (Sec. 5.3), whose matrices are
symmetric multilevel Toeplitz (Sec. 2, Sec. 4).

Definition (the tau algebra of Bini and Di Benedetto).  On n = N - 1 nodes
per axis the orthonormal sine vectors

    S[j, k] = sqrt(2 / N) sin(pi (j + 1) (k + 1) / N),   j, k = 0 .. n-1,

diagonalise every matrix of the tau class.  For a symmetric multilevel
Toeplitz matrix T with generator t_m (m >= 0 per axis, m < n), the tau matrix
tau(T) is the member of the class whose eigenvalues are the cosine sums

    lambda_k = sum_m t_m prod_axes w(m_i) cos(pi m_i (k_i + 1) / N),
    w(0) = 1, w(m > 0) = 2,

and, entrywise, tau(T) is T minus its two Hankel corrections on every level:
with sigma(i, j) ranging over |i - j| (sign +1), i + j + 2 (sign -1) and
2n - i - j (sign -1),

    tau(T)[i, j] = sum over the sigma of each axis of prod(signs) t_{sigma}

(t_m = 0 for m >= n).  ``tau_apply_gen`` evaluates M^{-1} r for
M = s0 I + s1 tau(T) from the first form; ``tau_matrix_gen`` writes the
second form out entry by entry.  The tests pin the first against the second,
and against the central-difference Laplacian, which lies in the class (its
tau matrix is itself).

Where the circulant embedding of the scheme's matrix (period P per axis, the
smallest power of two >= max(8, 2n - 1)) is longer than 2(n + 1) -- every N
that is not a power of two, and every box -- the preconditioner lives on the
n' = P/2 - 1 nodes whose sine basis the embedding's transforms provide: the
tau matrix of the n'-node Toeplitz matrix with the same generator (t_m = 0
for m >= n), inverted, and restricted to the operator's nodes (a principal
submatrix of an SPD matrix, so SPD).  It requires n <= n' on every axis,
which fails only for N = 2^k + 1.
"""

import numpy as np

from . import const


def sine_basis(n: int) -> np.ndarray:
    """Orthonormal, symmetric DST-I matrix on n points (N = n + 1 intervals)."""
    N = n + 1
    j = np.arange(1, n + 1)
    return np.sqrt(2.0 / N) * np.sin(np.pi * np.outer(j, j) / N)


def tau_eigenvalues_gen(t: np.ndarray) -> np.ndarray:
    """lambda_k on the sine frequencies pi (k+1)/N, k in [0, n)^d, from the generator t
    (numpy index order, every axis of length n): the cosine sums above."""
    t = np.asarray(t, dtype=np.float64)
    n = t.shape[0]
    N = n + 1
    m = np.arange(n)
    k = np.arange(1, n + 1)
    Cw = np.where(m == 0, 1.0, 2.0)[:, None] * np.cos(np.pi * np.outer(m, k) / N)
    lam = t
    for ax in range(t.ndim):  # contract every axis of t with Cw[m, k]
        lam = np.moveaxis(np.tensordot(lam, Cw, axes=([ax], [0])), -1, ax)
    return lam


def _sine_transform(x: np.ndarray, S: np.ndarray) -> np.ndarray:
    for ax in range(x.ndim):
        x = np.moveaxis(np.tensordot(x, S, axes=([ax], [0])), -1, ax)
    return x


def tau_apply_gen(t: np.ndarray, r: np.ndarray, s0: float = 0.0, s1: float = 1.0) -> np.ndarray:
    """z = (s0 I + s1 tau(T))^{-1} r, r flat with the x index fastest (numpy order)."""
    t = np.asarray(t, dtype=np.float64)
    n, d = t.shape[0], t.ndim
    S = sine_basis(n)
    mu = s0 + s1 * tau_eigenvalues_gen(t)
    R = np.asarray(r, dtype=np.float64).reshape((n,) * d)
    return _sine_transform(_sine_transform(R, S) / mu, S).ravel()


def tau_matrix_gen(t: np.ndarray) -> np.ndarray:
    """tau(T) written out entry by entry: T minus its Hankel corrections on every level
    (small n only)."""
    t = np.asarray(t, dtype=np.float64)
    n, d = t.shape[0], t.ndim

    def gen(idx):
        return t[idx] if all(0 <= m < n for m in idx) else 0.0

    def sig(i, j):
        return ((abs(i - j), 1.0), (i + j + 2, -1.0), (2 * n - i - j, -1.0))

    idx = list(np.ndindex(*((n,) * d)))
    M = np.zeros((n ** d, n ** d))
    for a, I in enumerate(idx):
        for b, J in enumerate(idx):
            v = 0.0
            terms = [((), 1.0)]
            for ax in range(d):
                terms = [(m + (mm,), s * ss) for m, s in terms for mm, ss in sig(I[ax], J[ax])]
            for m, s in terms:
                v += s * gen(m)
            M[a, b] = v
    return M


def generator(d: int, N: int, alpha: float, a: np.ndarray) -> np.ndarray:
    """Toeplitz generator t_m = -c a_m, m in [0, n)^d, of the scheme's matrix (Sec. 2, Sec. 4)."""
    a = np.asarray(a)
    sl = tuple([slice(0, N - 1)] * d)
    return -const(d, alpha) * a[sl]


def embedding_nodes(N: int) -> int:
    """n' = P/2 - 1 for the embedding period P = the smallest power of two >= max(8, 2n - 1)."""
    n = N - 1
    P = 8
    while P < 2 * n - 1:
        P *= 2
    return P // 2 - 1


def tau_apply(d: int, N: int, alpha: float, a: np.ndarray, r: np.ndarray, s0: float = 0.0,
              s1: float = 1.0, shape=None) -> np.ndarray:
    """The sine-transform preconditioner of s0 I + s1 A applied to r, A the scheme's
    matrix with N intervals per axis on the square or cube, or on the box of
    ``shape`` interior nodes per axis (x first): the tau matrix on the n' nodes of
    the embedding, inverted and restricted to the operator's nodes."""
    n = N - 1
    n2 = embedding_nodes(N)
    nk = [n] * d if shape is None else [int(k) for k in shape]
    if max(nk) > n2:
        raise ValueError("no sine basis of the embedding holds %d nodes (n' = %d)" % (max(nk), n2))
    t = np.zeros((n2,) * d)
    t[tuple([slice(0, n)] * d)] = generator(d, N, alpha, a)
    idx = tuple(slice(0, k) for k in reversed(nk))  # numpy order: the last axis is x
    R = np.zeros((n2,) * d)
    R[idx] = np.asarray(r, dtype=np.float64).reshape(tuple(reversed(nk)))
    z = tau_apply_gen(t, R.ravel(), s0, s1).reshape((n2,) * d)
    return z[idx].ravel()
