"""Pins of the oracle's sine-transform (tau) preconditioner (CPU).

The oracle evaluates (s0 I + s1 tau(T))^{-1} r from the tau matrix's
eigenvalues (cosine sums of the Toeplitz generator) and the DST-I basis.  The
pins check it against what fixes the tau matrix independently:
- its entrywise form, T minus the two Hankel corrections on every level
  (t_{i+j+2} and t_{2n-i-j}), written out term by term;
- the central-difference Laplacian, which lies in the tau class, so that the
  preconditioner inverts it exactly;
- the scheme's generator read back from the dense oracle matrix (Sec. 2,
  Sec. 4);
- the shift s0 I, which the class contains.
"""

import numpy as np
import pytest

import oracle
from oracle import tau


@pytest.mark.parametrize("d,n", [(1, 9), (1, 16), (2, 5), (2, 7), (3, 3), (3, 4)])
def test_eigen_form_matches_the_two_hankel_form(d, n):
    rng = np.random.default_rng(100 + 10 * d + n)
    t = rng.standard_normal((n,) * d)
    M = tau.tau_matrix_gen(t)
    E = np.eye(n ** d)
    Minv = np.stack([tau.tau_apply_gen(t, E[:, k]) for k in range(n ** d)], 1)
    assert np.abs(Minv @ M - E).max() < 1e-11 * max(1.0, np.linalg.cond(M))


def test_two_hankel_form_by_hand_1d():
    # n = 4, t = (t0, t1, t2, t3): tau(T) = T - H1 - H2 with H1[i, j] = t_{i+j+2},
    # H2[i, j] = t_{2n-i-j} = t_{8-i-j} (zero for indices >= n)
    t = np.array([4.0, -1.5, 0.5, -0.25])
    T = np.array([[t[abs(i - j)] for j in range(4)] for i in range(4)])
    H1 = np.array([[0.5, -0.25, 0, 0], [-0.25, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]])
    H2 = np.array([[0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, -0.25], [0, 0, -0.25, 0.5]])
    assert np.allclose(tau.tau_matrix_gen(t), T - H1 - H2, atol=0, rtol=0)


@pytest.mark.parametrize("d,n", [(1, 12), (2, 7), (3, 5)])
def test_exact_inverse_of_the_central_difference_laplacian(d, n):
    t = np.zeros((n,) * d)
    t[(0,) * d] = 2.0 * d
    for ax in range(d):
        idx = [0] * d
        idx[ax] = 1
        t[tuple(idx)] = -1.0
    # the dense discrete Laplacian, built independently of the tau code
    L1 = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    L = np.zeros((n ** d, n ** d))
    for ax in range(d):
        mats = [np.eye(n)] * d
        mats[ax] = L1
        K = mats[0]
        for m in mats[1:]:
            K = np.kron(K, m)
        L += K
    assert np.abs(tau.tau_matrix_gen(t) - L).max() == 0.0
    r = np.random.default_rng(7).standard_normal(n ** d)
    assert np.abs(tau.tau_apply_gen(t, L @ r) - r).max() < 1e-13


@pytest.mark.parametrize("d,N", [(1, 10), (2, 6), (3, 4)])
def test_generator_is_the_dense_matrix_first_row(d, N):
    alpha = 1.3
    a = oracle.coeffs(d, alpha, 2.0 / N, N)
    A = oracle.dense(d, N, alpha, a)
    t = tau.generator(d, N, alpha, a)
    assert np.array_equal(A[0].reshape((N - 1,) * d), t)


def test_shift_lies_in_the_class():
    rng = np.random.default_rng(3)
    n = 6
    t = rng.standard_normal((n, n))
    t[0, 0] += 20.0
    M = tau.tau_matrix_gen(t)
    r = rng.standard_normal(n * n)
    s0, s1 = 0.7, 0.003
    z = tau.tau_apply_gen(t, r, s0, s1)
    assert np.abs((s0 * np.eye(n * n) + s1 * M) @ z - r).max() < 1e-12


@pytest.mark.parametrize("N", [8, 16, 24])
@pytest.mark.parametrize("alpha", [0.3, 1.0, 1.5, 1.9])
def test_preconditioned_spectrum_is_clustered(N, alpha):
    # property (not a pin): the eigenvalues of M^{-1} A stay in a fixed interval
    # near 1 while cond(A) grows like N^alpha
    a = oracle.coeffs(2, alpha, 2.0 / N, N)
    A = oracle.dense(2, N, alpha, a)
    t = tau.generator(2, N, alpha, a)
    E = np.eye((N - 1) ** 2)
    Minv = np.stack([tau.tau_apply_gen(t, E[:, k]) for k in range(E.shape[0])], 1)
    ev = np.linalg.eigvals(Minv @ A).real
    assert ev.min() > 0.6 and ev.max() < 1.01


@pytest.mark.parametrize("d,N,shape", [(1, 12, None), (2, 6, None), (2, 8, (7, 4)), (2, 10, (9, 5)), (3, 6, None),
                                       (3, 8, (7, 3, 5))])
def test_restricted_preconditioner_is_a_principal_submatrix(d, N, shape):
    # off the power-of-two squares the preconditioner is the inverse of the tau matrix on
    # the embedding's n' nodes, restricted to the operator's nodes: check against the
    # two-Hankel form of that tau matrix, inverted densely
    alpha = 1.3
    a = oracle.coeffs(d, alpha, 2.0 / N, N)
    n, n2 = N - 1, tau.embedding_nodes(N)
    nk = [n] * d if shape is None else list(shape)
    t = np.zeros((n2,) * d)
    t[tuple([slice(0, n)] * d)] = tau.generator(d, N, alpha, a)
    Minv = np.linalg.inv(tau.tau_matrix_gen(t))
    # operator nodes in the n'-grid's flat (numpy) order
    keep = np.zeros((n2,) * d, dtype=bool)
    keep[tuple(slice(0, k) for k in reversed(nk))] = True
    sel = np.flatnonzero(keep.ravel())
    r = np.random.default_rng(5).standard_normal(int(np.prod(nk)))
    z = tau.tau_apply(d, N, alpha, a, r, shape=shape)
    assert np.abs(z - Minv[np.ix_(sel, sel)] @ r).max() < 1e-12 * np.abs(z).max()
    if shape is None and n == n2:
        assert np.array_equal(z, tau.tau_apply_gen(tau.generator(d, N, alpha, a), r))


def test_embedding_nodes_and_the_excluded_sizes():
    # P = max(8, 2^ceil(log2(2n - 1))): n' = n on power-of-two N, n' < n only for N = 2^k + 1
    assert [tau.embedding_nodes(N) for N in (4, 8, 16, 1024)] == [3, 7, 15, 1023]
    assert [tau.embedding_nodes(N) for N in (6, 12, 100, 700)] == [7, 15, 127, 1023]
    assert all(tau.embedding_nodes(N) == N - 2 for N in (5, 9, 17, 1025))
    with pytest.raises(ValueError):
        tau.tau_apply(2, 17, 1.0, oracle.coeffs(2, 1.0, 2.0 / 17, 17), np.zeros(16 * 16))
