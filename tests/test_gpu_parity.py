"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle.

Error measures (floating point; the paper fixes no precision):
  e_rel = ||y - y_ref||_inf / ||y_ref||_inf
  e_sc  = ||y - y_ref||_inf / || |A| |u| ||_inf   (size of the sum's terms)
Both the FFT path and the oracle's explicit sum are backward stable only with
respect to |A||u|; e_sc is gated everywhere (1e-14 FP64, 1e-6 FP32) and e_rel
where the operator is well conditioned for the input (1e-12 FP64, 1e-5 FP32).
"""
import numpy as np
import pytest

import oracle
from paper_1804_02718_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1804_02718_amd import fl
    fl.load()
    return torch.device("cuda:0")


def _fl():
    from paper_1804_02718_amd import fl
    return fl


def _t(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def _errs(y, ref, absref):
    d = np.abs(y - ref).max()
    return d / np.abs(ref).max(), d / np.abs(absref).max()


# ---------------------------------------------------------------------------
# coefficients and eigenvalues
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,N,alpha", [(1, 2, 1.5), (1, 3, 0.3), (1, 17, 1.0), (1, 100, 1.9), (1, 1025, 0.7),
                                       (2, 2, 1.5), (2, 3, 0.3), (2, 5, 1.9), (2, 17, 1.0), (2, 32, 1.5),
                                       (2, 100, 0.7), (2, 257, 1.2), (3, 2, 1.0), (3, 3, 1.7), (3, 6, 0.4),
                                       (3, 9, 1.2), (3, 16, 1.9), (1, 40, 0.05), (1, 40, 1.99), (2, 33, 0.05),
                                       (2, 33, 1.99), (3, 9, 0.05), (3, 9, 1.99)])
def test_coefficients_match_oracle(dev, d, N, alpha):
    h = 2.0 / N
    op = _fl().Operator(d, alpha, h, N)
    a_gpu = op.coeffs()
    a_ref = oracle.coeffs(d, alpha, h, N)
    rel = np.abs(a_gpu - a_ref) / np.abs(a_ref)
    assert rel.max() < 1e-13, (rel.max(), np.unravel_index(rel.argmax(), rel.shape))
    assert op.a0 == a_gpu.flat[0]
    assert op.c == pytest.approx(oracle.const(d, alpha), rel=1e-15)
    op.close()


@pytest.mark.parametrize("d,N,alpha", [(1, 5, 1.3), (1, 300, 0.6), (1, 1025, 1.9), (2, 5, 1.3), (2, 32, 0.6),
                                       (3, 7, 1.5)])
def test_symbol_is_fft_of_embedded_generator(dev, d, N, alpha):
    h = 2.0 / N
    op = _fl().Operator(d, alpha, h, N)
    P, Q, n = op.P, op.Q, op.n
    a = oracle.coeffs(d, alpha, h, N)
    c = oracle.const(d, alpha)
    # generator t_m = -c a_{|m|}, |m_i| <= n-1, embedded with period P, zero in the gap
    idx = np.arange(P)
    f = np.where(idx <= n - 1, idx, np.where(idx >= P - (n - 1), P - idx, -1))
    mask = f >= 0
    fi = np.where(mask, f, 0)
    if d == 1:
        emb = -c * a[fi] * mask
    elif d == 2:
        emb = -c * a[np.ix_(fi, fi)] * np.outer(mask, mask)
    else:
        emb = -c * a[np.ix_(fi, fi, fi)] * (mask[:, None, None] & mask[None, :, None] & mask[None, None, :])
    lam = np.fft.fftn(emb).real / P ** d
    ref = lam[(slice(0, Q),) * d]
    got = op.symbol()
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    op.close()


# ---------------------------------------------------------------------------
# matvec against the explicit sum
# ---------------------------------------------------------------------------
APPLY_CASES = [(1, 2, 1.2), (1, 3, 0.5), (1, 9, 1.5), (1, 64, 1.9), (1, 100, 0.8), (1, 513, 1.1), (1, 1025, 0.4),
               (2, 2, 1.2), (2, 3, 0.5), (2, 4, 1.9), (2, 5, 1.0), (2, 9, 1.5), (2, 17, 0.2), (2, 32, 1.5),
               (2, 33, 1.1), (2, 64, 1.9), (2, 100, 0.8), (3, 2, 1.3), (3, 3, 0.6), (3, 5, 1.9), (3, 8, 1.2),
               (3, 12, 0.4), (3, 17, 1.6),
               # the ends of (0, 2): A near the identity, and near the 5- and 7-point Laplacians
               (1, 40, 0.05), (1, 40, 1.99), (2, 33, 0.05), (2, 33, 1.99), (2, 100, 0.05), (2, 100, 1.99),
               (3, 9, 0.05), (3, 9, 1.99)]


@pytest.mark.parametrize("d,N,alpha", APPLY_CASES)
def test_apply_fp64_random(dev, d, N, alpha):
    fl = _fl()
    h = 2.0 / N
    op = fl.Operator(d, alpha, h, N)
    u = inputs.uniform((N - 1) ** d, seed=1)
    a = oracle.coeffs(d, alpha, h, N)
    ref = oracle.apply(d, N, alpha, a, u)
    absref = oracle.apply(d, N, alpha, a, u, absmode=True)
    y = op.apply(_t(u)).cpu().numpy()
    e_rel, e_sc = _errs(y, ref, absref)
    assert e_sc < 1e-14, (e_rel, e_sc)
    assert e_rel < 1e-12, (e_rel, e_sc)
    op.close()


@pytest.mark.parametrize("d,N,alpha", APPLY_CASES)
def test_apply_fp32_random(dev, d, N, alpha):
    fl = _fl()
    h = 2.0 / N
    op = fl.Operator(d, alpha, h, N)
    u32 = inputs.uniform((N - 1) ** d, seed=2).astype(np.float32)
    u = u32.astype(np.float64)
    a = oracle.coeffs(d, alpha, h, N)
    ref = oracle.apply(d, N, alpha, a, u)
    absref = oracle.apply(d, N, alpha, a, u, absmode=True)
    y = op.apply(_t(u32, torch.float32)).cpu().numpy().astype(np.float64)
    e_rel, e_sc = _errs(y, ref, absref)
    assert e_sc < 1e-6, (e_rel, e_sc)
    assert e_rel < 1e-5, (e_rel, e_sc)
    op.close()


def test_apply_c1_bump(dev):
    # 2D, N = 32 on (-1,1)^2, alpha = 1.5, u = (1-|x|^2)_+^{alpha/2}
    fl = _fl()
    N, alpha = 32, 1.5
    h = 2.0 / N
    u = inputs.bump(2, N, alpha)
    op = fl.Operator(2, alpha, h, N)
    a = oracle.coeffs(2, alpha, h, N)
    ref = oracle.apply(2, N, alpha, a, u)
    absref = oracle.apply(2, N, alpha, a, u, absmode=True)
    y = op.apply(_t(u)).cpu().numpy()
    e_rel, e_sc = _errs(y, ref, absref)
    assert e_rel < 1e-12 and e_sc < 1e-14, (e_rel, e_sc)
    y32 = op.apply(_t(u, torch.float32)).cpu().numpy().astype(np.float64)
    ref32 = oracle.apply(2, N, alpha, a, u.astype(np.float32).astype(np.float64))
    e_rel32, e_sc32 = _errs(y32, ref32, absref)
    assert e_rel32 < 1e-5 and e_sc32 < 1e-6, (e_rel32, e_sc32)
    op.close()


def _sample_rows(M, k, seed):
    rng = np.random.default_rng(seed)
    head = np.arange(min(8, M))
    tail = np.arange(max(0, M - 8), M)
    mid = np.arange(M // 2 - 4, M // 2 + 4)
    rnd = rng.choice(M, size=k, replace=False)
    return np.unique(np.concatenate([head, tail, mid, rnd]))


@pytest.mark.parametrize("alpha", [0.5, 1.0, 1.5, 1.9])
def test_apply_c2_full_size_sampled(dev, alpha):
    # 2D, N = 1024: Gaussian on (-4,4)^2 and seeded uniform u on (-1,1)^2, FP64 and FP32,
    # in the launch configuration the benchmark times; checked on sampled rows.
    fl = _fl()
    N = 1024
    M = (N - 1) ** 2
    rows = _sample_rows(M, 48, seed=7)
    for lo, u in ((-4.0, inputs.gaussian(2, N)), (-1.0, inputs.uniform(M, seed=1))):
        h = -2.0 * lo / N
        op = fl.Operator(2, alpha, h, N)
        a = oracle.coeffs(2, alpha, h, N)
        ref = oracle.apply_rows(2, N, alpha, a, u, rows)
        absref = oracle.apply_rows(2, N, alpha, a, u, rows, absmode=True)
        y = op.apply(_t(u)).cpu().numpy()[rows]
        e_rel, e_sc = _errs(y, ref, absref)
        assert e_sc < 1e-14, ("fp64", lo, e_rel, e_sc)
        u32 = u.astype(np.float32)
        ref32 = oracle.apply_rows(2, N, alpha, a, u32.astype(np.float64), rows)
        y32 = op.apply(_t(u32, torch.float32)).cpu().numpy()[rows].astype(np.float64)
        e_rel32, e_sc32 = _errs(y32, ref32, absref)
        assert e_sc32 < 1e-6, ("fp32", lo, e_rel32, e_sc32)
        if lo == -1.0:  # random input: well conditioned, the literal gates hold
            assert e_rel < 1e-12 and e_rel32 < 1e-5, (e_rel, e_rel32)
        op.close()


@pytest.mark.timeout(900)
def test_apply_c2_as_benched_all_rows(dev):
    # The benchmark's workload exactly: 2D N = 1024 on (-4,4)^2, alpha = 1.5, u = exp(-|x|^2),
    # default kernel variants, against the oracle's explicit sum on every one of the 1,046,529
    # rows.  Both precisions take the FP32-rounded input, so one oracle sum serves both.
    # u >= 0, so |A||u| = 2 A_ii u - A u (the identity the oracle's |A||u| mode is pinned by).
    fl = _fl()
    N, alpha = 1024, 1.5
    h = 8.0 / N
    op = fl.Operator(2, alpha, h, N)
    u32 = inputs.gaussian(2, N).astype(np.float32)
    u = u32.astype(np.float64)
    y64 = op.apply(_t(u)).cpu().numpy()
    y32 = op.apply(_t(u32, torch.float32)).cpu().numpy().astype(np.float64)
    a = oracle.coeffs(2, alpha, h, N)
    print("oracle: explicit sum over all rows on %d threads" % oracle.num_threads(), flush=True)
    ref = oracle.apply(2, N, alpha, a, u)
    absref = 2.0 * (-oracle.const(2, alpha) * a[0, 0]) * u - ref
    kappa = np.abs(absref).max() / np.abs(ref).max()
    e_rel, e_sc = _errs(y64, ref, absref)
    e_rel32, e_sc32 = _errs(y32, ref, absref)
    print("C2 all rows: kappa_mv %.1f  fp64 e_rel %.3e e_sc %.3e  fp32 e_rel %.3e e_sc %.3e"
          % (kappa, e_rel, e_sc, e_rel32, e_sc32), flush=True)
    assert e_sc < 1e-14 and e_rel < 1e-12, (e_rel, e_sc)
    # FP32: the scaled gate; the literal relative error is kappa_mv times it (kappa_mv ~ 3e3 here)
    assert e_sc32 < 1e-6, (e_rel32, e_sc32)
    assert e_rel32 <= kappa * 1e-6
    op.close()


@pytest.mark.parametrize("N,alpha,nrows", [(130, 0.7, 24), (256, 1.2, 12)])
def test_apply_3d_p512_sampled(dev, N, alpha, nrows):
    # 3D with FFT length 512 per axis: N = 130 (n = 129) and the full N = 256 (255^3 unknowns)
    # of the Allen--Cahn workload, seeded uniform u in [-0.9, 0.9], FP64 and FP32, sampled rows
    fl = _fl()
    h = 2.0 / N
    M = (N - 1) ** 3
    op = fl.Operator(3, alpha, h, N)
    assert op.P == 512
    u = inputs.ac_initial(M, seed=3)
    rows = _sample_rows(M, nrows, seed=8)
    a = oracle.coeffs(3, alpha, h, N)
    ref = oracle.apply_rows(3, N, alpha, a, u, rows)
    absref = oracle.apply_rows(3, N, alpha, a, u, rows, absmode=True)
    y = op.apply(_t(u)).cpu().numpy()[rows]
    e_rel, e_sc = _errs(y, ref, absref)
    assert e_sc < 1e-14 and e_rel < 1e-12, (e_rel, e_sc)
    u32 = u.astype(np.float32)
    ref32 = oracle.apply_rows(3, N, alpha, a, u32.astype(np.float64), rows)
    y32 = op.apply(_t(u32, torch.float32)).cpu().numpy()[rows].astype(np.float64)
    e_rel32, e_sc32 = _errs(y32, ref32, absref)
    assert e_sc32 < 1e-6 and e_rel32 < 1e-5, (e_rel32, e_sc32)
    op.close()


@pytest.mark.parametrize("d,N,alpha", [(2, 65, 1.1), (2, 129, 0.9), (2, 257, 1.6), (2, 513, 0.6), (2, 1024, 1.9),
                                       (3, 129, 1.3), (3, 200, 0.8)])
def test_every_kernel_variant_matches_oracle(dev, d, N, alpha):
    # every compiled variant (points per thread, tile width, rows per block) computes
    # the same operator: FP64 and FP32 against the oracle on sampled rows
    fl = _fl()
    h = 2.0 / N
    M = (N - 1) ** d
    op = fl.Operator(d, alpha, h, N)
    u = inputs.uniform(M, seed=4)
    u32 = u.astype(np.float32)
    rows = _sample_rows(M, 24, seed=9)
    a = oracle.coeffs(d, alpha, h, N)
    ref = oracle.apply_rows(d, N, alpha, a, u, rows)
    ref32 = oracle.apply_rows(d, N, alpha, a, u32.astype(np.float64), rows)
    absref = oracle.apply_rows(d, N, alpha, a, u, rows, absmode=True)
    for prec, uu, rr, gate in (("fp64", _t(u), ref, 1e-14), ("fp32", _t(u32, torch.float32), ref32, 1e-6)):
        for k, desc in enumerate(op.variants(prec)):
            op.select_variant(prec, k)
            y = op.apply(uu).cpu().numpy()[rows].astype(np.float64)
            e_rel, e_sc = _errs(y, rr, absref)
            assert e_sc < gate, (prec, k, desc, e_rel, e_sc)
    best, ms = op.autotune("fp32", reps=3)
    assert 0 <= best < len(ms) and ms[best] == min(ms)
    y = op.apply(_t(u32, torch.float32)).cpu().numpy()[rows].astype(np.float64)
    assert _errs(y, ref32, absref)[1] < 1e-6
    op.close()


def test_apply_deterministic_and_stream_ordered(dev):
    fl = _fl()
    N = 256
    op = fl.Operator(2, 1.3, 2.0 / N, N)
    u = _t(inputs.uniform((N - 1) ** 2, seed=9))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        y1 = op.apply(u)
        y2 = op.apply(u)
    s.synchronize()
    assert torch.equal(y1, y2)
    op.close()


def test_apply_rejects_overlap_and_dtype_mix(dev):
    fl = _fl()
    op = fl.Operator(2, 1.0, 0.25, 8)
    u = torch.zeros(49, dtype=torch.float64, device="cuda:0")
    with pytest.raises(fl.FlError):
        fl.fl_apply(op.handle, u, u)
    with pytest.raises(TypeError):
        fl.fl_apply(op.handle, u, torch.zeros(49, dtype=torch.float32, device="cuda:0"))
    op.close()


@pytest.mark.parametrize("d,N,alpha,gamma", [(1, 100, 0.9, 1.4), (2, 33, 0.7, 1.35), (2, 64, 1.5, 1.75),
                                             (3, 9, 1.2, 1.6)])
def test_gamma_below_two_coeffs_and_apply(dev, d, N, alpha, gamma):
    """Splitting parameter gamma < 2 (Sec. 2): coefficients and the FP64 matvec against the oracle."""
    fl = _fl()
    h = 2.0 / N
    op = fl.Operator(d, alpha, h, N, gamma=gamma)
    assert op.desc["gamma"] == gamma
    a_ref = oracle.coeffs(d, alpha, h, N, gamma=gamma)
    a_gpu = op.coeffs()
    rel = np.abs(a_gpu - a_ref) / np.abs(a_ref)
    assert rel.max() < 1e-13, rel.max()
    u = inputs.uniform((N - 1) ** d, 7)
    y = op.apply(torch.as_tensor(u, device="cuda:0")).cpu().numpy()
    ref = oracle.apply(d, N, alpha, a_ref, u)
    absref = oracle.apply(d, N, alpha, a_ref, u, absmode=True)
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(absref).max()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_gamma_rejects(dev):
    fl = _fl()
    with pytest.raises(fl.FlError):
        fl.Operator(2, 1.5, 0.1, 20, gamma=1.4)  # gamma <= alpha
    with pytest.raises(fl.FlError):
        fl.Operator(2, 1.5, 0.1, 20, gamma=2.1)


# ---------------------------------------------------------------------------
# boxes: Nk intervals per axis, the square's coefficients (N = max Nk), the
# scheme's sums bounded by each axis's own node count (Sec. 2, Sec. 4)
# ---------------------------------------------------------------------------
BOX_CASES = [(2, (40, 17), 1.3), (2, (17, 40), 0.5), (2, (2, 9), 1.9), (2, (33, 2), 1.0), (2, (100, 64), 1.5),
             (2, (130, 7), 0.8), (3, (9, 5, 7), 1.2), (3, (5, 9, 2), 0.6), (3, (2, 2, 9), 1.7),
             (3, (17, 12, 6), 1.9), (3, (12, 17, 17), 0.4), (3, (33, 3, 20), 1.5)]


@pytest.mark.parametrize("d,Nk,alpha", BOX_CASES)
def test_box_apply_fp64_fp32(dev, d, Nk, alpha):
    fl = _fl()
    N = max(Nk)
    h = 1.0 / N
    op = fl.Operator(d, alpha, h, None, Nk=Nk)
    shape = [k - 1 for k in Nk]
    M = int(np.prod(shape))
    assert op.desc["nk"] == shape and op.M == M and op.N == N
    a = oracle.coeffs(d, alpha, h, N)
    u = inputs.uniform(M, seed=21)
    ref = oracle.apply(d, N, alpha, a, u, shape=shape)
    absref = oracle.apply(d, N, alpha, a, u, absmode=True, shape=shape)
    y = op.apply(_t(u)).cpu().numpy()
    e_rel, e_sc = _errs(y, ref, absref)
    assert e_sc < 1e-14 and e_rel < 1e-12, (e_rel, e_sc)
    u32 = u.astype(np.float32)
    ref32 = oracle.apply(d, N, alpha, a, u32.astype(np.float64), shape=shape)
    y32 = op.apply(_t(u32, torch.float32)).cpu().numpy().astype(np.float64)
    e_rel, e_sc = _errs(y32, ref32, absref)
    assert e_sc < 1e-6 and e_rel < 1e-5, (e_rel, e_sc)
    op.close()


@pytest.mark.parametrize("d,Nk,alpha", [(2, (1025, 300), 1.5), (2, (257, 1024), 0.7), (3, (257, 100, 40), 1.2),
                                        (3, (60, 200, 129), 1.9)])
def test_box_apply_large_sampled_every_variant(dev, d, Nk, alpha):
    fl = _fl()
    N = max(Nk)
    h = 1.0 / N
    op = fl.Operator(d, alpha, h, None, Nk=Nk)
    shape = [k - 1 for k in Nk]
    M = int(np.prod(shape))
    u = inputs.uniform(M, seed=5)
    u32 = u.astype(np.float32)
    rows = _sample_rows(M, 16, seed=17)
    a = oracle.coeffs(d, alpha, h, N)
    ref = oracle.apply_rows(d, N, alpha, a, u, rows, shape=shape)
    ref32 = oracle.apply_rows(d, N, alpha, a, u32.astype(np.float64), rows, shape=shape)
    absref = oracle.apply_rows(d, N, alpha, a, u, rows, absmode=True, shape=shape)
    for prec, uu, rr, gate in (("fp64", _t(u), ref, 1e-14), ("fp32", _t(u32, torch.float32), ref32, 1e-6)):
        for k, desc in enumerate(op.variants(prec)):
            op.select_variant(prec, k)
            y = op.apply(uu).cpu().numpy()[rows].astype(np.float64)
            e_rel, e_sc = _errs(y, rr, absref)
            assert e_sc < gate, (prec, k, desc, e_rel, e_sc)
    op.close()


@pytest.mark.parametrize("d,Nk,alpha", [(2, (60, 25), 1.4), (3, (14, 9, 6), 0.9)])
@pytest.mark.parametrize("solver", ["cg64", "refine"])
def test_box_poisson_vs_dense(dev, d, Nk, alpha, solver):
    fl = _fl()
    N = max(Nk)
    h = 1.0 / N
    op = fl.Operator(d, alpha, h, None, Nk=Nk)
    shape = [k - 1 for k in Nk]
    a = oracle.coeffs(d, alpha, h, N)
    A = oracle.dense(d, N, alpha, a, shape=shape)
    f = inputs.uniform(A.shape[0], seed=8) + 0.5
    uref = oracle.solve_dense(A, f)
    u, info = op.poisson_solve(_t(f), tol=1e-11, solver=solver)
    ug = u.cpu().numpy()
    assert np.linalg.norm(f - A @ ug) <= 1.05e-11 * np.linalg.norm(f)
    assert np.abs(ug - uref).max() <= 2e-11 * np.linalg.cond(A) * np.abs(uref).max()
    op.close()


def test_box_allen_cahn_general_vs_oracle(dev):
    # (0, 1) x (0, 0.4) with u = -1 outside, shifted field ubar = u + 1 (Sec. 5.3 form)
    fl = _fl()
    N, alpha, delta, tau = 40, 1.3, 0.05, 5e-4
    h = 1.0 / N
    Nk = fl.box_intervals([1.0, 0.4], h)
    assert Nk == [40, 16]
    op = fl.Operator(2, alpha, h, None, Nk=Nk)
    shape = [k - 1 for k in Nk]
    a = oracle.coeffs(2, alpha, h, N)
    A = oracle.dense(2, N, alpha, a, shape=shape)
    x = h * np.arange(1, Nk[0])
    y = h * np.arange(1, Nk[1])
    r = np.sqrt((x[None, :] - 0.5) ** 2 + (y[:, None] - 0.2) ** 2)
    ub = (np.tanh((0.12 - r) / (np.sqrt(2) * delta)) + 1.0).ravel()
    gamma = delta ** -alpha
    ref = ub.copy()
    u = _t(ub)
    for _ in range(3):
        info = op.allen_cahn_step_gen(u, tau, 1.0, gamma, 1.0)
        assert info["relres"] <= 1e-8
        ref = oracle.ac_step_gen(2, N, alpha, a, ref, tau, 1.0, gamma, 1.0, 0.5, A=A)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-7 * np.abs(ref).max()
    op.close()


def test_box_rejects(dev):
    fl = _fl()
    with pytest.raises(fl.FlError):
        fl.fl_coeffs_box(2, 1.0, 2.0, 0.1, [10, 1])
    with pytest.raises(fl.FlError):
        fl.fl_coeffs_box(3, 1.0, 2.0, 0.1, [10, 600, 4])
    with pytest.raises(fl.FlError):
        fl.fl_coeffs_box(2, 1.0, 0.9, 0.1, [10, 5])
    op = fl.Operator(2, 1.0, 0.1, None, Nk=[10, 5])
    with pytest.raises(ValueError):
        op.apply(torch.zeros(81, dtype=torch.float64, device="cuda:0"))
    net = fl.UNet(16, seed=1)
    op.set_preconditioner(net)
    with pytest.raises(fl.FlError):
        op.poisson_solve(torch.ones(36, dtype=torch.float64, device="cuda:0"), solver="fpcg")
    op.close()



def test_1d_apply_profiled_single_pass(dev):
    # d = 1 is one fused pass (forward, lambda, inverse) per vector pair
    fl = _fl()
    N = 1024
    op = fl.Operator(1, 1.3, 2.0 / N, N)
    u = _t(inputs.uniform(N - 1, seed=3))
    ms = fl.fl_apply_profiled(op.handle, u, torch.empty_like(u), 5)
    assert len(ms) == 1 and ms[0] > 0
    assert len(op.variants("fp32")) == 1 and len(op.variants("fp64")) == 1
    op.close()


@pytest.mark.parametrize("d,N,alpha", [(2, 1025, 1.3), (3, 300, 1.6), (3, 513, 0.9)])
def test_apply_largest_sizes_sampled(dev, d, N, alpha):
    # the largest operators of the built range (2D N = 1025 and 3D N = 513: n = P / 2, the
    # embedding exactly twice the grid) and a ragged 3D size at FFT length 1024; FP64 and
    # FP32 against the oracle's explicit sum on a few rows (head, tail and random)
    fl = _fl()
    h = 2.0 / N
    M = (N - 1) ** d
    op = fl.Operator(d, alpha, h, N)
    assert op.P == (2048 if d == 2 else 1024)
    rng = np.random.default_rng(31)
    rows = np.unique(np.concatenate([np.arange(4), np.arange(M - 4, M), rng.choice(M, 6, replace=False)]))
    u = inputs.uniform(M, seed=12)
    a = oracle.coeffs(d, alpha, h, N)
    ref = oracle.apply_rows(d, N, alpha, a, u, rows)
    absref = oracle.apply_rows(d, N, alpha, a, u, rows, absmode=True)
    y = op.apply(_t(u)).cpu().numpy()[rows]
    e_rel, e_sc = _errs(y, ref, absref)
    assert e_sc < 1e-14 and e_rel < 1e-12, (e_rel, e_sc)
    u32 = u.astype(np.float32)
    ref32 = oracle.apply_rows(d, N, alpha, a, u32.astype(np.float64), rows)
    y32 = op.apply(_t(u32, torch.float32)).cpu().numpy()[rows].astype(np.float64)
    e_rel32, e_sc32 = _errs(y32, ref32, absref)
    assert e_sc32 < 1e-6 and e_rel32 < 1e-5, (e_rel32, e_sc32)
    op.close()


@pytest.mark.parametrize("d,Nk,alpha", [(2, (1100, 1100), 1.3), (2, (2049, 2049), 0.7), (2, (4000, 4000), 1.9),
                                        (2, (3000, 700), 1.1), (2, (8193, 8193), 1.5), (2, (8193, 600), 0.9)])
def test_large_operator_sampled(dev, d, Nk, alpha):
    # 2D operators past the LDS kernels' FFT length (2048): the global-memory passes at
    # P = 4096, 8192 and 16384 (the largest, N = 8193), boxes among them; FP64 and FP32
    # against the oracle's explicit sum on sampled rows.  At P = 16384 the FP64 forward
    # row pass loops over rows (fewer workgroups than rows: 599 rows take a ragged last
    # round), so FP64 and FP32 are also compared on every row: a row the loop skipped or
    # took twice would differ by O(1)
    fl = _fl()
    N = max(Nk)
    h = 2.0 / N
    op = fl.Operator(d, alpha, h, None, Nk=Nk)
    assert op.P > 2048
    shape = [k - 1 for k in Nk]
    M = int(np.prod(shape))
    rows = _sample_rows(M, 8, seed=41)
    u = inputs.uniform(M, seed=14)
    a = oracle.coeffs(d, alpha, h, N)
    a_gpu = op.coeffs()
    sub = (slice(0, 40), slice(0, 40))
    assert np.abs(a_gpu[sub] / a[sub] - 1.0).max() < 1e-13
    assert np.abs(a_gpu[-3:, -3:] / a[-3:, -3:] - 1.0).max() < 1e-13
    assert a_gpu[0, 0] == pytest.approx(a[0, 0], rel=1e-13)
    ref = oracle.apply_rows(d, N, alpha, a, u, rows, shape=shape)
    absref = oracle.apply_rows(d, N, alpha, a, u, rows, absmode=True, shape=shape)
    y = op.apply(_t(u)).cpu().numpy()[rows]
    e_rel, e_sc = _errs(y, ref, absref)
    assert e_sc < 1e-14 and e_rel < 1e-12, (e_rel, e_sc)
    u32 = u.astype(np.float32)
    ref32 = oracle.apply_rows(d, N, alpha, a, u32.astype(np.float64), rows, shape=shape)
    y32_full = op.apply(_t(u32, torch.float32))
    y32 = y32_full.cpu().numpy()[rows].astype(np.float64)
    e_rel32, e_sc32 = _errs(y32, ref32, absref)
    assert e_sc32 < 1e-6 and e_rel32 < 1e-5, (e_rel32, e_sc32)
    y64_full = op.apply(_t(u))
    assert bool(torch.isfinite(y64_full).all()) and bool(torch.isfinite(y32_full).all())
    row_gap = float((y64_full - y32_full.double()).abs().max() / y64_full.abs().max())
    assert row_gap < 1e-3, row_gap
    op.close()


def test_large_operator_limits(dev):
    # per-pass timing, the autotuner and batches refuse FFT lengths above 2048
    fl = _fl()
    N = 1100
    op = fl.Operator(2, 1.0, 2.0 / N, N)
    f = torch.ones(op.M, dtype=torch.float64, device="cuda:0")
    with pytest.raises(fl.FlError):
        fl.fl_apply_profiled(op.handle, f, torch.empty_like(f), 2)
    with pytest.raises(fl.FlError):
        op.autotune("fp64", reps=1)
    assert op.variants("fp64") == []
    with pytest.raises(fl.FlError):
        fl.Batch(2, [64, 1100], [1.0, 1.0], [2.0 / 64, 2.0 / 1100])
    op.close()


@pytest.mark.parametrize("solver", ["cg64", "refine"])
def test_large_operator_poisson_sampled_residual(dev, solver):
    # Poisson on a large operator (FFT length 4096): the library's FP64 residual meets the
    # tolerance, and the oracle's explicit sum of A u at sampled rows reproduces f there
    fl = _fl()
    N, alpha = 1100, 1.3
    h = 2.0 / N
    M = (N - 1) ** 2
    op = fl.Operator(2, alpha, h, N)
    f = inputs.gauss_sum(2, N, 4, seed=6)
    u, info = op.poisson_solve(_t(f), tol=1e-10, solver=solver)
    assert info["relres"] <= 1e-10
    rows = _sample_rows(M, 16, seed=3)
    a = oracle.coeffs(2, alpha, h, N)
    ug = u.cpu().numpy()
    Au = oracle.apply_rows(2, N, alpha, a, ug, rows)
    absAu = oracle.apply_rows(2, N, alpha, a, ug, rows, absmode=True)
    assert np.abs(Au - f[rows]).max() <= 1e-9 * np.abs(absAu).max() + 1e-9 * np.abs(f).max()
    op.close()


def test_large_operator_allen_cahn_step_sampled(dev):
    # one semi-implicit step on a large operator: at sampled rows the oracle's sums of A u and
    # A u+ satisfy (I + theta s A) u+ = u - (1 - theta) s A u + tau (u - u^3)
    fl = _fl()
    N, alpha, tau, eps, theta = 1100, 1.2, 1e-3, 0.05, 0.5
    h = 2.0 / N
    M = (N - 1) ** 2
    op = fl.Operator(2, alpha, h, N)
    u0 = inputs.ac_initial(M, seed=3)
    u = _t(u0)
    info = op.allen_cahn_step(u, tau, eps, theta=theta, tol=1e-11, solver="cg64")
    assert info["relres"] <= 1e-11
    rows = _sample_rows(M, 16, seed=5)
    a = oracle.coeffs(2, alpha, h, N)
    u1 = u.cpu().numpy()
    s = tau * eps * eps
    Au0 = oracle.apply_rows(2, N, alpha, a, u0, rows)
    Au1 = oracle.apply_rows(2, N, alpha, a, u1, rows)
    lhs = u1[rows] + theta * s * Au1
    rhs = u0[rows] - (1 - theta) * s * Au0 + tau * (u0[rows] - u0[rows] ** 3)
    scale = np.abs(oracle.apply_rows(2, N, alpha, a, u1, rows, absmode=True)).max() * s + 1.0
    assert np.abs(lhs - rhs).max() <= 1e-9 * scale
    op.close()
