"""fl_apply_noalloc (the matvec with its workspaces in the library's static per-GPU
array) through the C-ABI, against fl_apply and the FP64 oracle: two calls in a
row, the second on a smaller operator, in both precisions; and the size limits."""
import numpy as np
import pytest

import oracle
from paper_1804_02718_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1804_02718_amd import fl as _fl
    _fl.load()
    return _fl


def _rows(M, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(min(8, M)), np.arange(max(0, M - 8), M),
                                     rng.choice(M, size=min(k, M), replace=False)]))


def _check(fl, d, N, alpha, dtype, seed):
    h = 2.0 / N
    op = fl.Operator(d, alpha, h, N)
    M = op.M
    u_np = inputs.uniform(M, seed=seed)
    if dtype == torch.float32:
        u_np = u_np.astype(np.float32).astype(np.float64)
    u = torch.as_tensor(u_np, dtype=dtype, device="cuda:0")
    y_ref = fl.fl_apply(op.handle, u, torch.empty_like(u))
    # fill the output with NaN first: every entry must be written
    y = torch.full_like(u, float("nan"))
    fl.fl_apply_noalloc(op.handle, u, y)
    torch.cuda.synchronize()
    # same kernels and variant as fl_apply: the same bits
    assert torch.equal(y, y_ref), (d, N, dtype)
    rows = _rows(M, 64, seed + 1)
    a = oracle.coeffs(d, alpha, h, N)
    ref = oracle.apply_rows(d, N, alpha, a, u_np, rows)
    absref = oracle.apply_rows(d, N, alpha, a, u_np, rows, absmode=True)
    got = y.cpu().numpy()[rows].astype(np.float64)
    e_sc = np.abs(got - ref).max() / np.abs(absref).max()
    e_rel = np.abs(got - ref).max() / np.abs(ref).max()
    if dtype == torch.float64:
        assert e_sc < 1e-14 and e_rel < 1e-12, (d, N, e_sc, e_rel)
    else:
        assert e_sc < 1e-6 and e_rel < 1e-5, (d, N, e_sc, e_rel)
    op.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_apply_two_calls_second_smaller(fl, dtype):
    # the benchmark's 2D size, then a smaller 2D operator, then a 3D one within the limit
    _check(fl, 2, 1024, 1.5, dtype, seed=41)
    _check(fl, 2, 100, 0.8, dtype, seed=42)
    _check(fl, 3, 33, 1.2, dtype, seed=43)


def test_noalloc_1d(fl):
    _check(fl, 1, 1025, 1.3, torch.float64, seed=44)
    _check(fl, 1, 17, 0.6, torch.float32, seed=45)


def test_noalloc_rejects_what_does_not_fit(fl):
    # 3D FFT length 512 in FP64 needs far more than the 64 MiB static workspace
    op = fl.Operator(3, 1.2, 2.0 / 200, 200)
    u = torch.zeros(op.M, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(u)
    with pytest.raises(fl.FlError) as e:
        fl.fl_apply_noalloc(op.handle, u, y)
    assert e.value.args[0].startswith("FL_E_INVAL")
    assert "64 MiB" in str(e.value)
    # overlap and null checks happen before any GPU work
    with pytest.raises(fl.FlError):
        fl.fl_apply_noalloc(op.handle, u, u)
    op.close()
