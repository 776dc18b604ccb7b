"""The paper's printed accuracy tables, every column, reproduced by the GPU path.

Sec. 5.1 Tables 1 and 2 (the operator on u = ((1 - x^2)(1 - y^2))^s, s = 1, 2)
and the Sec. 5.2 Example 5.2.1 / 5.2.2 tables (fractional Poisson with exact
solutions s = 2, 1) at h = 1/16 ... 1/512 on (-1, 1)^2 (N = 32 ... 1024).  As in
the paper, the exact operator is the scheme at h = 2^-12 (N = 8192, FFT length
16384: the large-operator passes), applied to u in FP64 and read at the coarse
nodes; the coarse operators and Poisson solves are the LDS path in FP64.  The
expected values are the paper's printed ones (tests/golden/*_all.txt); the
2-norm is (h^2 sum e^2)^(1/2).
"""
import os

import numpy as np
import pytest

from paper_1804_02718_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NF = 8192
COARSE = (32, 64, 128, 256, 512, 1024)
# Printed values carry 4 significant digits.  The operator tables are matched to
# 1.5 half-units of the last printed digit (a computed value that sits on a
# rounding boundary may round either way); the Poisson tables to 1e-3 relative,
# which allows for the residual the coarse FP64 solves reach (3e-12 at
# N = 1024, alpha = 1.4, where the largest gap, 4.9e-4, occurs).
HALF_UNITS = 1.5
RTOL_POISSON = 1e-3
_FINE = {}


def _read(name):
    rows = []
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                num, den = line[1].split("/")
                rows.append((float(line[0]), round(int(den) * 2), float(line[2]), float(line[3])))
    return rows


@pytest.fixture(scope="module")
def fl():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1804_02718_amd import fl as _fl
    _fl.load()
    return _fl


def _fine_rows(Nc):
    r = NF // Nc
    ii, jj = np.meshgrid(np.arange(1, Nc), np.arange(1, Nc), indexing="xy")
    return ((jj * r - 1) * (NF - 1) + (ii * r - 1)).ravel()


def _fine(fl, alpha, s):
    """The h = 2^-12 scheme applied to u (s) in FP64, at the coarse nodes of every column."""
    key = (alpha, s)
    if key not in _FINE:
        op = fl.Operator(2, alpha, 2.0 / NF, NF)
        assert op.P == 16384
        u = torch.as_tensor(inputs.paper_family(2, NF, s), device="cuda:0")
        y = op.apply(u)
        _FINE[key] = {Nc: y[torch.as_tensor(_fine_rows(Nc), device="cuda:0")].cpu().numpy() for Nc in COARSE}
        op.close()
        del u, y
    return _FINE[key]


def _norms(e, h):
    return np.abs(e).max(), np.sqrt(h * h * np.sum(e * e))


def _operator_errors(fl, alpha, s, Nc):
    op = fl.Operator(2, alpha, 2.0 / Nc, Nc)
    uc = torch.as_tensor(inputs.paper_family(2, Nc, s), device="cuda:0")
    yc = op.apply(uc).cpu().numpy()
    op.close()
    return _norms(yc - _fine(fl, alpha, s)[Nc], 2.0 / Nc)


def _poisson_errors(fl, alpha, s, Nc):
    op = fl.Operator(2, alpha, 2.0 / Nc, Nc)
    f = torch.as_tensor(_fine(fl, alpha, s)[Nc], device="cuda:0")
    # 3e-12: the FP64 residual the refinement reaches at N = 1024, alpha = 1.4 (cond near 1e5)
    uh, info = op.poisson_solve(f, tol=3e-12, solver="refine")
    op.close()
    return _norms(uh.cpu().numpy() - inputs.paper_family(2, Nc, s), 2.0 / Nc)


def _half_unit(v):
    return 0.5 * 10.0 ** (np.floor(np.log10(v)) - 3)


def _check_digits(got, einf, e2):
    for g, v in zip(got, (einf, e2)):
        assert abs(g - v) <= HALF_UNITS * _half_unit(v), (got, (einf, e2), abs(g - v) / _half_unit(v))


def _check_rel(got, einf, e2):
    assert got[0] == pytest.approx(einf, rel=RTOL_POISSON) and got[1] == pytest.approx(e2, rel=RTOL_POISSON), \
        (got, (einf, e2), (got[0] / einf - 1, got[1] / e2 - 1))


@pytest.mark.parametrize("alpha,Nc,einf,e2", _read("table1_operator_s1_all.txt"))
def test_table1_every_column(fl, alpha, Nc, einf, e2):
    _check_digits(_operator_errors(fl, alpha, 1.0, Nc), einf, e2)


@pytest.mark.parametrize("alpha,Nc,einf,e2", _read("table2_operator_s2_all.txt"))
def test_table2_every_column(fl, alpha, Nc, einf, e2):
    _check_digits(_operator_errors(fl, alpha, 2.0, Nc), einf, e2)


@pytest.mark.parametrize("alpha,Nc,einf,e2", _read("tab_poisson_s2_all.txt"))
def test_poisson_example_521_every_column(fl, alpha, Nc, einf, e2):
    _check_rel(_poisson_errors(fl, alpha, 2.0, Nc), einf, e2)


@pytest.mark.parametrize("alpha,Nc,einf,e2", _read("tab_poisson_s1_all.txt"))
def test_poisson_example_522_every_column(fl, alpha, Nc, einf, e2):
    _check_rel(_poisson_errors(fl, alpha, 1.0, Nc), einf, e2)


def test_golden_tables_complete():
    for name in ("table1_operator_s1_all.txt", "table2_operator_s2_all.txt", "tab_poisson_s2_all.txt",
                 "tab_poisson_s1_all.txt"):
        rows = _read(name)
        assert len(rows) == 18 and sorted({r[1] for r in rows}) == list(COARSE)
