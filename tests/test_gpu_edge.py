"""GPU edge cases through the C ABI, against closed forms and the oracle:
no constraints (separable box QP: x* = clip(-c/q, l, u)), one dense
constraint row (dense K; multiplier from bisection), free and one-sided
variables, a single variable, and batches holding such instances.

Bars: closed-form x within 1e-6 (absolute; solved to tol 1e-10, the dense
row to 1e-12, tolerances at which the oracle meets the same bar); otherwise
the parity rule
(|f - f_ref| / max(1, |f_ref|) <= 1e-6 and the oracle's checker P, D, C <=
1e-6 from the returned vectors)."""
import numpy as np
import pytest

from oracle import checker, ipm as oipm
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _diag_q(n, q):
    return w.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), q)


def _box_qp(n, seed, with_row=False):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.5, 2.0, n)
    c = rng.standard_normal(n) * 2
    xl = rng.uniform(-1.0, 0.0, n)
    xu = xl + rng.uniform(0.5, 3.0, n)
    p = w.Problem(n=n, m=0, c=c, b=np.zeros(0), Q=_diag_q(n, q), xl=xl, xu=xu, name=f"box{n}")
    if with_row:
        a = rng.uniform(0.2, 1.0, n)
        x_free = np.clip(-c / q, xl, xu)
        p.m = 1
        p.A = w.CSR(1, n, np.array([0, n], dtype=np.int64), np.arange(n, dtype=np.int32), a)
        p.b = np.array([float(a @ x_free) + 0.3 * float(a @ (xu - x_free))])
    return p, q


def _solve(p, precision, tol=1e-6):
    s = L.IpmSolver(p, precision=precision, tol=tol).bind()
    r = s.solve()
    return r, s.solution()


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
@pytest.mark.parametrize("n", [1, 37, 400])
def test_unconstrained_box_qp_closed_form(n, precision):
    p, q = _box_qp(n, 11 + n)
    r, sol = _solve(p, precision, tol=1e-10)
    assert r["status"] == 0
    assert np.max(np.abs(sol["x"] - np.clip(-p.c / q, p.xl, p.xu))) <= 1e-6


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_one_dense_row_bisection(precision):
    p, q = _box_qp(300, 5, with_row=True)
    a, beta = p.A.val, p.b[0]

    def x_of(nu):
        return np.clip((a * nu - p.c) / q, p.xl, p.xu)

    lo, hi = 0.0, 1.0
    while a @ x_of(hi) < beta:
        hi *= 2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if a @ x_of(mid) < beta else (lo, mid)
    nu = 0.5 * (lo + hi)
    # at tol 1e-10 the oracle itself is 3.6e-6 away from the bisection point
    r, sol = _solve(p, precision, tol=1e-12)
    assert r["status"] == 0
    assert np.max(np.abs(sol["x"] - x_of(nu))) <= 1e-6
    assert abs(sol["lam"][0] - nu) <= 1e-5 * max(1.0, nu)


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_free_and_one_sided_variables(precision):
    p = w.qp_instance(240, 31)
    rng = np.random.default_rng(3)
    kind = rng.integers(0, 4, p.n)           # 0 box, 1 free, 2 lower only, 3 upper only
    xl, xu = p.xl.copy(), p.xu.copy()
    xl[(kind == 1) | (kind == 3)] = -np.inf
    xu[(kind == 1) | (kind == 2)] = np.inf
    p.xl, p.xu = xl, xu
    ref = oipm.solve(p, tol=1e-9)
    assert ref["status"] == 0
    r, sol = _solve(p, precision)
    assert r["status"] == 0
    chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
    assert abs(chk["f"] - ref["f"]) / max(1.0, abs(ref["f"])) <= 1e-6
    assert chk["P"] <= 1e-6 and chk["D"] <= 1e-6 and chk["C"] <= 1e-6


def test_batch_with_edge_instances():
    ps = [_box_qp(1, 2)[0], _box_qp(50, 3)[0], _box_qp(120, 4, with_row=True)[0], w.qp_instance(80, 9), w.lp_small(1)]
    for precision in (L.PDIPM_FP64, L.PDIPM_FP32):
        b = L.BatchSolver(ps, precision=precision).bind()
        res, info = b.solve()
        sol = b.solution()
        for p, r, s in zip(ps, res, sol):
            ref = oipm.solve(p, tol=1e-9)
            assert r["status"] == 0, (p.name, r)
            chk = checker.check(p, s["x"], s["s"], s["lam"], s["zl"], s["zu"])
            assert abs(chk["f"] - ref["f"]) / max(1.0, abs(ref["f"])) <= 1e-6, p.name
            assert chk["P"] <= 1e-6 and chk["D"] <= 1e-6 and chk["C"] <= 1e-6, (p.name, chk)
    single = L.BatchSolver(ps[3:4], precision=L.PDIPM_FP64).bind()
    res, info = single.solve()
    assert res[0]["status"] == 0 and info["solved"] == 1
