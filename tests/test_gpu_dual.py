"""GPU parity of the dual condensed (normal-equations) form, Section 3,
eq. kkt_dual, against the oracle (through the C ABI).

Bars:
  assembly   M values within 1e-13 * max|M| of the oracle's
             delta_d I + S/Lambda + J D J' (D = (H + Sigma_x + delta_p)^-1)
  K solve    the K solve through M (d = D (r - J' M^-1 J D r), refined in
             FP64 against K) has backward error <= 1e-13 against the
             oracle's primal condensed K, and equals the oracle's dense
             solve of K within kappa(K) times that
  IPM        |f - f_ref| / max(1, |f_ref|) <= 1e-6 and the oracle's checker
             recomputes P, D, C <= 1e-6 from the returned vectors
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import checker, ipm as oipm, kkt as okkt, model
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda:0")


def _point(p, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.5, 2.0, p.n); lam = rng.uniform(0.1, 1, p.m)
    sig_s = rng.uniform(0.01, 100, p.m); sig_x = rng.uniform(0, 10, p.n)
    return x, lam, sig_s, sig_x


@pytest.mark.parametrize("which", ["lp", "qp", "block"])
def test_dual_assembly_matches_oracle(which):
    p = {"lp": lambda: w.lp_small(2), "qp": lambda: w.qp_instance(600, 8),
         "block": lambda: w.lp_block(nblocks=4, block_rows=200, block_cols=400, link_cols_per_block=20)}[which]()
    print(f"case dual assembly {which}", flush=True)
    x, lam, sig_s, sig_x = _point(p, 1)
    s = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_DUAL).bind()
    s.assemble(dev(x), dev(lam), dev(sig_s), dev(sig_x), L.PDIPM_FP64)
    mv = s.k_values()
    rp, ci = s.k_pattern()
    Mg = sp.csr_matrix((mv, ci, rp), shape=(p.m, p.m))
    J = model.jacobian(p, x)
    d = okkt.dual_scaling(model.hessian(p, x, lam), sig_x, 1e-8)
    dd = 1e-8
    # M's diagonal term delta_d + s/lambda equals 1/Sigma_s: s/lambda = 1/Sigma_s - delta_d
    Mo = sp.tril(okkt.dual_matrix(J, d, 1.0 / sig_s - dd, np.ones(p.m), dd))
    assert abs(Mg - Mo).max() <= 1e-13 * abs(Mo).max()
    # K solve through the factor of M, refined against K
    assert s.factor(L.PDIPM_FP64)["status"] == 0
    K = okkt.condensed_matrix(model.hessian(p, x, lam), J, sig_s, sig_x, 1e-8)
    b = np.random.default_rng(2).standard_normal(p.n)
    xs, info = s.solve_kkt(dev(b))
    xs = xs.cpu().numpy()
    kmax = K.diagonal().max()
    res = np.max(np.abs(K @ xs - b)) / (kmax * np.max(np.abs(xs)) + np.max(np.abs(b)))
    assert res <= 1e-13, res
    if p.n <= 1600:
        xd = np.linalg.solve(K.toarray(), b)
        kappa = np.linalg.cond(K.toarray())
        assert np.max(np.abs(xs - xd)) <= 1e-13 * kappa * np.max(np.abs(xd))


CASES = {
    "lp_small": lambda: w.lp_small(0),
    "lp_small_3": lambda: w.lp_small(3),
    "qp_batch_member": lambda: w.qp_instance(900, 17),
    "lp_block_small": lambda: w.lp_block(nblocks=4, block_rows=200, block_cols=400, link_cols_per_block=20),
}

_REF = {}


def _ref(name, maker):
    if name not in _REF:
        p = maker()
        r = oipm.solve(p, tol=1e-9, form="dual", dense_max=0)
        assert r["status"] == 0
        _REF[name] = (p, r)
    return _REF[name]


def _parity(p, res, sol, f_ref, tol=1e-6):
    chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
    assert res["status"] == 0, res
    assert abs(res["f"] - f_ref) / max(1.0, abs(f_ref)) <= tol
    assert abs(chk["f"] - f_ref) / max(1.0, abs(f_ref)) <= tol
    assert chk["P"] <= tol and chk["D"] <= tol and chk["C"] <= tol, chk
    return chk


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_ipm_dual_form_matches_oracle(name, precision):
    p, ref = _ref(name, CASES[name])
    print(f"case dual {name} precision={precision}", flush=True)
    s = L.IpmSolver(p, precision=precision, kkt_form=L.PDIPM_KKT_DUAL).bind()
    res = s.solve()
    _parity(p, res, s.solution(), ref["f"])


def _mid_block():
    return w.lp_block(nblocks=3, block_rows=1200, block_cols=2400, link_cols_per_block=100)


@pytest.mark.parametrize("form", [L.PDIPM_KKT_PRIMAL, L.PDIPM_KKT_DUAL])
@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_mid_size_block_lp_matches_oracle(form, precision):
    """3 blocks of 1,200 x 2,400 plus linking rows: dense fronts of about
    2,400 (primal: several 8-tile column groups and rank-512 outer blocks)
    and 1,200 (dual) columns run the blocked MFMA path; f_ref from the
    oracle's dual form at tol 1e-9."""
    p, ref = _ref("mid_block", _mid_block)
    print(f"case mid block form={form} precision={precision}", flush=True)
    s = L.IpmSolver(p, precision=precision, kkt_form=form).bind()
    res = s.solve()
    _parity(p, res, s.solution(), ref["f"])
