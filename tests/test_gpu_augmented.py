"""GPU parity of the augmented SQD form (Section 3, eq. augmentedKKT) with
its signed factorisation P'AP = L S L' (Section 2: strong factorisability
of symmetric quasi-definite matrices, no pivoting), against the oracle.

Bars:
  assembly   values within 1e-13 * max|A| of the oracle's augmented matrix
  factor     L within 1e-10 * max|L| (FP64) of the oracle's unit LDL' factor
             scaled by sqrt|D| column by column, S = sign(D) equal to the
             block signs, ||P'AP - L S L'||_F / ||A||_F <= 1e-12; FP32 L
             within 2e-4 * max|L|
  K solve    backward error <= 1e-13 against the primal condensed K
  IPM        |f - f_ref| / max(1, |f_ref|) <= 1e-6 and the oracle's checker
             recomputes P, D, C <= 1e-6 from the returned vectors
"""
import numpy as np
import pytest
import scipy.sparse as sp

from _util import sparse_from_panels
from oracle import checker, ipm as oipm, kkt as okkt, model, symbolic as osym
from oracle import cholesky as ochol
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda:0")


MATS = {
    "lp_small": lambda: w.lp_small(2),
    "qp": lambda: w.qp_instance(900, 17),
    "nlp": lambda: w.nlp_grid(30, 26),
    "block": lambda: w.lp_block(nblocks=4, block_rows=200, block_cols=400, link_cols_per_block=20),
    "random_lp": lambda: w.random_lp(1500, 600, 6, 5),
}


@pytest.mark.parametrize("which", list(MATS))
@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_signed_factor_matches_oracle_ldlt(which, precision):
    p = MATS[which]()
    print(f"case augmented factor {which} precision={precision}", flush=True)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.5, 2.0, p.n); lam = rng.uniform(0.1, 1, p.m)
    sig_s = rng.uniform(0.01, 100, p.m); sig_x = rng.uniform(0, 10, p.n)
    s = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_AUGMENTED, precision=precision).bind()
    s.assemble(dev(x), dev(lam), dev(sig_s), dev(sig_x), precision)
    av = s.k_values()
    rp, ci = s.k_pattern()
    N = p.n + p.m
    Ag = sp.csr_matrix((av, ci, rp), shape=(N, N))
    H = model.hessian(p, x, lam); J = model.jacobian(p, x).tocsr()
    dd = 1e-8
    A = okkt.augmented_matrix(H, J, 1.0 / sig_s - dd, np.ones(p.m), sig_x, 1e-8, dd)
    assert abs(Ag - sp.tril(A)).max() <= 1e-13 * abs(A).max()
    info = s.factor(precision)
    assert info["status"] == 0
    sym = s.symbolic()
    Lg = sparse_from_panels(sym, s.factor_values()).toarray()
    Hl = sp.tril(H).tocsr()
    ref = osym.analyze(osym.augmented_pattern(p.n, p.m, J.indptr, J.indices, Hl.indptr, Hl.indices), N)
    assert np.array_equal(sym["perm"], ref["perm"])
    F = ochol.SparseFactor(ref["perm"], ref["structs"]).factor_ldlt(A)
    sign = np.concatenate([np.ones(p.n), -np.ones(p.m)])[ref["perm"]]
    assert np.array_equal(np.sign(F.D), sign)
    Lo = F.to_dense() * np.sqrt(np.abs(F.D))[None, :]
    tol = 1e-10 if precision == L.PDIPM_FP64 else 2e-4
    assert np.max(np.abs(Lg - Lo)) <= tol * np.max(np.abs(Lo))
    if precision == L.PDIPM_FP64:
        Ap = A.toarray()[np.ix_(ref["perm"], ref["perm"])]
        assert np.linalg.norm(Ap - Lg @ np.diag(sign) @ Lg.T) / np.linalg.norm(Ap) <= 1e-12
    # K solve through the augmented factor, refined against K
    K = okkt.condensed_matrix(H, J, sig_s, sig_x, 1e-8)
    b = rng.standard_normal(p.n)
    xs, _ = s.solve_kkt(dev(b))
    xs = xs.cpu().numpy()
    res = np.max(np.abs(K @ xs - b)) / (K.diagonal().max() * np.max(np.abs(xs)) + np.max(np.abs(b)))
    assert res <= 1e-13, res


CASES = {
    "lp_small": lambda: w.lp_small(0),
    "qp_batch_member": lambda: w.qp_instance(900, 17),
    "nlp_grid": lambda: w.nlp_grid(40, 36),
    "lp_block_small": lambda: w.lp_block(nblocks=4, block_rows=200, block_cols=400, link_cols_per_block=20),
    "qp_param_small": lambda: w.qp_param(20, 30).base,
}
_REF = {}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_ipm_augmented_form_matches_oracle(name, precision):
    if name not in _REF:
        p = CASES[name]()
        r = oipm.solve(p, tol=1e-9, form="augmented")
        assert r["status"] == 0
        _REF[name] = (p, r)
    p, ref = _REF[name]
    print(f"case augmented {name} precision={precision}", flush=True)
    s = L.IpmSolver(p, precision=precision, kkt_form=L.PDIPM_KKT_AUGMENTED).bind()
    res = s.solve()
    sol = s.solution()
    chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
    assert res["status"] == 0, res
    assert abs(res["f"] - ref["f"]) / max(1.0, abs(ref["f"])) <= 1e-6
    assert abs(chk["f"] - ref["f"]) / max(1.0, abs(ref["f"])) <= 1e-6
    assert chk["P"] <= 1e-6 and chk["D"] <= 1e-6 and chk["C"] <= 1e-6, chk


def test_augmented_form_reports_an_indefinite_hessian():
    p = w.nlp_grid_nonconvex(20, 20, 0, 0.5, 0.2, 5.0)
    s = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_AUGMENTED).bind()
    with pytest.raises(L.PdipmError) as e:
        s.solve()
    assert e.value.code == L.PDIPM_ERR_NUMERICAL
