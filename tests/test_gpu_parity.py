"""GPU parity of the HIP hot path against the CPU oracle (through the C ABI).

Bars (derived from the arithmetic of each step):
  factor      entries of L within 1e-10 * max|L| (FP64) of the oracle's
              L = chol(P'KP) for the same P; ||P'KP - LL'||_F/||K||_F <= 1e-12
  solve       ||K x - b||_inf / (||K||_inf ||x||_inf) <= 1e-13 (FP64), and
              after FP32 factor + FP64 refinement <= 1e-11
  evaluation  derivative values within 1e-12 relative of the oracle's
  assembly    K values within 1e-13 * max|K| of the oracle's condensed K
  IPM         |f - f_ref| / max(1, |f_ref|) <= 1e-6 and the oracle's checker
              recomputes P, D, C <= 1e-6 from the returned vectors
"""
import numpy as np
import pytest
import scipy.sparse as sp

from _util import dense_from_panels, sparse_from_panels
from oracle import checker, ipm as oipm, kkt as okkt, model, symbolic as osym
from oracle import cholesky as ochol
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda:0")


def _spd(n, seed, deg=4, dense_block=0):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, n, size=n * deg)
    cols = rng.integers(0, n, size=n * deg)
    B = sp.csr_matrix((rng.standard_normal(n * deg), (rows, cols)), shape=(n, n))
    K = (B @ B.T + sp.eye(n) * 0.5).tocsr()
    if dense_block:
        D = rng.standard_normal((dense_block, dense_block))
        Kd = sp.lil_matrix((n, n))
        Kd[:dense_block, :dense_block] = D @ D.T / dense_block
        K = (K + Kd.tocsr()).tocsr()
    return K


def _factor_case(K, precision):
    n = K.shape[0]
    Kl = sp.tril(K).tocsr(); Kl.sort_indices()
    opts = L.default_options(precision=precision)
    s = L.KktSolver(n, Kl.indptr, Kl.indices, opts).bind()
    s.set_values(dev(Kl.data))
    info = s.factor(precision)
    return s, Kl, info


@pytest.mark.parametrize("n,seed,dense", [(300, 1, 0), (1500, 2, 0), (700, 3, 450), (2000, 4, 1300)])
def test_factor_fp64_matches_oracle(n, seed, dense):
    K = _spd(n, seed, dense_block=dense)
    print(f"case n={n} seed={seed} dense={dense}", flush=True)
    s, Kl, info = _factor_case(K, L.PDIPM_FP64)
    assert info["status"] == 0
    sym = s.symbolic()
    Lg = sparse_from_panels(sym, s.factor_values())
    adj = osym.pattern_from_lower_csr(n, Kl.indptr, Kl.indices)
    ref = osym.analyze(adj, n)
    Fo = ochol.SparseFactor(ref["perm"], ref["structs"]).factor(K)
    Lo = Fo.to_dense()
    Ld = Lg.toarray()
    assert np.max(np.abs(Ld - Lo)) <= 1e-10 * np.max(np.abs(Lo))
    Kp = K.toarray()[np.ix_(ref["perm"], ref["perm"])]
    assert np.linalg.norm(Kp - Ld @ Ld.T) / np.linalg.norm(Kp) <= 1e-12
    b = np.random.default_rng(seed).standard_normal(n)
    x, sinfo = s.solve_kkt(dev(b))
    x = x.cpu().numpy()
    Kn = np.max(np.abs(K).sum(1))
    assert np.max(np.abs(K @ x - b)) / (Kn * np.max(np.abs(x))) <= 1e-13
    assert np.max(np.abs(x - Fo.solve(b))) <= 1e-8 * np.max(np.abs(x))


# (2600, 9, 1400): a dense front of 1,400 columns spans two groups of eight
# 128-column tile columns and two rank-512 outer blocks of the FP32 path
@pytest.mark.parametrize("n,seed,dense", [(900, 5, 0), (1800, 6, 1000), (2600, 9, 1400)])
def test_factor_fp32_with_fp64_refinement(n, seed, dense):
    K = _spd(n, seed, dense_block=dense)
    print(f"case n={n} seed={seed} dense={dense} fp32", flush=True)
    s, Kl, info = _factor_case(K, L.PDIPM_FP32)
    assert info["status"] == 0
    sym = s.symbolic()
    Ld = dense_from_panels(sym, s.factor_values())
    adj = osym.pattern_from_lower_csr(n, Kl.indptr, Kl.indices)
    ref = osym.analyze(adj, n)
    Lo = ochol.SparseFactor(ref["perm"], ref["structs"]).factor(K).to_dense()
    # FP32 factor: elementwise within single-precision growth of the oracle's
    assert np.max(np.abs(Ld - Lo)) <= 2e-4 * np.max(np.abs(Lo))
    b = np.random.default_rng(seed).standard_normal(n)
    x, sinfo = s.solve_kkt(dev(b))
    x = x.cpu().numpy()
    Kn = np.max(np.abs(K).sum(1))
    assert sinfo["ir_steps"] >= 1
    assert np.max(np.abs(K @ x - b)) / (Kn * np.max(np.abs(x))) <= 1e-11
    # the refined FP32 direction against the FP64 one: forward error within
    # kappa(K) times the backward errors of both solves
    s64, _, info64 = _factor_case(K, L.PDIPM_FP64)
    x64, _ = s64.solve_kkt(dev(b))
    x64 = x64.cpu().numpy()
    kappa = np.linalg.cond(K.toarray()) if n <= 3000 else 1e8
    rel = np.max(np.abs(x - x64)) / np.max(np.abs(x64))
    print(f"fp32+refinement vs fp64 direction: {rel:.2e} (kappa {kappa:.1e})", flush=True)
    assert rel <= 1e-12 * kappa


def test_not_positive_definite_is_reported():
    K = _spd(400, 7).tolil()
    K[123, 123] = -5.0
    K = K.tocsr()
    s, Kl, info = _factor_case(K, L.PDIPM_FP64)
    assert info["status"] == L.PDIPM_ERR_NOT_PD
    assert info["first_bad_col"] >= 0


@pytest.mark.parametrize("which", ["nlp", "qp", "lp"])
def test_evaluation_matches_oracle(which):
    p = {"nlp": lambda: w.nlp_grid(30, 26), "qp": lambda: w.qp_instance(500, 2),
         "lp": lambda: w.lp_small()}[which]()
    rng = np.random.default_rng(0)
    x = rng.uniform(0.5, 2.0, p.n); lam = rng.uniform(0.1, 1, p.m)
    s = L.IpmSolver(p).bind()
    f, gf, g, jv, hv = s.evaluate(dev(x), dev(lam))
    (jrp, jci), (hrp, hci) = s.patterns()
    J = sp.csr_matrix((jv.cpu().numpy(), jci, jrp), shape=(p.m, p.n))
    Hl = sp.csr_matrix((hv.cpu().numpy(), hci, hrp), shape=(p.n, p.n))
    Jo = model.jacobian(p, x)
    Ho = sp.tril(model.hessian(p, x, lam))
    tol = 1e-12
    assert abs(f - model.objective(p, x)) <= tol * max(1, abs(f))
    assert np.max(np.abs(gf.cpu().numpy() - model.gradient(p, x))) <= tol * max(1, np.max(np.abs(gf.cpu().numpy())))
    assert np.max(np.abs(g.cpu().numpy() - model.constraints(p, x))) <= tol * max(1, np.max(np.abs(g.cpu().numpy())))
    assert abs(J - Jo).max() <= tol * max(1, abs(Jo).max())
    assert abs(Hl - Ho).max() <= tol * max(1, abs(Ho).max())


@pytest.mark.parametrize("which", ["nlp", "qp"])
def test_assembly_matches_oracle(which):
    p = w.nlp_grid(24, 20) if which == "nlp" else w.qp_instance(600, 8)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.5, 2.0, p.n); lam = rng.uniform(0.1, 1, p.m)
    sig_s = rng.uniform(0.01, 100, p.m); sig_x = rng.uniform(0, 10, p.n)
    s = L.IpmSolver(p).bind()
    s.assemble(dev(x), dev(lam), dev(sig_s), dev(sig_x), L.PDIPM_FP64)
    kv = s.k_values()
    rp, ci = s.k_pattern()
    Kg = sp.csr_matrix((kv, ci, rp), shape=(p.n, p.n))
    Ko = sp.tril(okkt.condensed_matrix(model.hessian(p, x, lam), model.jacobian(p, x), sig_s, sig_x, 1e-8))
    assert abs(Kg - Ko).max() <= 1e-13 * abs(Ko).max()
    info = s.factor(L.PDIPM_FP64)
    assert info["status"] == 0


def _parity(p, res, sol, f_ref, tol=1e-6):
    chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
    assert res["status"] == 0, res
    assert abs(res["f"] - f_ref) / max(1.0, abs(f_ref)) <= tol
    assert abs(chk["f"] - f_ref) / max(1.0, abs(f_ref)) <= tol
    assert chk["P"] <= tol and chk["D"] <= tol and chk["C"] <= tol, chk
    return chk


def _strong_convexity(p):
    """Smallest eigenvalue of a diagonal Q (0 when not known)."""
    if p.Q is None or p.W is not None or p.q4 is not None:
        return 0.0
    rp = np.asarray(p.Q.rowptr)
    if not np.all(np.diff(rp) == 1) or not np.array_equal(np.asarray(p.Q.colind), np.arange(p.n)):
        return 0.0
    return float(np.min(p.Q.val))


CASES = {
    "lp_small": lambda: w.lp_small(0),
    "lp_small_3": lambda: w.lp_small(3),
    "qp_batch_member": lambda: w.qp_instance(900, 17),
    "nlp_grid": lambda: w.nlp_grid(40, 36),
    "lp_block_small": lambda: w.lp_block(nblocks=4, block_rows=200, block_cols=400, link_cols_per_block=20),
    "qp_param_small": lambda: w.qp_param(20, 30).base,
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_ipm_matches_oracle(name, precision):
    p = CASES[name]()
    print(f"case {name} precision={precision}", flush=True)
    ref = oipm.solve(p, tol=1e-9)
    assert ref["status"] == 0
    s = L.IpmSolver(p, precision=precision).bind()
    res = s.solve()
    sol = s.solution()
    chk = _parity(p, res, sol, ref["f"])
    qmin = _strong_convexity(p)
    if qmin > 0:
        # unique minimiser: ||x - x*||_2^2 <= 2 (f(x) - f*) / qmin, with the
        # optimality gap bounded by the three scaled measures times (1 + |f|)
        gap = (chk["P"] + chk["D"] + chk["C"] + 1e-9) * (1 + abs(ref["f"])) * 3
        assert np.linalg.norm(sol["x"] - ref["x"]) <= np.sqrt(2 * gap / qmin)


def test_ipm_deterministic():
    p = w.nlp_grid(30, 30)
    s = L.IpmSolver(p).bind()
    r1 = s.solve(); x1 = s.solution()["x"]
    r2 = s.solve(); x2 = s.solution()["x"]
    assert r1["iterations"] == r2["iterations"]
    assert np.array_equal(x1, x2)


def test_ipm_warm_start_push():
    p = w.qp_instance(400, 21)
    ref = oipm.solve(p, tol=1e-9)
    s = L.IpmSolver(p).bind()
    cold = s.solve()
    warm = s.solve(start=(ref["x"], ref["lam"]))
    sol = s.solution()
    _parity(p, warm, sol, ref["f"])
    assert warm["iterations"] < cold["iterations"]


def test_ipm_max_iter_status():
    s = L.IpmSolver(w.lp_small(), max_iter=3).bind()
    r = s.solve()
    assert r["status"] == L.PDIPM_MAX_ITER and r["iterations"] == 3
