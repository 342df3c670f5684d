"""GPU tests of the FP32 form's reproducibility and fallbacks, and of the
pushed warm start against the oracle (through the C ABI).

* FP32 form, bitwise repeatable: the switch to FP64 factors is decided from
  modelled costs (counts), never from clocks, so two solves of the same
  instance give identical iterates.
* kkt_solve with an FP32 factor that refinement cannot bring to the
  backward-error target refactors in FP64 (info fallback = 1) and then meets
  the FP64 bar.
* The pushed start (bound-push rule) equals the oracle's push_start to
  rounding (1e-14 relative): ipm_solve with max_iter = 0 returns it.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ipm as oipm, model
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda:0")


CASES = {
    "nlp_grid": lambda: w.nlp_grid(40, 36),
    "lp_block_small": lambda: w.lp_block(nblocks=4, block_rows=200, block_cols=400, link_cols_per_block=20),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_form_bitwise_repeatable(name):
    p = CASES[name]()
    print(f"case {name} fp32 twice", flush=True)
    s = L.IpmSolver(p, precision=L.PDIPM_FP32).bind()
    r1 = s.solve(); a = s.solution()
    r2 = s.solve(); b = s.solution()
    assert r1["status"] == 0 and r2["status"] == 0
    for k in ("iterations", "fp64_refactors", "ir_steps", "f", "P", "D", "C"):
        assert r1[k] == r2[k], (k, r1[k], r2[k])
    for k in ("x", "s", "lam", "zl", "zu"):
        assert np.array_equal(a[k], b[k]), k


def _ill_conditioned(n, cond, seed):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    K = (Qm * np.logspace(0, -np.log10(cond), n)) @ Qm.T
    return 0.5 * (K + K.T)


def _solver_for_dense(K, **kw):
    n = K.shape[0]
    Kl = sp.tril(sp.csr_matrix(K)).tocsr()
    Kl.sort_indices()
    s = L.KktSolver(n, Kl.indptr, Kl.indices, L.default_options(**kw)).bind()
    s.set_values(dev(Kl.data))
    return s


def test_kkt_solve_fp32_falls_back_to_fp64():
    K = _ill_conditioned(160, 1e11, 3)
    print("case kkt_solve fallback n=160 cond=1e11", flush=True)
    s = _solver_for_dense(K, precision=L.PDIPM_FP32, ir_max=1)
    info = s.factor(L.PDIPM_FP32)
    assert info["status"] == 0
    b = np.random.default_rng(4).standard_normal(K.shape[0])
    x, si = s.solve_kkt(dev(b))
    x = x.cpu().numpy()
    assert si["fallback"] == 1
    kn = np.max(np.abs(K).sum(1))
    assert np.max(np.abs(K @ x - b)) / (kn * np.max(np.abs(x)) + np.max(np.abs(b))) <= 1e-14


def test_kkt_solve_fp32_no_fallback_when_refinement_converges():
    K = _ill_conditioned(160, 1e3, 5)
    print("case kkt_solve no fallback n=160 cond=1e3", flush=True)
    s = _solver_for_dense(K, precision=L.PDIPM_FP32)
    assert s.factor(L.PDIPM_FP32)["status"] == 0
    b = np.random.default_rng(6).standard_normal(K.shape[0])
    x, si = s.solve_kkt(dev(b))
    assert si["fallback"] == 0 and si["ir_steps"] >= 1


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_pushed_start_matches_oracle(precision):
    p = w.qp_instance(300, 23)
    rng = np.random.default_rng(7)
    # a predicted point partly outside the bounds, multipliers partly tiny
    xh = rng.uniform(-2.0, 12.0, p.n)
    lh = np.where(rng.random(p.m) < 0.5, 1e-4, rng.uniform(0.1, 3.0, p.m))
    s = L.IpmSolver(p, precision=precision, max_iter=0).bind()
    r = s.solve(start=(xh, lh))
    assert r["status"] == L.PDIPM_MAX_ITER and r["iterations"] == 0
    got = s.solution()
    xl, xu = model.bounds(p)
    ref = oipm.push_start(p, xh, lh, xl, xu)
    for k, rv in zip(("x", "s", "lam", "zl", "zu"), ref):
        g = got[k]
        assert np.max(np.abs(g - rv)) <= 1e-14 * max(1.0, np.max(np.abs(rv))), k


def test_set_precision_checks_the_workspace():
    p = w.lp_small()
    s = L.IpmSolver(p, precision=L.PDIPM_FP64, fp64_fallback=0)
    with pytest.raises(L.PdipmError):
        s.set_precision(L.PDIPM_FP32)
    s32 = L.IpmSolver(p, precision=L.PDIPM_FP32).bind()
    r32 = s32.solve()
    s32.set_precision(L.PDIPM_FP64)
    r64 = s32.solve()
    assert r32["status"] == 0 and r64["status"] == 0
    assert r64["fp64_refactors"] == 0
    assert abs(r32["f"] - r64["f"]) <= 1e-6 * max(1.0, abs(r64["f"]))


def test_automatic_precision_solves_to_parity():
    """PDIPM_PRECISION_AUTO on a latency-bound LP resolves to FP64 factors
    and solves it like the FP64 form (same iterates bit for bit), within the
    parity bar of the oracle."""
    p = w.lp_small()
    ref = oipm.solve(p, tol=1e-9)
    sa = L.IpmSolver(p, precision=L.PDIPM_PRECISION_AUTO).bind()
    assert sa.stats()["precision"] == L.PDIPM_FP64
    ra = sa.solve()
    r64 = L.IpmSolver(p, precision=L.PDIPM_FP64).bind().solve()
    print(ra, r64, flush=True)
    assert ra["status"] == 0 and ra["fp64_refactors"] == 0
    for k in ("iterations", "f", "P", "D", "C"):
        assert ra[k] == r64[k], k
    assert abs(ra["f"] - ref["f"]) <= 1e-6 * max(1.0, abs(ref["f"]))
