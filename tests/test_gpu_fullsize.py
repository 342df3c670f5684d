"""Full-size GPU checks in the launch configuration of bench.py, where the
oracle cannot solve the whole problem: properties that hold at any size.

  block-angular LP (n = 2,000,000, m = 1,020,000), FP32 form: status OK;
      the oracle's checker recomputes P, D, C <= 1e-6 from the returned
      vectors; the LP dual objective equals f within 1e-5 (1 + |f|); an FP64
      factorisation at the final point solves K d = r with backward error
      <= 1e-11, K formed independently by the oracle (scipy, CPU).
  grid NLP (700 x 700, n = 490,000): FP32 form and FP64 form both reach
      status OK with checker P, D, C <= 1e-6 and the same f within 1e-6.
  4,096 batched QPs: every instance OK; checker on 64 instances spread over
      the sizes; oracle f (tol 1e-9) for 4 of them within 1e-6.
"""
import time

import numpy as np
import pytest

from oracle import checker, ipm as oipm, kkt as okkt, model
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(1200)]

torch = pytest.importorskip("torch")


def _log(msg):
    print(msg, flush=True)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float64), device="cuda:0")


def test_block_lp_full_size():
    t = time.time()
    p = w.lp_block()
    _log(f"lp_block generated n={p.n} m={p.m} in {time.time() - t:.1f}s")
    s = L.IpmSolver(p, precision=L.PDIPM_FP32, fp64_fallback=1).bind()
    _log(f"analysed and bound at {time.time() - t:.1f}s")
    r = s.solve()
    _log(f"solved: {r['status']} it {r['iterations']} f {r['f']:.10e} at {time.time() - t:.1f}s")
    assert r["status"] == 0
    sol = s.solution()
    chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
    _log(f"checker {chk['P']:.2e} {chk['D']:.2e} {chk['C']:.2e}")
    assert chk["P"] <= 1e-6 and chk["D"] <= 1e-6 and chk["C"] <= 1e-6
    dual = checker.lp_qp_dual_objective(p, sol["x"], sol["lam"], sol["zl"], sol["zu"])
    assert abs(dual - chk["f"]) <= 1e-5 * (1 + abs(chk["f"])), (dual, chk["f"])
    # FP64 factor at the final point against the oracle's condensed matrix
    x, lam = sol["x"], sol["lam"]
    xl, xu = model.bounds(p)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    sig_s, sig_x = okkt.sigmas(x, sol["s"], lam, sol["zl"], sol["zu"], xl, xu, il, iu, 1e-8)
    s.assemble(_dev(x), _dev(lam), _dev(sig_s), _dev(sig_x), L.PDIPM_FP64)
    info = s.factor(L.PDIPM_FP64)
    assert info["status"] == 0
    rng = np.random.default_rng(7)
    b = rng.standard_normal(p.n)
    d, _ = s.solve_kkt(_dev(b))
    d = d.cpu().numpy()
    K = okkt.condensed_matrix(model.hessian(p, x, lam), model.jacobian(p, x), sig_s, sig_x, 1e-8)
    res = np.max(np.abs(K @ d - b))
    knorm = np.max(np.abs(K).sum(axis=1))
    omega = res / (knorm * np.max(np.abs(d)) + np.max(np.abs(b)))
    _log(f"FP64 solve backward error {omega:.2e} at {time.time() - t:.1f}s")
    assert omega <= 1e-11


def test_nlp_grid_full_size_both_forms():
    p = w.nlp_grid()
    fs = []
    for prec in (L.PDIPM_FP32, L.PDIPM_FP64):
        t = time.time()
        s = L.IpmSolver(p, precision=prec, fp64_fallback=1).bind()
        r = s.solve()
        sol = s.solution()
        chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
        _log(f"nlp_grid prec={prec} status {r['status']} it {r['iterations']} f {r['f']:.10e} "
             f"P {chk['P']:.1e} D {chk['D']:.1e} C {chk['C']:.1e} in {time.time() - t:.1f}s")
        assert r["status"] == 0
        assert chk["P"] <= 1e-6 and chk["D"] <= 1e-6 and chk["C"] <= 1e-6
        fs.append(chk["f"])
        del s
        torch.cuda.empty_cache()
    assert abs(fs[0] - fs[1]) <= 1e-6 * max(1.0, abs(fs[1]))


def test_batch_4096_full_size():
    t = time.time()
    ps = w.qp_batch(4096)
    b = L.BatchSolver(ps, precision=L.PDIPM_FP32).bind()
    _log(f"batch created in {time.time() - t:.1f}s")
    res, info = b.solve()
    _log(f"batch solved: {info}")
    assert info["solved"] == 4096 and all(r["status"] == 0 for r in res)
    sol = b.solution()
    order = np.argsort([q.n for q in ps])
    picks = order[np.linspace(0, len(ps) - 1, 64).astype(int)]
    for i in picks:
        c = checker.check(ps[i], sol[i]["x"], sol[i]["s"], sol[i]["lam"], sol[i]["zl"], sol[i]["zu"])
        assert c["P"] <= 1e-6 and c["D"] <= 1e-6 and c["C"] <= 1e-6, (i, c)
    for i in picks[[0, 10, 20, 30]]:
        ref = oipm.solve(ps[i], tol=1e-9)
        assert abs(res[i]["f"] - ref["f"]) / max(1.0, abs(ref["f"])) <= 1e-6, (i, res[i]["f"], ref["f"])
    _log(f"batch checks done in {time.time() - t:.1f}s")
