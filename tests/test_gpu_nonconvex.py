"""GPU parity on nonconvex NLPs (the primal condensed form with inertia
correction, Section 3: Regularization, nonconvex case) against the oracle.

The grid NLP with mixed-sign stencil weights has an indefinite Lagrangian
Hessian, so K = H + Sigma_x + delta_p I + J' Sigma_s J meets non-positive
pivots; both sides then add delta_w I by the same schedule (1e-4 first,
times 100, then times 8; later max(1e-20, last/3)).  Bars: the parity rule
(|f - f_ref| / max(1, |f_ref|) <= 1e-6 and the oracle's checker P, D, C <=
1e-6 on the returned vectors), and the same number of corrected iterations
as the oracle in FP64 (FP32: the FP32 factor fails first, then FP64 decides).
"""
import numpy as np
import pytest

from oracle import checker, ipm as oipm
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (nx, ny, instance, fraction of negative weights, |weight|, scale of c):
# each has active constraints at its solution and needs delta_w > 0 at
# least once
CASES = {
    "grid20": (20, 20, 0, 0.5, 0.2, 5.0),
    "grid30": (30, 30, 1, 0.5, 0.3, 4.0),
    "grid40x36": (40, 36, 0, 0.4, 0.2, 4.0),
}
_REF = {}


def _ref(name):
    if name not in _REF:
        p = w.nlp_grid_nonconvex(*CASES[name])
        r = oipm.solve(p, tol=1e-9)
        assert r["status"] == 0
        assert np.sum(r["lam"] > 1e-6) > 0      # some constraints are active
        _REF[name] = (p, r, sum(1 for h in r["history"] if h["delta_w"] > 0))
    return _REF[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_nonconvex_inertia_correction_matches_oracle(name, precision):
    p, ref, ref_corr = _ref(name)
    assert ref_corr > 0
    print(f"case nonconvex {name} precision={precision} oracle corrections={ref_corr}", flush=True)
    s = L.IpmSolver(p, precision=precision).bind()
    res = s.solve()
    sol = s.solution()
    assert res["status"] == 0, res
    assert res["inertia_corrections"] > 0
    if precision == L.PDIPM_FP64:
        assert res["inertia_corrections"] == ref_corr
    chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
    assert abs(res["f"] - ref["f"]) / max(1.0, abs(ref["f"])) <= 1e-6
    assert abs(chk["f"] - ref["f"]) / max(1.0, abs(ref["f"])) <= 1e-6
    assert chk["P"] <= 1e-6 and chk["D"] <= 1e-6 and chk["C"] <= 1e-6, chk


def test_convex_grid_needs_no_correction():
    p = w.nlp_grid(30, 30)
    s = L.IpmSolver(p).bind()
    res = s.solve()
    assert res["status"] == 0 and res["inertia_corrections"] == 0
