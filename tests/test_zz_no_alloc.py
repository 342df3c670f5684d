"""ipm_solve_static (the allocation-free entry point) against ipm_solve
with a caller workspace, through the C ABI: two calls in a row on the
library's static device array, the second with a smaller instance, each
equal to the workspace path (same kernels, same arithmetic: iterates equal
to 1e-12 relative, f within the 1e-6 parity rule and far below it)."""
import numpy as np
import pytest

from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _with_workspace(p, precision):
    s = L.IpmSolver(p, precision=precision).bind()
    return s.solve(), s.solution()


def _close(a, b, what):
    scale = max(1.0, float(np.max(np.abs(b)))) if b.size else 1.0
    assert np.max(np.abs(a - b), initial=0.0) <= 1e-12 * scale, what


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_static_solve_matches_workspace_solve(precision):
    big, small = w.qp_instance(900, 17), w.lp_small(0)
    ref_big = _with_workspace(big, precision)
    ref_small = _with_workspace(small, precision)
    print(f"case static precision={precision} big n={big.n} small n={small.n}", flush=True)
    hb = L.IpmSolver(big, precision=precision)
    hs = L.IpmSolver(small, precision=precision)
    assert hs.workspace_bytes() < hb.workspace_bytes() <= 64 << 20
    for h, p, (rr, rs) in ((hb, big, ref_big), (hs, small, ref_small)):
        r = h.solve_static()
        sol = h.solution()
        assert r["status"] == rr["status"] == 0
        assert r["iterations"] == rr["iterations"]
        assert abs(r["f"] - rr["f"]) <= 1e-12 * max(1.0, abs(rr["f"]))
        for k in ("x", "s", "lam", "zl", "zu"):
            _close(sol[k], rs[k], k)
    # the first handle again after the smaller one used the array
    r = hb.solve_static()
    assert r["iterations"] == ref_big[0]["iterations"]
    _close(hb.solution()["x"], ref_big[1]["x"], "x again")


def test_static_solve_rejects_a_workspace_above_its_limit():
    p = w.lp_block(nblocks=4, block_rows=1000, block_cols=2000, link_cols_per_block=50)
    s = L.IpmSolver(p)
    assert s.workspace_bytes() > 64 << 20
    with pytest.raises(L.PdipmError) as e:
        s.solve_static()
    assert e.value.code == L.PDIPM_ERR_OUT_OF_MEMORY
