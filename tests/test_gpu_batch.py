"""GPU parity of the batched solve (many LP/QP instances as one
block-diagonal problem, per-instance steps and termination, HIP graphs)
against the CPU oracle solving each instance alone.

Bars: every instance reaches status OK with |f - f_ref| / max(1, |f_ref|)
<= 1e-6 and the oracle's checker recomputes P, D, C <= 1e-6 from its slice
of the returned vectors (f_ref: oracle at tol 1e-9); strictly convex
instances also have ||x - x_ref||_inf within the strong-convexity bound.
Graph replays and eager launches of the same kernels agree bitwise.
"""
import numpy as np
import pytest

from oracle import checker, ipm as oipm
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [50, 64, 90, 131, 200, 263, 333, 57, 150, 410]


def _problems():
    ps = [w.qp_instance(n, 100 + i) for i, n in enumerate(SIZES)]
    ps += [w.lp_small(0), w.lp_small(3)]
    return ps


_REF = {}


def _refs(ps):
    key = tuple(p.name for p in ps)
    if key not in _REF:
        _REF[key] = [oipm.solve(p, tol=1e-9) for p in ps]
    return _REF[key]


def _check(ps, refs, results, sols, tol=1e-6):
    for i, (p, ref, r, s) in enumerate(zip(ps, refs, results, sols)):
        assert ref["status"] == 0
        assert r["status"] == 0, (i, r)
        f_ref = ref["f"]
        assert abs(r["f"] - f_ref) / max(1.0, abs(f_ref)) <= tol, (i, r["f"], f_ref)
        chk = checker.check(p, s["x"], s["s"], s["lam"], s["zl"], s["zu"])
        assert abs(chk["f"] - f_ref) / max(1.0, abs(f_ref)) <= tol, (i, chk)
        assert chk["P"] <= tol and chk["D"] <= tol and chk["C"] <= tol, (i, chk)
        if p.Q is not None:
            qmin = float(np.min(p.Q.val))
            gap = max(abs(chk["f"] - f_ref), 1e-300) + tol * (1 + abs(f_ref))
            bound = np.sqrt(2 * gap / qmin) + 1e-6
            assert np.max(np.abs(s["x"] - ref["x"])) <= bound, i


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_batch_matches_oracle(precision):
    ps = _problems()
    refs = _refs(ps)
    print(f"batch of {len(ps)} precision={precision}", flush=True)
    b = L.BatchSolver(ps, precision=precision).bind()
    results, info = b.solve()
    print(info, flush=True)
    assert info["solved"] == len(ps)
    # the whole solve is one replay of one captured graph of iterations
    assert info["graph_launches"] == 1
    _check(ps, refs, results, b.solution())


def test_batch_graphs_equal_eager_launches():
    ps = _problems()[:6]
    out = []
    for graphs in (1, 0, 1):
        b = L.BatchSolver(ps, precision=L.PDIPM_FP32, use_graphs=graphs).bind()
        results, info = b.solve()
        # the second replay set of a handle must agree with its first
        results2, _ = b.solve()
        assert results2 == results
        out.append((results, b.solution(), info))
        torch.cuda.synchronize()
    (r0, s0, i0), (r1, s1, i1), (r2, s2, _) = out
    assert i0["graph_launches"] > 0 and i1["graph_launches"] == 0
    assert r0 == r1 == r2
    for a, c in zip(s0, s1):
        for k in a:
            assert np.array_equal(a[k], c[k]), k
    _check(ps, _refs(ps), r0, s0)


def test_batch_autotune_and_blockings():
    ps = _problems()
    refs = _refs(ps)
    b = L.BatchSolver(ps, precision=L.PDIPM_FP32).bind()
    cands = b.blockings()
    chosen, ms = b.autotune(reps=1)
    print("blockings", cands, "ms", ms, "chosen", chosen, flush=True)
    assert 0 <= chosen < len(cands)
    assert np.all(ms > 0) and ms[chosen] == ms.min()
    results, info = b.solve()
    assert info["blocking"] == chosen
    _check(ps, refs, results, b.solution())
    other = (chosen + 3) % len(cands)
    b.set_blocking(other)
    results, info = b.solve()
    assert info["blocking"] == other
    _check(ps, refs, results, b.solution())
    # the tuned choice is remembered for batches of the same size bucket
    b2 = L.BatchSolver(ps, precision=L.PDIPM_FP32).bind()
    results, info = b2.solve()
    assert info["blocking"] == chosen
    _check(ps, refs, results, b2.solution())


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_batch_every_blocking(precision):
    """Every autotuner candidate solves the batch: the map of K entries to
    panel positions is built once, so the panel layout must not depend on
    the blocking (fronts of height 33-64 are small under one candidate and
    blocked under another)."""
    ps = _problems()
    refs = _refs(ps)
    b = L.BatchSolver(ps, precision=precision).bind()
    for idx in range(len(b.blockings())):
        b.set_blocking(idx)
        results, info = b.solve()
        assert info["blocking"] == idx
        _check(ps, refs, results, b.solution())


def test_batch_warm_start():
    ps = _problems()
    refs = _refs(ps)
    b = L.BatchSolver(ps, precision=L.PDIPM_FP64).bind()
    cold, _ = b.solve()
    x0 = np.concatenate([r["x"] for r in refs])
    l0 = np.concatenate([r["lam"] for r in refs])
    warm, info = b.solve(start=(x0, l0))
    _check(ps, refs, warm, b.solution())
    assert np.mean([r["iterations"] for r in warm]) < np.mean([r["iterations"] for r in cold])


def test_batch_matches_single_instance_path():
    ps = _problems()[:4]
    b = L.BatchSolver(ps, precision=L.PDIPM_FP64).bind()
    results, _ = b.solve()
    for p, r in zip(ps, results):
        s = L.IpmSolver(p, precision=L.PDIPM_FP64).bind()
        rs = s.solve()
        assert rs["status"] == 0 and r["status"] == 0
        assert abs(rs["f"] - r["f"]) / max(1.0, abs(rs["f"])) <= 1e-6


def test_batch_fp32_miss_repeats_the_iteration_in_fp64():
    """A tolerance of 1e-10 puts the refinement target (1e-2 tol (1 +
    ||grad f||)) out of reach of a few FP32-preconditioned steps: running
    instances miss it, do not take that iteration's step, and repeat it with
    FP64 factors; the results still meet the parity rule at the tighter
    tolerance's reference."""
    ps = _problems()[:8]
    refs = _refs(ps)
    b = L.BatchSolver(ps, precision=L.PDIPM_FP32, tol=1e-10, ir_max=1).bind()
    results, info = b.solve()
    print(info, flush=True)
    assert info["refine_misses"] >= 1 and info["fp64_from"] >= 0
    assert info["graph_launches"] >= 1
    _check(ps, refs, results, b.solution())
    for r in results:
        assert max(r["P"], r["D"], r["C"]) <= 1e-10


def _same(a, b):
    """Result lists equal entry by entry, NaN equal to NaN."""
    assert len(a) == len(b)
    for ra, rb in zip(a, b):
        assert ra.keys() == rb.keys()
        for k in ra:
            assert ra[k] == rb[k] or (np.isnan(ra[k]) and np.isnan(rb[k])), (k, ra, rb)


@pytest.mark.parametrize("precision", [L.PDIPM_FP64, L.PDIPM_FP32])
def test_batch_graph_holds_whole_iterations(precision):
    """With three iterations per graph the batch replays it several times
    (the FP32 batch, whose tolerance one refinement step of FP32 factors
    cannot reach, switches to FP64 factors inside a replay); the result
    equals the eager launches' bit for bit."""
    ps = _problems()[:5]
    kw = dict(tol=1e-6) if precision == L.PDIPM_FP64 else dict(tol=1e-10, ir_max=1)
    b = L.BatchSolver(ps, precision=precision, graph_iters=3, **kw).bind()
    results, info = b.solve()
    e = L.BatchSolver(ps, precision=precision, use_graphs=0, **kw).bind()
    eager, einfo = e.solve()
    print(info, einfo, flush=True)
    assert info["iterations"] == einfo["iterations"] > 3
    assert info["graph_launches"] == -(-(info["iterations"] + 1) // 3)
    assert info["fp64_from"] == einfo["fp64_from"]
    if precision == L.PDIPM_FP32:
        assert info["fp64_from"] >= 1
    _same(results, eager)
    sb, se = b.solution(), e.solution()
    for a, c in zip(sb, se):
        for k in a:
            assert np.array_equal(a[k], c[k]), k
    _check(ps, _refs(ps), results, sb)


def test_batch_iterates_stay_finite_at_a_tight_tolerance():
    """At tol 1e-12 late FP64 factors of some blocks meet non-positive
    pivots (ended instances are still factored).  Every instance ends OK or
    NUMERICAL; either way the returned iterate and its measures are finite
    (an instance with a non-finite direction ends at its last iterate, and
    an instance that takes no step keeps its point exactly)."""
    ps = _problems()[:5]
    b = L.BatchSolver(ps, precision=L.PDIPM_FP64, tol=1e-12).bind()
    results, info = b.solve()
    e = L.BatchSolver(ps, precision=L.PDIPM_FP64, tol=1e-12, use_graphs=0).bind()
    eager, _ = e.solve()
    print(info, results, flush=True)
    _same(results, eager)
    for p, r, sol in zip(ps, results, b.solution()):
        assert r["status"] in (L.PDIPM_OK, L.PDIPM_ERR_NUMERICAL), r
        assert np.isfinite([r["f"], r["P"], r["D"], r["C"]]).all(), r
        for k, vec in sol.items():
            assert np.isfinite(vec).all(), (p.name, k)
        chk = checker.check(p, sol["x"], sol["s"], sol["lam"], sol["zl"], sol["zu"])
        assert abs(chk["f"] - r["f"]) <= 1e-9 * max(1.0, abs(r["f"])), (chk, r)


def test_batch_automatic_precision():
    """PDIPM_PRECISION_AUTO on a batch of small QPs resolves to FP64 factors
    (FP32 ones would save less than their refinement costs) and solves to the
    parity bar."""
    ps = _problems()
    refs = _refs(ps)
    b = L.BatchSolver(ps, precision=L.PDIPM_PRECISION_AUTO).bind()
    assert b.stats()["precision"] == L.PDIPM_FP64
    results, info = b.solve()
    assert info["fp64_from"] == -1 and info["solved"] == len(ps)
    _check(ps, refs, results, b.solution())
