"""CPU checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host-side symbolic analysis (ordering, elimination
tree, column counts, supernodes) is bit-exact with the oracle's."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from _util import header_functions
from oracle import symbolic as osym
from paper_2508_16094_amd import lib as L
from paper_2508_16094_amd import workloads as w


def test_library_exports_every_declared_symbol():
    so = ctypes.CDLL(L.SO_PATH)
    declared = header_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(so, name), name
    assert set(L.exported_symbols()) <= set(declared)


def _lib_vs_oracle(p):
    s = L.IpmSolver(p)
    got = s.symbolic()
    (jrp, jci), (hrp, hci) = s.patterns()
    adj = osym.kkt_pattern(p.n, jrp, jci, hrp, hci)
    ref = osym.analyze(adj, p.n)
    for k in ["perm", "etree", "colcount", "sn_start", "sn_rowptr", "sn_rows"]:
        assert np.array_equal(got[k], ref[k]), k
    st = s.stats()
    assert st["nnz_L"] == ref["nnz_L"] and st["flops"] == ref["flops"]
    return st


@pytest.mark.parametrize("name", ["lp_small", "qp", "nlp_grid", "lp_block", "qp_param"])
def test_symbolic_bit_exact(name):
    p = {"lp_small": lambda: w.lp_small(3),
         "qp": lambda: w.qp_instance(700, 11),
         "nlp_grid": lambda: w.nlp_grid(45, 37),
         "lp_block": lambda: w.lp_block(nblocks=6, block_rows=300, block_cols=600, link_cols_per_block=30),
         "qp_param": lambda: w.qp_param(25, 30).base}[name]()
    _lib_vs_oracle(p)


@pytest.mark.parametrize("seed", range(4))
def test_symbolic_bit_exact_random_lower_patterns(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(50, 900))
    B = sp.random(n, n, density=min(1.0, 3.0 / n), random_state=seed, format="csr")
    K = sp.tril((B + B.T + sp.eye(n)).tocsr()).tocsr()
    K.sort_indices()
    s = L.KktSolver(n, K.indptr, K.indices)
    got = s.symbolic()
    adj = osym.pattern_from_lower_csr(n, K.indptr, K.indices)
    ref = osym.analyze(adj, n)
    for k in ["perm", "etree", "colcount", "sn_start", "sn_rowptr", "sn_rows"]:
        assert np.array_equal(got[k], ref[k]), k


def test_create_rejects_bad_input():
    p = w.lp_small()
    p.xl = p.xu.copy()
    with pytest.raises(L.PdipmError) as e:
        L.IpmSolver(p)
    assert e.value.code == L.PDIPM_ERR_INVALID_ARG
    p = w.lp_small()
    p.c = p.c.copy(); p.c[3] = np.nan
    with pytest.raises(L.PdipmError):
        L.IpmSolver(p)
    with pytest.raises(L.PdipmError):
        L.KktSolver(3, np.array([0, 1, 2, 3]), np.array([0, 0, 2]))  # row 1 lacks its diagonal


def test_workspace_query_is_host_only():
    s = L.IpmSolver(w.nlp_grid(20, 20), precision=L.PDIPM_FP32)
    assert s.workspace_bytes() > 0
    st = s.stats()
    assert st["n"] == 400 and st["n_super"] >= 1 and st["flops"] > 0


def test_batch_create_offsets_and_blockings():
    ps = [w.qp_instance(n, 40 + i) for i, n in enumerate([50, 90, 140])] + [w.lp_small(2)]
    b = L.BatchSolver(ps, precision=L.PDIPM_FP32)
    assert b.xoff.tolist() == [0, 50, 140, 280, 780]
    assert b.roff.tolist() == [0, 25, 70, 140, 340]
    st = b.stats()
    assert st["n"] == 780
    cands = b.blockings()
    assert len(cands) >= 2 and all(1 <= sh <= 64 and ob >= 1 for sh, ob in cands)
    assert b.workspace_bytes() > 0


def test_batch_symbolic_is_the_union_of_the_instances():
    """The block-diagonal batch has the factor of each instance: its nnz(L)
    and flops are the sums of the oracle's per-instance figures."""
    ps = [w.qp_instance(n, 60 + i) for i, n in enumerate([70, 120, 66])]
    b = L.BatchSolver(ps)
    nnz = flops = 0
    for p in ps:
        s = L.IpmSolver(p)
        (jrp, jci), (hrp, hci) = s.patterns()
        ref = osym.analyze(osym.kkt_pattern(p.n, jrp, jci, hrp, hci), p.n)
        nnz += ref["nnz_L"]
        flops += ref["flops"]
    st = b.stats()
    assert st["nnz_L"] == nnz and st["flops"] == flops


def test_batch_rejects_nonlinear_instances():
    ps = [w.qp_instance(60, 1), w.nlp_grid(6, 5)]
    with pytest.raises(L.PdipmError) as e:
        L.BatchSolver(ps)
    assert e.value.code == L.PDIPM_ERR_INVALID_ARG
    with pytest.raises(L.PdipmError):
        L.BatchSolver([])


@pytest.mark.parametrize("threads", [2, 5, 8])
def test_host_setup_does_not_depend_on_thread_count(threads, monkeypatch):
    """The graph of K, the K map, the graph permutations and the panel map
    run on several host threads over contiguous ranges; forcing the thread
    count (PDIPM_HOST_THREADS, applied at any size) changes none of the
    exported symbolic arrays, the K pattern or the statistics (triples and
    update bytes included)."""
    probs = [w.lp_block(nblocks=6, block_rows=300, block_cols=600, link_cols_per_block=30),
             w.nlp_grid(40, 33), w.qp_instance(500, 3)]

    def run(p, t):
        monkeypatch.setenv("PDIPM_HOST_THREADS", str(t))
        s = L.IpmSolver(p)
        return s.symbolic(), s.k_pattern(), s.stats()

    for p in probs:
        sym1, (rp1, ci1), st1 = run(p, 1)
        symt, (rpt, cit), stt = run(p, threads)
        for k in sym1:
            assert np.array_equal(sym1[k], symt[k]), (p.name, k)
        assert np.array_equal(rp1, rpt) and np.array_equal(ci1, cit), p.name
        assert st1 == stt, p.name
    ps = [w.qp_instance(n, 80 + i) for i, n in enumerate([60, 140, 90])]
    monkeypatch.setenv("PDIPM_HOST_THREADS", "1")
    b1 = L.BatchSolver(ps).stats()
    monkeypatch.setenv("PDIPM_HOST_THREADS", str(threads))
    assert L.BatchSolver(ps).stats() == b1


@pytest.mark.parametrize("name", ["lp_small", "qp", "lp_block", "lp_block_wide_link"])
def test_dual_form_symbolic_bit_exact(name):
    """Dual condensed form: the library orders and analyses M = diag + J D J'
    (m x m) exactly as the oracle does on the structure of J J'."""
    p = {"lp_small": lambda: w.lp_small(1),
         "qp": lambda: w.qp_instance(800, 12),
         "lp_block": lambda: w.lp_block(nblocks=6, block_rows=300, block_cols=600, link_cols_per_block=30),
         "lp_block_wide_link": lambda: w.lp_block(nblocks=8, block_rows=120, block_cols=240,
                                                  link_cols_per_block=40)}[name]()
    s = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_DUAL)
    got = s.symbolic()
    (jrp, jci), _ = s.patterns()
    ref = osym.analyze(osym.dual_pattern(p.m, p.n, jrp, jci), p.m)
    for k in ["perm", "etree", "colcount", "sn_start", "sn_rowptr", "sn_rows"]:
        assert np.array_equal(got[k], ref[k]), k
    st = s.stats()
    assert st["n"] == p.m and st["nnz_L"] == ref["nnz_L"] and st["flops"] == ref["flops"]
    # the pattern of M is the lower structure of J J' with its diagonal
    rp, ci = s.k_pattern()
    Jb = sp.csr_matrix((np.ones(len(jci)), jci, jrp), shape=(p.m, p.n))
    S = sp.tril((Jb @ Jb.T + sp.eye(p.m)).tocsr()).tocsr()
    S.sort_indices()
    assert np.array_equal(rp, S.indptr) and np.array_equal(ci, S.indices)


def test_dual_form_rejects_what_it_cannot_solve():
    with pytest.raises(L.PdipmError) as e:
        L.IpmSolver(w.nlp_grid(10, 10), kkt_form=L.PDIPM_KKT_DUAL)   # Laplacian Hessian
    assert e.value.code == L.PDIPM_ERR_INVALID_ARG
    p = w.qp_instance(60, 2)
    p.m, p.A, p.b = 0, None, np.zeros(0)
    with pytest.raises(L.PdipmError):
        L.IpmSolver(p, kkt_form=L.PDIPM_KKT_DUAL)
    with pytest.raises(L.PdipmError):
        L.BatchSolver([w.qp_instance(60, 2)], kkt_form=L.PDIPM_KKT_DUAL)
    with pytest.raises(L.PdipmError):
        L.IpmSolver(w.lp_small(), kkt_form=4)
    for gi in (0, 1001):
        with pytest.raises(L.PdipmError) as e:
            L.BatchSolver([w.qp_instance(60, 2)], graph_iters=gi)
        assert e.value.code == L.PDIPM_ERR_INVALID_ARG


@pytest.mark.parametrize("name", ["lp_small", "qp", "nlp_grid", "lp_block"])
def test_augmented_form_symbolic_bit_exact(name):
    """Augmented SQD form: the library orders and analyses [H J'; J diag]
    (order n + m, x block first) exactly as the oracle does."""
    p = {"lp_small": lambda: w.lp_small(1),
         "qp": lambda: w.qp_instance(500, 12),
         "nlp_grid": lambda: w.nlp_grid(30, 26),
         "lp_block": lambda: w.lp_block(nblocks=5, block_rows=200, block_cols=400, link_cols_per_block=20)}[name]()
    s = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_AUGMENTED)
    got = s.symbolic()
    (jrp, jci), (hrp, hci) = s.patterns()
    N = p.n + p.m
    ref = osym.analyze(osym.augmented_pattern(p.n, p.m, jrp, jci, hrp, hci), N)
    for k in ["perm", "etree", "colcount", "sn_start", "sn_rowptr", "sn_rows"]:
        assert np.array_equal(got[k], ref[k]), k
    st = s.stats()
    assert st["n"] == N and st["nnz_L"] == ref["nnz_L"] and st["flops"] == ref["flops"]
    rp, ci = s.k_pattern()
    Jb = sp.csr_matrix((np.ones(len(jci)), jci, jrp), shape=(p.m, p.n))
    Hb = sp.csr_matrix((np.ones(len(hci)), hci, hrp), shape=(p.n, p.n))
    S = sp.tril(sp.bmat([[Hb + Hb.T, None], [Jb, sp.eye(p.m)]], format="csr")).tocsr()
    S.sort_indices()
    assert np.array_equal(rp, S.indptr) and np.array_equal(ci, S.indices)


def _geometric_lower(n, k, seed):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    P = rng.random((n, 2))
    _, nb = cKDTree(P).query(P, k + 1)
    r = np.repeat(np.arange(n), k)
    S = sp.csr_matrix((np.ones(n * k), (r, nb[:, 1:].ravel())), shape=(n, n))
    K = sp.tril((((S + S.T) > 0).astype(float) + sp.eye(n)).tocsr()).tocsr()
    K.sort_indices()
    return K


@pytest.mark.parametrize("seed", range(3))
def test_multilevel_ordering_bit_exact_on_irregular_graphs(seed):
    n = [1500, 4000, 9000][seed]
    K = _geometric_lower(n, 6, 60 + seed)
    s = L.KktSolver(n, K.indptr, K.indices, L.default_options(ordering=L.PDIPM_ORDER_MULTILEVEL))
    got = s.symbolic()
    ref = osym.analyze(osym.pattern_from_lower_csr(n, K.indptr, K.indices), n, method="multilevel")
    for k in ["perm", "etree", "colcount", "sn_start", "sn_rowptr", "sn_rows"]:
        assert np.array_equal(got[k], ref[k]), k


@pytest.mark.parametrize("name,form", [("nlp_grid", 0), ("lp_block", 0), ("lp_block", 1), ("qp", 2), ("lp_small", 0)])
def test_multilevel_ordering_bit_exact_on_workloads(name, form):
    p = {"lp_small": lambda: w.lp_small(3),
         "qp": lambda: w.qp_instance(700, 11),
         "nlp_grid": lambda: w.nlp_grid(45, 37),
         "lp_block": lambda: w.lp_block(nblocks=6, block_rows=300, block_cols=600, link_cols_per_block=30)}[name]()
    s = L.IpmSolver(p, kkt_form=form, ordering=L.PDIPM_ORDER_MULTILEVEL)
    got = s.symbolic()
    (jrp, jci), (hrp, hci) = s.patterns()
    if form == 0:
        adj, N = osym.kkt_pattern(p.n, jrp, jci, hrp, hci), p.n
    elif form == 1:
        adj, N = osym.dual_pattern(p.m, p.n, jrp, jci), p.m
    else:
        adj, N = osym.augmented_pattern(p.n, p.m, jrp, jci, hrp, hci), p.n + p.m
    ref = osym.analyze(adj, N, method="multilevel")
    for k in ["perm", "etree", "colcount", "sn_start", "sn_rowptr", "sn_rows"]:
        assert np.array_equal(got[k], ref[k]), k


def test_ordering_option_is_checked():
    with pytest.raises(L.PdipmError):
        L.IpmSolver(w.lp_small(), ordering=2)


@pytest.mark.parametrize("name", ["lp_block", "lp_small", "nlp_grid", "qp"])
def test_automatic_form_keeps_the_cheaper_condensed_system(name):
    """kkt_form AUTO: with a diagonal Hessian both condensed systems are
    analysed and the one with fewer factorisation flops is factored (its
    analysis is the one the explicit form gives); otherwise the primal."""
    p = {"lp_block": lambda: w.lp_block(nblocks=6, block_rows=300, block_cols=600, link_cols_per_block=30),
         "lp_small": lambda: w.lp_small(3),
         "nlp_grid": lambda: w.nlp_grid(30, 26),
         "qp": lambda: w.qp_instance(700, 11)}[name]()
    auto = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_AUTO)
    st = auto.stats()
    prim = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_PRIMAL).stats()
    if name == "nlp_grid":
        assert st["kkt_form"] == L.PDIPM_KKT_PRIMAL and st["flops"] == prim["flops"]
        return
    dual = L.IpmSolver(p, kkt_form=L.PDIPM_KKT_DUAL).stats()
    want = L.PDIPM_KKT_DUAL if dual["flops"] < prim["flops"] else L.PDIPM_KKT_PRIMAL
    assert st["kkt_form"] == want
    ref = L.IpmSolver(p, kkt_form=want)
    assert st["flops"] == min(dual["flops"], prim["flops"])
    a, b = auto.symbolic(), ref.symbolic()
    for k in ["perm", "etree", "colcount", "sn_start", "sn_rowptr", "sn_rows"]:
        assert np.array_equal(a[k], b[k]), k
    if name == "lp_block":
        assert st["kkt_form"] == L.PDIPM_KKT_DUAL


def test_automatic_precision_follows_the_cost_model():
    """PDIPM_PRECISION_AUTO resolves at create, from counts only: FP64
    factors where FP32 ones would save less factorisation time than two
    extra triangular solves cost (a 500-column LP, a 1,440-point grid NLP),
    FP32 factors where the factorisation dominates (a 20-block
    block-angular LP, 1.3e12 flops); explicit precisions report themselves."""
    cases = [(w.lp_small(), L.PDIPM_FP64), (w.nlp_grid(40, 36), L.PDIPM_FP64),
             (w.lp_block(nblocks=20), L.PDIPM_FP32)]
    for p, want in cases:
        got = [L.IpmSolver(p, precision=L.PDIPM_PRECISION_AUTO).stats()["precision"] for _ in range(2)]
        assert got == [want, want], (p.name, got)
    p = w.lp_small()
    for prec in (L.PDIPM_FP64, L.PDIPM_FP32):
        assert L.IpmSolver(p, precision=prec).stats()["precision"] == prec
    # the automatic choice keeps space for both factor precisions
    s = L.IpmSolver(p, precision=L.PDIPM_PRECISION_AUTO)
    assert s.workspace_bytes() >= L.IpmSolver(p, precision=L.PDIPM_FP32).workspace_bytes()
    # a batch of small QPs resolves to FP64 factors as well; the standalone
    # KKT handle takes an explicit precision
    b = L.BatchSolver([w.qp_instance(60 + 10 * i, 2 + i) for i in range(8)], precision=L.PDIPM_PRECISION_AUTO)
    assert b.stats()["precision"] == L.PDIPM_FP64
    K = sp.random(30, 30, density=0.2, random_state=1) + 30 * sp.eye(30)
    lo = sp.tril(K + K.T, format="csr")
    with pytest.raises(L.PdipmError):
        L.KktSolver(30, lo.indptr, lo.indices, L.default_options(precision=L.PDIPM_PRECISION_AUTO))
    with pytest.raises(L.PdipmError):
        L.IpmSolver(p, precision=3)
