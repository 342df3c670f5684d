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
