"""Pins of the oracle's symbolic analysis (test infrastructure).

P6: dense boolean elimination (brute force) gives the fill, elimination tree,
column counts and fundamental supernodes; an explicit-matrix minimum degree
elimination cross-checks the set-based one; hand-derived orders for a path,
a 3x3 grid, a star, two cliques joined by a separator, and a disconnected
graph pin the ordering rule (its steps are listed in oracle/symbolic.py).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import symbolic


def _adj_from_edges(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b); adj[b].add(a)
    return [sorted(s) for s in adj]


def _brute_symbolic(adj, perm):
    n = len(perm)
    pinv = np.empty(n, int); pinv[perm] = np.arange(n)
    M = np.zeros((n, n), bool)
    for v in range(n):
        for u in adj[v]:
            M[pinv[v], pinv[u]] = True
    for k in range(n):
        R = np.nonzero(M[k + 1:, k])[0] + k + 1
        M[np.ix_(R, R)] = True
        M[R, k] = True
    structs = [np.nonzero(M[j + 1:, j])[0] + j + 1 for j in range(n)]
    parent = np.array([s[0] if len(s) else -1 for s in structs])
    cc = np.array([len(s) + 1 for s in structs])
    return structs, parent, cc


def _random_graph(n, seed, p=0.08):
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return _adj_from_edges(n, edges)


@pytest.mark.parametrize("n,seed", [(30, 1), (90, 2), (200, 3), (300, 4)])
def test_p6_brute_force_structure(n, seed):
    adj = _random_graph(n, seed, p=3.0 / n)
    r = symbolic.analyze(adj, n, menu=(1, 0, 0, 1))   # no amalgamation
    structs, parent, cc = _brute_symbolic(adj, r["perm"])
    assert sorted(r["perm"].tolist()) == list(range(n))
    assert np.array_equal(parent, r["etree"])
    assert np.array_equal(cc, r["colcount"])
    for a, b in zip(r["structs"], structs):
        assert np.array_equal(a, b)
    # fundamental supernodes straight from the definition on the brute data
    nchild = np.bincount(parent[parent >= 0], minlength=n)
    starts = [0] + [j + 1 for j in range(n - 1)
                    if not (parent[j] == j + 1 and cc[j] == cc[j + 1] + 1 and nchild[j + 1] == 1)]
    assert r["sn_start"].tolist() == starts + [n]
    # supernode rows = columns + structure of the last column
    for k in range(len(starts)):
        a, b = r["sn_start"][k], r["sn_start"][k + 1]
        rows = r["sn_rows"][r["sn_rowptr"][k]:r["sn_rowptr"][k + 1]]
        assert rows.tolist() == list(range(a, b)) + structs[b - 1].tolist()
    # postordered: every subtree is a contiguous range ending at its root
    size = np.ones(n, int)
    for j in range(n):
        if parent[j] >= 0:
            size[parent[j]] += size[j]
    for j in range(n):
        if parent[j] >= 0:
            assert j >= parent[j] - size[parent[j]] + 1


def _md_dense(adj, verts):
    verts = sorted(verts)
    idx = {v: k for k, v in enumerate(verts)}
    M = np.zeros((len(verts), len(verts)), bool)
    for v in verts:
        for u in adj[v]:
            if u in idx:
                M[idx[v], idx[u]] = True
    alive = np.ones(len(verts), bool)
    out = []
    for _ in verts:
        deg = np.where(alive, (M & alive[None, :]).sum(1), 10 ** 9)
        k = int(np.argmin(deg))            # argmin takes the smallest index on ties
        out.append(verts[k])
        nb = np.nonzero(M[k] & alive)[0]
        M[np.ix_(nb, nb)] = True
        M[nb, nb] = False
        alive[k] = False
    return out


@pytest.mark.parametrize("seed", range(5))
def test_p6_minimum_degree_cross_check(seed):
    n = 40 + seed * 5
    adj = _random_graph(n, 50 + seed, p=0.1)
    inset = [True] * n
    got = symbolic.exact_minimum_degree(adj, list(range(n)), inset)
    assert got == _md_dense(adj, range(n))


def test_p6_path_hand_derived():
    n = 200
    adj = _adj_from_edges(n, [(i, i + 1) for i in range(n - 1)])
    nd = symbolic.nested_dissection(adj, n)
    expect = (list(range(0, 49)) + list(range(50, 99)) + [49]
              + list(range(100, 149)) + list(range(150, 200)) + [149, 99])
    assert nd == expect
    r = symbolic.analyze(adj, n)
    assert r["perm"].tolist() == expect


def test_p6_grid3x3_hand_derived():
    edges = []
    for i in range(3):
        for j in range(3):
            if i < 2: edges.append((3 * i + j, 3 * i + j + 3))
            if j < 2: edges.append((3 * i + j, 3 * i + j + 1))
    adj = _adj_from_edges(9, edges)
    assert symbolic.nested_dissection(adj, 9) == [0, 2, 6, 8, 1, 3, 4, 5, 7]
    r = symbolic.analyze(adj, 9)
    assert r["perm"].tolist() == [8, 6, 0, 2, 1, 3, 4, 5, 7]


def test_p6_star_hand_derived():
    n = 100
    adj = _adj_from_edges(n, [(0, i) for i in range(1, n)])
    r = symbolic.analyze(adj, n)
    assert r["perm"].tolist() == list(range(1, n)) + [0]
    assert r["sn_start"].tolist() == list(range(0, 93)) + [100]


def test_p6_two_cliques_and_separator_hand_derived():
    A = list(range(0, 40)); B = list(range(42, 82)); S = [40, 41]
    edges = [(a, b) for X in (A, B) for a in X for b in X if a < b]
    edges += [(s, v) for s in S for v in A + B] + [(40, 41)]
    adj = _adj_from_edges(82, edges)
    assert symbolic.nested_dissection(adj, 82) == [0] + B + list(range(1, 42))
    r = symbolic.analyze(adj, 82)
    assert r["perm"].tolist() == B + list(range(0, 42))


def test_p6_disconnected_components_in_order():
    # path 3-0-6 and a star centred at 4 with leaves 1, 2, 5, 7, 8; both are
    # leaf components, ordered by minimum degree with smallest-index ties
    adj = _adj_from_edges(9, [(3, 0), (0, 6), (4, 1), (4, 2), (4, 5), (4, 7), (4, 8)])
    nd = symbolic.nested_dissection(adj, 9)
    assert nd == [3, 0, 6, 1, 2, 5, 7, 4, 8]


def _two_supernode_columns(k9):
    """Lower structures of a hand-built factor pattern on 20 columns: a chain
    0..9 whose last column reaches rows 10..10+k9-1, under a dense 10 x 10
    root block 10..19.  Column j < 10 has rows j+1..9 and 10..10+k9-1."""
    cols = []
    for j in range(10):
        cols.append(np.array(list(range(j + 1, 10)) + list(range(10, 10 + k9)), dtype=np.int64))
    for j in range(10, 20):
        cols.append(np.arange(j + 1, 20, dtype=np.int64))
    return cols


def test_p6_amalgamation_merges_by_zero_fraction_at_width_20():
    """Hand-derived: child c = columns 0..9 with c_j = 19 - j (its last
    column reaches rows 10..18), parent s = dense root 10..19 with
    c_j = 20 - j.  c_9 = 10 != c_10 + 1 = 11, so the fundamental supernodes
    are [0, 10) and [10, 20).  Merging gives w = 20, h = 20, a trapezoid of
    w h - w (w - 1) / 2 = 400 - 190 = 210 entries, of which
    sum(19..10) + sum(10..1) = 145 + 55 = 200 are true: 10 zeros, and
    10 * 10 <= 1 * 210, so the default rule (zero fraction 1/10, w = 20 > 8)
    merges them into one supernode."""
    structs, parent = symbolic.symbolic_factor(_two_supernode_columns(9))
    cc = np.array([len(s) + 1 for s in structs])
    assert cc.tolist() == [19 - j for j in range(10)] + [20 - j for j in range(10, 20)]
    assert parent.tolist() == list(range(1, 20)) + [-1]
    fund = symbolic.fundamental_supernodes(parent, cc)
    assert fund == [0, 10]
    assert symbolic.amalgamate(fund, parent, cc) == [0, 20]
    # a width cap of 16 forbids the merge (menu entries: max_w, small_w, num, den)
    assert symbolic.amalgamate(fund, parent, cc, (16, 8, 1, 10)) == [0, 10, 20]
    # a stricter zero fraction (1/25: 10 * 25 = 250 > 210) rejects it
    assert symbolic.amalgamate(fund, parent, cc, (1 << 30, 8, 1, 25)) == [0, 10, 20]


def test_p6_amalgamation_rejects_too_many_zeros():
    """Hand-derived: the child's last column reaches row 10 only, so
    c_j = 11 - j for j < 10 (true entries 11 + ... + 2 = 65) and the merged
    trapezoid of 210 entries holds 210 - 65 - 55 = 90 zeros: 90 * 10 > 210,
    no merge; with w <= small_w (a menu with small_w = 20) it always merges."""
    structs, parent = symbolic.symbolic_factor(_two_supernode_columns(1))
    cc = np.array([len(s) + 1 for s in structs])
    assert cc.tolist() == [11 - j for j in range(10)] + [20 - j for j in range(10, 20)]
    fund = symbolic.fundamental_supernodes(parent, cc)
    assert fund == [0, 10]
    assert symbolic.amalgamate(fund, parent, cc) == [0, 10, 20]
    assert symbolic.amalgamate(fund, parent, cc, (1 << 30, 20, 1, 10)) == [0, 20]


# ------------------------------------------------- multilevel bisection
def _geometric_adj(n, k, seed):
    """k-nearest-neighbour graph of n random points in the unit square."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    P = rng.random((n, 2))
    _, nb = cKDTree(P).query(P, k + 1)
    r = np.repeat(np.arange(n), k)
    S = sp.csr_matrix((np.ones(n * k), (r, nb[:, 1:].ravel())), shape=(n, n))
    S = ((S + S.T) > 0).astype(float).tocsr()
    return symbolic.adjacency_from_sym(S, n)


def _local(adj, n):
    return symbolic._ml_local_graph(adj, list(range(n)), [True] * n)


@pytest.mark.parametrize("seed", range(3))
def test_ml_coarsening_invariants(seed):
    """Heavy-edge matching: each coarse vertex has one or two adjacent
    members, the matching is maximal (no edge joins two unmatched vertices),
    vertex weight is preserved, and the coarse edge weights are exactly the
    fine edges between different coarse vertices."""
    adj = _geometric_adj(300, 5, seed)
    nbrs, ew, vw = _local(adj, 300)
    for _ in range(3):
        cmap, cn, ce, cw = symbolic._ml_coarsen(nbrs, ew, vw)
        members = {}
        for v, c in enumerate(cmap):
            members.setdefault(c, []).append(v)
        assert sorted(members) == list(range(len(cw)))
        for c, ms in members.items():
            assert len(ms) in (1, 2)
            if len(ms) == 2:
                assert ms[1] in nbrs[ms[0]]
            assert cw[c] == sum(vw[v] for v in ms)
        singles = {ms[0] for ms in members.values() if len(ms) == 1}
        for v in singles:
            assert not any(u in singles for u in nbrs[v])
        want = {}
        for v in range(len(vw)):
            for u, wt in zip(nbrs[v], ew[v]):
                if cmap[u] != cmap[v]:
                    want[(cmap[v], cmap[u])] = want.get((cmap[v], cmap[u]), 0) + wt
        got = {(c, u): wt for c in range(len(cw)) for u, wt in zip(cn[c], ce[c])}
        assert got == want
        nbrs, ew, vw = cn, ce, cw


@pytest.mark.parametrize("seed", range(3))
def test_ml_refinement_is_locally_optimal(seed):
    """After refinement no single move has positive gain within the balance
    bound, the parts hold every vertex, and the cut never grew."""
    adj = _geometric_adj(200, 4, 10 + seed)
    nbrs, ew, vw = _local(adj, 200)
    part0 = symbolic._ml_initial(nbrs, vw)

    def cut(part):
        return sum(wt for v in range(200) for u, wt in zip(nbrs[v], ew[v]) if part[u] != part[v]) // 2
    c0 = cut(part0)
    part = symbolic._ml_refine(nbrs, ew, vw, list(part0))
    assert cut(part) <= c0
    total = sum(vw)
    maxw = symbolic.ML_BAL_NUM * total // symbolic.ML_BAL_DEN
    pw = [sum(vw[v] for v in range(200) if part[v] == p) for p in (0, 1)]
    for v in range(200):
        ext = sum(wt for u, wt in zip(nbrs[v], ew[v]) if part[u] != part[v])
        inn = sum(wt for u, wt in zip(nbrs[v], ew[v]) if part[u] == part[v])
        assert not (ext - inn > 0 and pw[1 - part[v]] + vw[v] <= maxw), v


@pytest.mark.parametrize("seed", range(4))
def test_ml_separator_separates(seed):
    """lower, upper and the separator partition the component, no edge joins
    lower to upper, and every separator vertex touches the other part."""
    n = 400 + 100 * seed
    adj = _geometric_adj(n, 5, 20 + seed)
    inset = [True] * n
    comps = symbolic._components(adj, list(range(n)), inset)
    comp = max(comps, key=len)
    inset = [False] * n
    for v in comp:
        inset[v] = True
    lower, upper, sep = symbolic.multilevel_separator(adj, comp, inset)
    assert sorted(lower + upper + sep) == comp
    lo = set(lower)
    for v in upper:
        assert not any(u in lo for u in adj[v])
    up = set(upper)
    for s in sep:
        assert any(inset[u] and (u in lo or u in up) for u in adj[s])


def test_ml_barbell_is_cut_at_one_vertex():
    """Two 30-cliques joined by a path of 5 vertices: the multilevel
    separator is a single path vertex (the optimum), and the ordering
    eliminates the two cliques before it."""
    A, P, B = list(range(30)), list(range(30, 35)), list(range(35, 65))
    edges = [(a, b) for X in (A, B) for a in X for b in X if a < b]
    edges += [(29, 30), (30, 31), (31, 32), (32, 33), (33, 34), (34, 35)]
    adj = _adj_from_edges(65, edges)
    lower, upper, sep = symbolic.multilevel_separator(adj, list(range(65)), [True] * 65)
    assert len(sep) == 1 and sep[0] in P
    nd = symbolic.nested_dissection(adj, 65, leaf=16, method="multilevel")
    assert nd[-1] == sep[0]


@pytest.mark.parametrize("seed", range(2))
def test_ml_ordering_fills_less_than_level_ordering(seed):
    """The reason for the multilevel rule: on irregular (geometric) graphs its
    separators are far smaller than BFS level sets, and so is the fill."""
    n = 3000
    adj = _geometric_adj(n, 6, 40 + seed)
    a = symbolic.analyze(adj, n)
    b = symbolic.analyze(adj, n, method="multilevel")
    assert b["nnz_L"] < 0.8 * a["nnz_L"] and b["flops"] < 0.5 * a["flops"]
