"""Symbolic analysis of the condensed KKT matrix: fill-reducing ordering,
elimination tree, column counts and supernodes.

The paper factors P'KP = LDL' (Section 2, LDL^T factorization) with a
fill-reducing permutation computed once on the CPU and reused (Section 2,
GPU direct solvers: minimum degree or nested dissection).  It fixes no
particular ordering, so this module follows one exact rule (the library
implements the same rule independently and must agree bit for bit):

ORD  Graph G = structure of K without its diagonal.
     order(S): connected components of G[S] in increasing order of their
       smallest vertex, each ordered by order_component.
     order_component(C):
       |C| <= leaf: exact minimum degree on G[C] (minimum current degree,
         ties to the smallest vertex; neighbours of the eliminated vertex
         become a clique).
       otherwise: root r = pseudo-peripheral vertex (start at the vertex of
         minimum degree in G[C], move to the minimum-degree vertex of the last
         BFS level while the BFS height grows; ties to the smallest vertex);
         BFS levels L_0..L_h from r; if h < 2 C is ordered by increasing
         degree in G[C] (ties to the smallest vertex);
         else separator level l in [1, h-1] minimising
         |L_l| / min(|L_<l|, |L_>l|), then |2l - h|, then l;
         if the largest connected component left after removing L_l keeps
         more than 7/8 of C the separator is rejected and C is ordered by
         increasing degree in G[C] (such graphs fill in densely under any
         order; high-degree hub vertices go last);
         result order(L_<l) ++ order(L_>l) ++ sorted(L_l).
     The ND order is then composed with a postorder of the elimination tree
     (children in increasing index, roots in increasing index).
SYM  struct(j) = row indices below the diagonal of column j of L;
     colcount c_j = |struct(j)| + 1; parent(j) = min struct(j) (or -1).
     Fundamental supernodes: j+1 joins j when parent(j) = j+1,
     c_j = c_{j+1} + 1 and j is the only child of j+1.
     Relaxed amalgamation (parameters max_w, small_w, zero fraction num/den):
     scanning supernodes s left to right, while the supernode c ending just
     before s is a child of s: with w = w_c + w_s, h = w_c + h_s,
     total = w*h - w(w-1)/2 and zeros = total - (true entries of c and s),
     merge c into s if w <= max_w and (w <= small_w or zeros*den <= num*total).
     Supernode rows = its columns followed by struct(last column).

Plain Python; meant for inputs up to a few tens of thousands of columns.
"""
from collections import deque

import numpy as np
import scipy.sparse as sp

AMALGAMATION_MENU = [(1 << 30, 8, 1, 10), (128, 16, 1, 20), (64, 8, 1, 10)]
ND_LEAF = 64


# ----------------------------------------------------------------- pattern
def kkt_pattern(n, J_rowptr, J_colind, H_rowptr=None, H_colind=None):
    """Adjacency lists (no self loops) of the structure of
    K = H + diag + J'J, from CSR patterns of J (m x n) and lower H (n x n)."""
    m = len(J_rowptr) - 1
    nnzj = int(J_rowptr[-1])
    Jb = sp.csr_matrix((np.ones(nnzj), np.asarray(J_colind), np.asarray(J_rowptr)),
                       shape=(m, n))
    S = (Jb.T @ Jb).tocsr()
    if H_rowptr is not None:
        nnzh = int(H_rowptr[-1])
        Hb = sp.csr_matrix((np.ones(nnzh), np.asarray(H_colind), np.asarray(H_rowptr)),
                           shape=(n, n))
        S = S + Hb + Hb.T
    return adjacency_from_sym(S.tocsr(), n)


def dual_pattern(m, n, J_rowptr, J_colind):
    """Adjacency lists (no self loops) of the structure of the dual
    condensed matrix M = diag + J D J' (m x m), from J's CSR pattern."""
    nnzj = int(J_rowptr[-1])
    Jb = sp.csr_matrix((np.ones(nnzj), np.asarray(J_colind), np.asarray(J_rowptr)), shape=(m, n))
    return adjacency_from_sym((Jb @ Jb.T).tocsr(), m)


def augmented_pattern(n, m, J_rowptr, J_colind, H_rowptr, H_colind):
    """Adjacency lists (no self loops) of the structure of the augmented
    matrix [H J'; J diag] (x block 0..n-1, lambda block n..n+m-1)."""
    nnzj = int(J_rowptr[-1])
    Jb = sp.csr_matrix((np.ones(nnzj), np.asarray(J_colind), np.asarray(J_rowptr)), shape=(m, n))
    nnzh = int(H_rowptr[-1])
    Hb = sp.csr_matrix((np.ones(nnzh), np.asarray(H_colind), np.asarray(H_rowptr)), shape=(n, n))
    S = sp.bmat([[Hb + Hb.T, Jb.T], [Jb, None]], format="csr")
    return adjacency_from_sym(S, n + m)


def pattern_from_lower_csr(n, rowptr, colind):
    nnz = int(rowptr[-1])
    L = sp.csr_matrix((np.ones(nnz), np.asarray(colind), np.asarray(rowptr)), shape=(n, n))
    return adjacency_from_sym((L + L.T).tocsr(), n)


def adjacency_from_sym(S, n):
    S.sort_indices()
    adj = []
    for v in range(n):
        row = S.indices[S.indptr[v]:S.indptr[v + 1]]
        adj.append([int(u) for u in row if u != v])
    return adj


# ---------------------------------------------------------------- ordering
def _components(adj, verts, inset):
    """Connected components of G[verts] (inset marks membership), each sorted,
    in increasing order of their smallest vertex."""
    seen = set()
    comps = []
    for v in sorted(verts):
        if v in seen:
            continue
        comp = [v]
        seen.add(v)
        q = deque([v])
        while q:
            u = q.popleft()
            for w in adj[u]:
                if inset[w] and w not in seen:
                    seen.add(w)
                    comp.append(w)
                    q.append(w)
        comps.append(sorted(comp))
    return comps


def _bfs_levels(adj, root, inset):
    levels = [[root]]
    seen = {root}
    while True:
        nxt = []
        for u in levels[-1]:
            for w in adj[u]:
                if inset[w] and w not in seen:
                    seen.add(w)
                    nxt.append(w)
        if not nxt:
            return levels
        levels.append(nxt)


def _min_degree_vertex(cands, deg):
    return min(cands, key=lambda v: (deg[v], v))


def pseudo_peripheral(adj, comp, inset):
    deg = {v: sum(1 for w in adj[v] if inset[w]) for v in comp}
    r = _min_degree_vertex(comp, deg)
    levels = _bfs_levels(adj, r, inset)
    while True:
        v = _min_degree_vertex(levels[-1], deg)
        lv = _bfs_levels(adj, v, inset)
        if len(lv) > len(levels):
            r, levels = v, lv
        else:
            return r, levels


def exact_minimum_degree(adj, comp, inset):
    nbr = {v: set(w for w in adj[v] if inset[w]) for v in comp}
    remaining = set(comp)
    out = []
    while remaining:
        v = min(remaining, key=lambda u: (len(nbr[u]), u))
        out.append(v)
        clique = nbr[v]
        for u in clique:
            nbr[u] |= clique
            nbr[u].discard(u)
            nbr[u].discard(v)
        remaining.discard(v)
        del nbr[v]
    return out


def _choose_separator(levels):
    h = len(levels) - 1
    sizes = [len(L) for L in levels]
    total = sum(sizes)
    best = None
    below = sizes[0]
    for l in range(1, h):
        above = total - below - sizes[l]
        denom = min(below, above)
        # compare sizes[l]/denom exactly: key as a fraction
        cand = (sizes[l], denom, abs(2 * l - h), l)
        if best is None:
            best = cand
        else:
            lhs = cand[0] * best[1]
            rhs = best[0] * cand[1]
            if lhs < rhs or (lhs == rhs and (cand[2], cand[3]) < (best[2], best[3])):
                best = cand
        below += sizes[l]
    return best[3]


# ------------------------------------------- multilevel bisection (ORD-ML)
# Multilevel graph bisection in the style of METIS (Karypis and Kumar):
# coarsen by heavy-edge matching, bisect the coarsest graph, refine the
# partition on every level on the way back, then take a vertex separator
# from the edge cut.  Every step is deterministic (ties by smallest index).
ML_COARSEN_TO = 64          # stop coarsening at this many vertices ...
ML_SHRINK_NUM, ML_SHRINK_DEN = 9, 10   # ... or when a level keeps > 9/10 of them
ML_PASSES = 8               # refinement passes per level
ML_BAL_NUM, ML_BAL_DEN = 11, 20        # a part may hold at most 11/20 of the weight


def _ml_local_graph(adj, comp, inset):
    """G[comp] with local ids (positions in the sorted comp), unit weights."""
    idx = {v: i for i, v in enumerate(comp)}
    nbrs = [[idx[w] for w in adj[v] if inset[w]] for v in comp]
    return nbrs, [[1] * len(r) for r in nbrs], [1] * len(comp)


def _ml_coarsen(nbrs, ew, vw):
    """Heavy-edge matching: vertices in increasing index; an unmatched v
    takes the unmatched neighbour of largest edge weight (ties: smaller
    vertex weight, then smaller index), or stays alone.  Coarse vertices are
    numbered in the order their first member is visited; parallel edges add
    their weights, vertex weights add."""
    n = len(vw)
    matched = [False] * n
    cmap = [-1] * n
    groups = []
    for v in range(n):
        if matched[v]:
            continue
        best, bkey = -1, None
        for u, w in zip(nbrs[v], ew[v]):
            if matched[u]:
                continue
            key = (-w, vw[u], u)
            if best < 0 or key < bkey:
                best, bkey = u, key
        matched[v] = True
        cmap[v] = len(groups)
        if best >= 0:
            matched[best] = True
            cmap[best] = len(groups)
            groups.append((v, best))
        else:
            groups.append((v,))
    cn, ce, cw = [], [], []
    for c, g in enumerate(groups):
        acc = {}
        for v in g:
            for u, w in zip(nbrs[v], ew[v]):
                if cmap[u] != c:
                    acc[cmap[u]] = acc.get(cmap[u], 0) + w
        keys = sorted(acc)
        cn.append(keys)
        ce.append([acc[k] for k in keys])
        cw.append(sum(vw[v] for v in g))
    return cmap, cn, ce, cw


def _ml_bfs_levels(nbrs, root):
    levels = [[root]]
    seen = {root}
    while True:
        nxt = []
        for u in levels[-1]:
            for w in nbrs[u]:
                if w not in seen:
                    seen.add(w)
                    nxt.append(w)
        if not nxt:
            return levels
        levels.append(nxt)


def _ml_initial(nbrs, vw):
    """Part 0 = the shortest prefix of a BFS order from a pseudo-peripheral
    vertex whose weight reaches half the total; the rest is part 1."""
    n = len(vw)
    total = sum(vw)
    deg = [len(r) for r in nbrs]
    r = min(range(n), key=lambda v: (deg[v], v))
    levels = _ml_bfs_levels(nbrs, r)
    while True:
        v = min(levels[-1], key=lambda u: (deg[u], u))
        lv = _ml_bfs_levels(nbrs, v)
        if len(lv) > len(levels):
            levels = lv
        else:
            break
    part = [1] * n
    w0 = 0
    for v in (u for L in levels for u in L):
        if 2 * w0 >= total:
            break
        part[v] = 0
        w0 += vw[v]
    return part


def _ml_refine(nbrs, ew, vw, part):
    """Greedy boundary refinement: each pass visits the boundary vertices in
    order of decreasing gain (cut edge weight removed by moving; ties by
    index), with gains kept current, and moves a vertex when its gain is
    positive and the target part stays within the balance bound, or when its
    gain is zero and the move strictly narrows the weight difference.  Passes
    repeat until none moves (at most ML_PASSES)."""
    n = len(vw)
    total = sum(vw)
    maxw = ML_BAL_NUM * total // ML_BAL_DEN
    pw = [0, 0]
    for v in range(n):
        pw[part[v]] += vw[v]
    ext, inn = [0] * n, [0] * n
    for v in range(n):
        for u, w in zip(nbrs[v], ew[v]):
            if part[u] == part[v]:
                inn[v] += w
            else:
                ext[v] += w
    for _ in range(ML_PASSES):
        cands = sorted((v for v in range(n) if ext[v] > 0), key=lambda v: (inn[v] - ext[v], v))
        moved = False
        for v in cands:
            gain = ext[v] - inn[v]
            src, dst = part[v], 1 - part[v]
            if not ((gain > 0 and pw[dst] + vw[v] <= maxw) or (gain == 0 and pw[src] > pw[dst] + vw[v])):
                continue
            part[v] = dst
            pw[src] -= vw[v]
            pw[dst] += vw[v]
            ext[v], inn[v] = inn[v], ext[v]
            for u, w in zip(nbrs[v], ew[v]):
                if part[u] == dst:
                    inn[u] += w
                    ext[u] -= w
                else:
                    ext[u] += w
                    inn[u] -= w
            moved = True
        if not moved:
            break
    return part


def multilevel_separator(adj, comp, inset):
    """(lower, upper, separator) of the connected component comp (sorted),
    or None when the bisection leaves a side empty.  The separator is the
    smaller of the two boundary sets of the refined edge bisection (ties:
    part 0's); lower = part 0 without it, upper = part 1 without it."""
    graphs = [_ml_local_graph(adj, comp, inset)]
    cmaps = []
    while len(graphs[-1][2]) > ML_COARSEN_TO:
        cmap, cn, ce, cw = _ml_coarsen(*graphs[-1])
        if len(cw) * ML_SHRINK_DEN > ML_SHRINK_NUM * len(graphs[-1][2]):
            break
        cmaps.append(cmap)
        graphs.append((cn, ce, cw))
    part = _ml_refine(*graphs[-1], _ml_initial(graphs[-1][0], graphs[-1][2]))
    for lvl in range(len(cmaps) - 1, -1, -1):
        part = _ml_refine(*graphs[lvl], [part[c] for c in cmaps[lvl]])
    nbrs = graphs[0][0]
    bnd = [[v for v in range(len(comp)) if part[v] == p and any(part[u] != p for u in nbrs[v])]
           for p in (0, 1)]
    sep = set(bnd[0] if len(bnd[0]) <= len(bnd[1]) else bnd[1])
    lower = [comp[v] for v in range(len(comp)) if part[v] == 0 and v not in sep]
    upper = [comp[v] for v in range(len(comp)) if part[v] == 1 and v not in sep]
    if not lower or not upper:
        return None
    return lower, upper, [comp[v] for v in sorted(sep)]


def _degree_order(adj, comp, inset):
    deg = {v: sum(1 for u in adj[v] if inset[u]) for v in comp}
    return sorted(comp, key=lambda v: (deg[v], v))


def nested_dissection(adj, n, leaf=ND_LEAF, method="levels"):
    """ND order as a list: entry k = vertex placed at position k.  method
    "levels": separators are BFS levels (ORD); "multilevel": separators from
    multilevel bisection (ORD-ML), the level rule where that leaves a side
    empty."""
    out = []
    inset = [False] * n
    # work stack of ("order", vertex list) or ("emit", vertex list)
    stack = [("order", list(range(n)))]
    while stack:
        kind, verts = stack.pop()
        if kind == "emit":
            out.extend(verts)
            continue
        for v in verts:
            inset[v] = True
        comps = _components(adj, verts, inset)
        tasks = []
        for comp in comps:
            if len(comp) <= leaf:
                tasks.append(("emit", exact_minimum_degree(adj, comp, inset)))
                continue
            _, levels = pseudo_peripheral(adj, comp, inset)
            h = len(levels) - 1
            if h < 2:
                tasks.append(("emit", _degree_order(adj, comp, inset)))
                continue
            ml = multilevel_separator(adj, comp, inset) if method == "multilevel" else None
            if ml is not None:
                lower, upper, sep = ml
            else:
                l = _choose_separator(levels)
                lower = [v for L in levels[:l] for v in L]
                upper = [v for L in levels[l + 1:] for v in L]
                sep = levels[l]
            for v in sep:
                inset[v] = False
            biggest = max(len(c) for c in _components(adj, lower + upper, inset))
            for v in sep:
                inset[v] = True
            if 8 * biggest > 7 * len(comp):
                tasks.append(("emit", _degree_order(adj, comp, inset)))
                continue
            tasks.append(("order", sorted(lower)))
            tasks.append(("order", sorted(upper)))
            tasks.append(("emit", sorted(sep)))
        for v in verts:
            inset[v] = False
        for t in reversed(tasks):
            stack.append(t)
    return out


# --------------------------------------------------------------- symbolic
def permuted_lower_columns(adj, perm):
    """For each column j of P'KP, the sorted row indices i > j."""
    n = len(perm)
    pinv = np.empty(n, dtype=np.int64)
    pinv[np.asarray(perm, dtype=np.int64)] = np.arange(n)
    cols = []
    for j in range(n):
        rows = pinv[np.asarray(adj[perm[j]], dtype=np.int64)]
        cols.append(np.sort(rows[rows > j]))
    return cols


def symbolic_factor(lower_cols):
    """Column structures of L (below the diagonal), elimination tree."""
    n = len(lower_cols)
    parent = np.full(n, -1, dtype=np.int64)
    pending = [[] for _ in range(n)]
    structs = []
    for j in range(n):
        parts = [lower_cols[j]] + [s[1:] for s in pending[j]]
        pending[j] = None
        st = np.unique(np.concatenate(parts)) if len(parts) > 1 else lower_cols[j]
        structs.append(st)
        if len(st):
            p = int(st[0])
            parent[j] = p
            pending[p].append(st)
    return structs, parent


def postorder(parent):
    n = len(parent)
    children = [[] for _ in range(n)]
    roots = []
    for j in range(n):
        (roots if parent[j] < 0 else children[parent[j]]).append(j)
    out = []
    for r in roots:
        stack = [(r, 0)]
        while stack:
            v, i = stack.pop()
            if i < len(children[v]):
                stack.append((v, i + 1))
                stack.append((children[v][i], 0))
            else:
                out.append(v)
    return out


def fundamental_supernodes(parent, cc):
    n = len(parent)
    nchild = np.zeros(n, dtype=np.int64)
    for j in range(n):
        if parent[j] >= 0:
            nchild[parent[j]] += 1
    starts = [0] if n else []
    for j in range(n - 1):
        joins = parent[j] == j + 1 and cc[j] == cc[j + 1] + 1 and nchild[j + 1] == 1
        if not joins:
            starts.append(j + 1)
    return starts


def amalgamate(starts, parent, cc, menu=AMALGAMATION_MENU[0]):
    max_w, small_w, num, den = menu
    n = len(parent)
    sns = [[s, e - 1] for s, e in zip(starts, starts[1:] + [n])]  # inclusive
    true_nz = [int(np.sum(cc[a:b + 1])) for a, b in sns]
    owner = np.empty(n, dtype=np.int64)
    for k, (a, b) in enumerate(sns):
        owner[a:b + 1] = k
    # owner ids must stay valid while the list shrinks: keep ids stable by
    # giving each supernode a token, mapping columns to tokens.
    token = list(range(len(sns)))
    i = 0
    while i < len(sns):
        while i > 0:
            c_first, c_last = sns[i - 1]
            s_first, s_last = sns[i]
            p = parent[c_last]
            if p < 0 or owner[p] != token[i]:
                break
            wc = c_last - c_first + 1
            ws = s_last - s_first + 1
            hs = ws + int(cc[s_last]) - 1
            w = wc + ws
            h = wc + hs
            if w > max_w:
                break
            total = w * h - w * (w - 1) // 2
            zeros = total - (true_nz[i - 1] + true_nz[i])
            if not (w <= small_w or zeros * den <= num * total):
                break
            owner[c_first:c_last + 1] = token[i]
            sns[i] = [c_first, s_last]
            true_nz[i] += true_nz[i - 1]
            del sns[i - 1], true_nz[i - 1], token[i - 1]
            i -= 1
        i += 1
    return [a for a, _ in sns] + [n]


def analyze(adj, n, leaf=ND_LEAF, menu=AMALGAMATION_MENU[0], method="levels"):
    """Full symbolic analysis.  Returns a dict with perm (perm[k] = original
    index at position k), etree, colcount, sn_start, sn_rowptr, sn_rows,
    nnz_L (true) and flops = sum_j (c_j^2 - 1).  method selects the
    separators of the nested dissection ("levels" or "multilevel")."""
    nd = nested_dissection(adj, n, leaf, method)
    cols = permuted_lower_columns(adj, nd)
    _, par0 = symbolic_factor(cols)
    post = postorder(par0)
    perm = [nd[k] for k in post]
    cols = permuted_lower_columns(adj, perm)
    structs, parent = symbolic_factor(cols)
    cc = np.array([len(s) + 1 for s in structs], dtype=np.int64)
    fund = fundamental_supernodes(parent, cc)
    sn_start = amalgamate(fund, parent, cc, menu)
    rowptr = [0]
    rows = []
    for a, b in zip(sn_start[:-1], sn_start[1:]):
        r = np.concatenate([np.arange(a, b), structs[b - 1]]).astype(np.int32)
        rows.append(r)
        rowptr.append(rowptr[-1] + len(r))
    return dict(perm=np.asarray(perm, dtype=np.int32), etree=parent.astype(np.int32),
                colcount=cc, sn_start=np.asarray(sn_start, dtype=np.int32),
                sn_rowptr=np.asarray(rowptr, dtype=np.int64),
                sn_rows=np.concatenate(rows) if rows else np.zeros(0, np.int32),
                structs=structs, nnz_L=int(cc.sum()), flops=int(np.sum(cc * cc - 1)))
