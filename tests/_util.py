"""Shared helpers of the tests (no solver arithmetic)."""
import re
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    """Names of the functions declared in include/*.h."""
    names = []
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(inc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.append(m.group(1))
    return names


def dense_from_panels(sym, lval):
    """Lower factor L (permuted numbering) from the exported panels."""
    n = len(sym["perm"])
    L = np.zeros((n, n))
    off = 0
    st, rp, rows = sym["sn_start"], sym["sn_rowptr"], sym["sn_rows"]
    for k in range(len(st) - 1):
        f, w = st[k], st[k + 1] - st[k]
        r = rows[rp[k]:rp[k + 1]]
        h = len(r)
        P = lval[off:off + h * w].reshape(w, h).T
        for c in range(w):
            L[r[c:], f + c] = P[c:, c]
        off += h * w
    return L


def sparse_from_panels(sym, lval):
    import scipy.sparse as sp
    st, rp, rows = sym["sn_start"], sym["sn_rowptr"], sym["sn_rows"]
    n = len(sym["perm"])
    R, C, V = [], [], []
    off = 0
    for k in range(len(st) - 1):
        f, w = st[k], st[k + 1] - st[k]
        r = rows[rp[k]:rp[k + 1]]
        h = len(r)
        P = lval[off:off + h * w].reshape(w, h).T
        for c in range(w):
            R.append(r[c:]); C.append(np.full(h - c, f + c)); V.append(P[c:, c])
        off += h * w
    return sp.csc_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(n, n))


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
