"""ctypes wrapper over oracle/cholesky.c (test infrastructure only).

``build()`` compiles the C file with gcc next to this module; the wrapper
compiles it on first use when the shared object is missing.
"""
import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cholesky.c")
_SO = os.path.join(_HERE, "_cholesky.so")
_lib = None


def build():
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        L.oracle_dense_cholesky.argtypes = [i64, p]
        L.oracle_dense_cholesky.restype = ctypes.c_int
        L.oracle_dense_solve.argtypes = [i64, p, p]
        L.oracle_sparse_cholesky.argtypes = [i64, p, p, p]
        L.oracle_sparse_cholesky.restype = ctypes.c_int
        L.oracle_sparse_solve.argtypes = [i64, p, p, p, p]
        L.oracle_sparse_ldlt.argtypes = [i64, p, p, p, p]
        L.oracle_sparse_ldlt.restype = ctypes.c_int
        L.oracle_sparse_ldlt_solve.argtypes = [i64, p, p, p, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def dense_cholesky(K):
    """Lower L with K = L L' (FP64).  Raises NotPositiveDefinite."""
    A = np.array(K, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    st = lib().oracle_dense_cholesky(n, _ptr(A))
    if st:
        raise NotPositiveDefinite(st - 1)
    return np.tril(A)


def dense_solve(L, b):
    L = np.ascontiguousarray(L, dtype=np.float64)
    x = np.array(b, dtype=np.float64, copy=True)
    lib().oracle_dense_solve(L.shape[0], _ptr(L), _ptr(x))
    return x


class SingularPivot(ArithmeticError):
    def __init__(self, col):
        super().__init__(f"zero or non-finite pivot at column {col}")
        self.col = col


class NotPositiveDefinite(ArithmeticError):
    def __init__(self, col):
        super().__init__(f"non-positive pivot at column {col}")
        self.col = col


class SparseFactor:
    """L (CSC, permuted numbering) of P'KP for a fixed symbolic structure."""

    def __init__(self, perm, structs):
        self.perm = np.asarray(perm, dtype=np.int64)
        n = len(self.perm)
        self.n = n
        counts = np.array([len(s) + 1 for s in structs], dtype=np.int64)
        self.Lp = np.zeros(n + 1, dtype=np.int64)
        self.Lp[1:] = np.cumsum(counts)
        self.Li = np.concatenate([np.concatenate([[j], s]) for j, s in enumerate(structs)]
                                 ).astype(np.int32) if n else np.zeros(0, np.int32)
        self.pinv = np.empty(n, dtype=np.int64)
        self.pinv[self.perm] = np.arange(n)
        self.Lx = None

    def factor(self, K):
        """K: symmetric scipy sparse matrix in the original numbering."""
        n = self.n
        Kp = sp.csc_matrix(K)[self.perm, :][:, self.perm]
        Kl = sp.tril(Kp).tocsc()
        Kl.sort_indices()
        Lx = np.zeros(len(self.Li))
        # place K's entries into L's structure
        col_of = np.repeat(np.arange(n), np.diff(Kl.indptr))
        pos = {}
        for j in range(n):
            rows = self.Li[self.Lp[j]:self.Lp[j + 1]]
            pos_j = self.Lp[j] + np.searchsorted(rows, Kl.indices[Kl.indptr[j]:Kl.indptr[j + 1]])
            Lx[pos_j] = Kl.data[Kl.indptr[j]:Kl.indptr[j + 1]]
        st = lib().oracle_sparse_cholesky(n, _ptr(self.Lp), _ptr(self.Li), _ptr(Lx))
        if st:
            raise NotPositiveDefinite(st - 1)
        self.Lx = Lx
        return self

    def _place(self, K):
        """K's lower entries (permuted) placed into L's structure."""
        n = self.n
        Kp = sp.csc_matrix(K)[self.perm, :][:, self.perm]
        Kl = sp.tril(Kp).tocsc()
        Kl.sort_indices()
        Lx = np.zeros(len(self.Li))
        for j in range(n):
            rows = self.Li[self.Lp[j]:self.Lp[j + 1]]
            pos_j = self.Lp[j] + np.searchsorted(rows, Kl.indices[Kl.indptr[j]:Kl.indptr[j + 1]])
            Lx[pos_j] = Kl.data[Kl.indptr[j]:Kl.indptr[j + 1]]
        return Lx

    def factor_ldlt(self, K):
        """P'KP = L D L' with unit lower L and D of either sign (no
        pivoting); self.D holds D.  Raises SingularPivot."""
        Lx = self._place(K)
        D = np.zeros(self.n)
        st = lib().oracle_sparse_ldlt(self.n, _ptr(self.Lp), _ptr(self.Li), _ptr(Lx), _ptr(D))
        if st:
            raise SingularPivot(st - 1)
        self.Lx, self.D = Lx, D
        return self

    def solve_ldlt(self, b):
        x = np.array(np.asarray(b, dtype=np.float64)[self.perm], copy=True)
        lib().oracle_sparse_ldlt_solve(self.n, _ptr(self.Lp), _ptr(self.Li), _ptr(self.Lx), _ptr(self.D),
                                       _ptr(x))
        out = np.empty(self.n)
        out[self.perm] = x
        return out

    def solve(self, b):
        x = np.array(np.asarray(b, dtype=np.float64)[self.perm], copy=True)
        lib().oracle_sparse_solve(self.n, _ptr(self.Lp), _ptr(self.Li), _ptr(self.Lx), _ptr(x))
        out = np.empty(self.n)
        out[self.perm] = x
        return out

    def to_dense(self):
        n = self.n
        L = np.zeros((n, n))
        for j in range(n):
            L[self.Li[self.Lp[j]:self.Lp[j + 1]], j] = self.Lx[self.Lp[j]:self.Lp[j + 1]]
        return L
