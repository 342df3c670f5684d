"""Seeded synthetic problem generators.

This module only draws random problem data; it holds none of the solver's
arithmetic.  Both the HIP path (through the tests and the benchmark) and the
CPU oracle's tests take their inputs from here.

Problem form (Section 1, problem (1), with the data layout of the library):
    minimise   c'x + 1/2 x'Qx + sum_i q4_i x_i^4 / 4
    subject to g(x) = A x - b - W (x*x) >= 0,   xl <= x <= xu
All matrices are CSR with 0-based, sorted, duplicate-free column indices.
Q is given by its lower triangle (diagonal included).

Workloads (shapes follow the paper's benchmark families; the public suites
themselves are not available, these synthetic instances stand in for them):
  lp_small      n=500, m=200 sparse LP, 5 nnz/col (small MIPLIB-like LP)
  lp_block      block-angular LP, 200 blocks of 5k rows x 10k cols, 6 nnz/col,
                plus 20k linking rows of 20 nnz (large MIPLIB-like LP)
  nlp_grid      x^4 + Laplacian objective on a grid with quadratic stencil
                constraints (COPS-like grid PDE NLP)
  qp_batch      4096 uneven parametric LP/QP instances, n log-uniform [50,2000]
  qp_param      fixed-structure QP with b(theta) = b0 + B theta (warm start)
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 250816094


def seed_for(config: int, instance: int = 0) -> int:
    return SEED_BASE + 1000 * config + instance


@dataclasses.dataclass
class CSR:
    nrows: int
    ncols: int
    rowptr: np.ndarray  # int64 [nrows+1]
    colind: np.ndarray  # int32 [nnz]
    val: np.ndarray     # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr),
                             shape=(self.nrows, self.ncols))


@dataclasses.dataclass
class Problem:
    n: int
    m: int
    c: np.ndarray
    b: np.ndarray
    A: Optional[CSR] = None
    Q: Optional[CSR] = None          # lower triangle incl. diagonal
    q4: Optional[np.ndarray] = None
    W: Optional[CSR] = None          # entries >= 0
    xl: Optional[np.ndarray] = None  # -inf allowed
    xu: Optional[np.ndarray] = None  # +inf allowed
    name: str = ""

    @property
    def kind(self) -> str:
        nonlinear = (self.W is not None and self.W.nnz > 0) or (
            self.q4 is not None and np.any(self.q4 != 0))
        if nonlinear:
            return "nlp"
        if self.Q is not None and self.Q.nnz > 0:
            return "qp"
        return "lp"


def csr_from_columns(nrows: int, ncols: int, col_rows: np.ndarray,
                     col_vals: np.ndarray) -> CSR:
    """Build a CSR from per-column entries given as flat (col-major) arrays.

    col_rows/col_vals have shape [ncols, k] (k entries per column)."""
    k = col_rows.shape[1]
    cols = np.repeat(np.arange(ncols, dtype=np.int64), k)
    rows = col_rows.reshape(-1).astype(np.int64)
    vals = col_vals.reshape(-1)
    return csr_from_coo(nrows, ncols, rows, cols, vals)


def csr_from_coo(nrows, ncols, rows, cols, vals) -> CSR:
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], np.asarray(vals, dtype=np.float64)[order]
    if len(rows) > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if np.any(dup):
            raise ValueError("duplicate entries")
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int64)
    return CSR(nrows, ncols, rowptr, cols.astype(np.int32), vals)


def _distinct_rows(rng: np.random.Generator, ncols: int, k: int, lo: np.ndarray,
                   span: np.ndarray) -> np.ndarray:
    """k distinct uniform rows per column, column j drawing from
    [lo[j], lo[j] + span[j]).  Vectorised draw with redraw of duplicates."""
    r = rng.integers(0, span[:, None], size=(ncols, k))
    while True:
        s = np.sort(r, axis=1)
        dup_cols = np.nonzero(np.any(s[:, 1:] == s[:, :-1], axis=1))[0]
        if len(dup_cols) == 0:
            break
        r[dup_cols] = rng.integers(0, span[dup_cols, None], size=(len(dup_cols), k))
    return np.sort(r, axis=1) + lo[:, None]


def _feasible_lp_tail(rng, A: CSR, n: int, m: int):
    """x0 ~ U(1,9), s ~ U(0.1,1), b = A x0 - s, c ~ N(0,1)."""
    x0 = rng.uniform(1.0, 9.0, size=n)
    s = rng.uniform(0.1, 1.0, size=m)
    b = A.to_scipy() @ x0 - s
    c = rng.standard_normal(n)
    return x0, s, b, c


def random_lp(n: int, m: int, nnz_per_col: int, seed: int, name: str = "lp") -> Problem:
    """LP min c'x s.t. Ax >= b, 0 <= x <= 10; A has nnz_per_col distinct
    uniform rows per column with N(0,1) values (draw order: rows, values,
    x0, s, c)."""
    rng = np.random.default_rng(seed)
    k = min(nnz_per_col, m)
    rows = _distinct_rows(rng, n, k, np.zeros(n, np.int64), np.full(n, m, np.int64))
    vals = rng.standard_normal((n, k))
    A = csr_from_columns(m, n, rows, vals)
    _, _, b, c = _feasible_lp_tail(rng, A, n, m)
    return Problem(n=n, m=m, c=c, b=b, A=A, xl=np.zeros(n), xu=np.full(n, 10.0), name=name)


def lp_small(instance: int = 0) -> Problem:
    """Plain FP64 LP: n=500, m=200, 5 nnz/col."""
    return random_lp(500, 200, 5, seed_for(1, instance), name=f"lp_small[{instance}]")


def lp_block(nblocks: int = 200, block_rows: int = 5000, block_cols: int = 10000,
             nnz_per_col: int = 6, n_link_rows: Optional[int] = None,
             link_nnz: int = 20, link_cols_per_block: int = 100,
             instance: int = 0) -> Problem:
    """Block-angular LP.  Block b owns rows [b*R, (b+1)*R) and columns
    [b*C, (b+1)*C); each column has nnz_per_col distinct uniform rows in its
    block.  Linking rows (default 2% of the block rows) each pick link_nnz
    distinct blocks and, in each, one of that block's first
    link_cols_per_block columns.  Defaults give n=2,000,000, m=1,020,000."""
    rng = np.random.default_rng(seed_for(2, instance))
    n = nblocks * block_cols
    mb = nblocks * block_rows
    if n_link_rows is None:
        n_link_rows = mb // 50
    m = mb + n_link_rows
    blk = np.arange(n, dtype=np.int64) // block_cols
    rows = _distinct_rows(rng, n, nnz_per_col, blk * block_rows,
                          np.full(n, block_rows, np.int64))
    vals = rng.standard_normal((n, nnz_per_col))
    r_all = [rows.reshape(-1)]
    c_all = [np.repeat(np.arange(n, dtype=np.int64), nnz_per_col)]
    v_all = [vals.reshape(-1)]
    if n_link_rows > 0:
        lk = min(link_nnz, nblocks)
        # distinct blocks per linking row: argsort of uniform keys
        keys = rng.random((n_link_rows, nblocks))
        blocks = np.sort(np.argsort(keys, axis=1)[:, :lk], axis=1)
        lcol = rng.integers(0, min(link_cols_per_block, block_cols), size=(n_link_rows, lk))
        lval = rng.standard_normal((n_link_rows, lk))
        r_all.append(np.repeat(mb + np.arange(n_link_rows, dtype=np.int64), lk))
        c_all.append((blocks * block_cols + lcol).reshape(-1))
        v_all.append(lval.reshape(-1))
    A = csr_from_coo(m, n, np.concatenate(r_all), np.concatenate(c_all), np.concatenate(v_all))
    _, _, b, c = _feasible_lp_tail(rng, A, n, m)
    return Problem(n=n, m=m, c=c, b=b, A=A, xl=np.zeros(n), xu=np.full(n, 10.0),
                   name=f"lp_block[{nblocks}x{block_rows}x{block_cols}]")


def grid_laplacian_lower(nx: int, ny: int, shift: float = 0.0) -> CSR:
    """Lower triangle of the 4-neighbour grid Laplacian (degree - adjacency)
    plus shift*I; node (i, j) has index i*ny + j."""
    idx = np.arange(nx * ny, dtype=np.int64).reshape(nx, ny)
    deg = np.zeros((nx, ny))
    deg[1:, :] += 1; deg[:-1, :] += 1; deg[:, 1:] += 1; deg[:, :-1] += 1
    rows = [idx.reshape(-1)]
    cols = [idx.reshape(-1)]
    vals = [deg.reshape(-1) + shift]
    # neighbour with smaller index: (i-1, j) and (i, j-1)
    rows.append(idx[1:, :].reshape(-1)); cols.append(idx[:-1, :].reshape(-1))
    vals.append(-np.ones((nx - 1) * ny))
    rows.append(idx[:, 1:].reshape(-1)); cols.append(idx[:, :-1].reshape(-1))
    vals.append(-np.ones(nx * (ny - 1)))
    return csr_from_coo(nx * ny, nx * ny, np.concatenate(rows), np.concatenate(cols),
                        np.concatenate(vals))


def nlp_grid(nx: int = 700, ny: int = 700, instance: int = 0) -> Problem:
    """min sum(x^4/4 + c x) + 1/2 x'Lx  s.t.  1 - sum_{j in N(k)} x_j^2/5 >= 0
    for every node k=(i,j) with i+j even; N(k) = k and its in-grid
    4-neighbours (boundary stencils are truncated, still divided by 5).
    c ~ N(0,1); no bounds on x."""
    rng = np.random.default_rng(seed_for(3, instance))
    n = nx * ny
    c = rng.standard_normal(n)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    sel = ((ii + jj) % 2 == 0).reshape(-1)
    centers = np.nonzero(sel)[0]
    m = len(centers)
    ci, cj = centers // ny, centers % ny
    rows, cols = [], []
    for di, dj in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
        ni, nj = ci + di, cj + dj
        ok = (ni >= 0) & (ni < nx) & (nj >= 0) & (nj < ny)
        rows.append(np.nonzero(ok)[0])
        cols.append((ni * ny + nj)[ok])
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    W = csr_from_coo(m, n, rows, cols, np.full(len(rows), 0.2))
    return Problem(n=n, m=m, c=c, b=-np.ones(m), W=W, q4=np.ones(n),
                   Q=grid_laplacian_lower(nx, ny), name=f"nlp_grid[{nx}x{ny}]")


def nlp_grid_nonconvex(nx: int = 40, ny: int = 36, instance: int = 0, neg_frac: float = 0.5,
                       weight: float = 0.2, c_scale: float = 4.0) -> Problem:
    """nlp_grid with mixed-sign stencil weights: each W entry is -weight
    with probability neg_frac, +weight otherwise.  Negative entries make g
    convex in those terms, the feasible set nonconvex and the Lagrangian
    Hessian L + diag(3 x^2) + 2 diag(W' lambda) indefinite where W' lambda
    is negative enough (a nonconvex NLP of the COPS grid shape).  The linear
    term is scaled by c_scale so that some constraints are active at the
    solution (with c ~ N(0,1) alone they are not)."""
    p = nlp_grid(nx, ny, instance)
    p.c = p.c * c_scale
    rng = np.random.default_rng(seed_for(3, 500 + instance))
    sign = np.where(rng.random(p.W.nnz) < neg_frac, -1.0, 1.0)
    p.W = CSR(p.W.nrows, p.W.ncols, p.W.rowptr, p.W.colind, sign * weight)
    p.name = f"nlp_grid_nonconvex[{nx}x{ny}]"
    return p


def qp_batch_sizes(count: int = 4096, nmin: int = 50, nmax: int = 2000,
                   seed: Optional[int] = None) -> np.ndarray:
    rng = np.random.default_rng(seed_for(4, 99999) if seed is None else seed)
    return np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)


def qp_instance(n: int, instance: int, nnz_per_col: int = 4) -> Problem:
    """One batched parametric instance: LP of random_lp form with m = n//2,
    plus diagonal Q = diag(U(0.1, 1)) drawn after c."""
    m = n // 2
    p = random_lp(n, m, nnz_per_col, seed_for(4, instance), name=f"qp_batch[{instance}]")
    rng = np.random.default_rng(seed_for(4, instance) + 500)
    q = rng.uniform(0.1, 1.0, size=n)
    idx = np.arange(n, dtype=np.int64)
    p.Q = CSR(n, n, np.arange(n + 1, dtype=np.int64), idx.astype(np.int32), q)
    return p


def qp_batch(count: int = 4096, nmin: int = 50, nmax: int = 2000) -> list:
    sizes = qp_batch_sizes(count, nmin, nmax)
    return [qp_instance(int(n), i) for i, n in enumerate(sizes)]


@dataclasses.dataclass
class ParamQP:
    base: Problem
    b0: np.ndarray
    B: np.ndarray       # m x p dense

    def instance(self, theta: np.ndarray) -> Problem:
        p = dataclasses.replace(self.base)
        p.b = self.b0 + self.B @ theta
        return p


def qp_param(nx: int = 100, ny: int = 200, nnz_per_col: int = 6, window: int = 64,
             n_theta: int = 64) -> ParamQP:
    """Fixed-structure QP: n = nx*ny, m = n/2, A with nnz_per_col distinct
    rows per column inside a local window of `window` rows starting at
    clamp(floor(j m / n) - window/2, 0, m - window); Q = grid Laplacian + 0.1 I;
    0 <= x <= 10; b(theta) = b0 + B theta, B ~ N(0, 0.1^2)."""
    rng = np.random.default_rng(seed_for(5, 0))
    n = nx * ny
    m = n // 2
    win = min(window, m)
    j = np.arange(n, dtype=np.int64)
    lo = np.clip(j * m // n - win // 2, 0, m - win)
    rows = _distinct_rows(rng, n, min(nnz_per_col, win), lo, np.full(n, win, np.int64))
    vals = rng.standard_normal(rows.shape)
    A = csr_from_columns(m, n, rows, vals)
    _, _, b0, c = _feasible_lp_tail(rng, A, n, m)
    B = rng.normal(0.0, 0.1, size=(m, n_theta))
    base = Problem(n=n, m=m, c=c, b=b0.copy(), A=A, Q=grid_laplacian_lower(nx, ny, 0.1),
                   xl=np.zeros(n), xu=np.full(n, 10.0), name=f"qp_param[{nx}x{ny}]")
    return ParamQP(base=base, b0=b0, B=B)


def thetas(count: int, set_id: int, n_theta: int = 64) -> np.ndarray:
    """theta ~ N(0, I); set 0 = training, set 1 = fresh test (disjoint seeds)."""
    rng = np.random.default_rng(seed_for(5, 1 + set_id))
    return rng.standard_normal((count, n_theta))


def mlp_init(dims, seed: int = seed_for(5, 777)):
    """Initial MLP parameters [(W, b)] for layer sizes dims (W: out x in):
    uniform(-sqrt(6/fan_in), sqrt(6/fan_in)) weights, zero biases; the last
    layer is scaled by 0.1."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        a = math.sqrt(6.0 / fan_in) * (0.1 if l == len(dims) - 2 else 1.0)
        params.append((rng.uniform(-a, a, size=(fan_out, fan_in)), np.zeros(fan_out)))
    return params
