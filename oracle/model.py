"""Model evaluation for  min f(x)  s.t.  g(x) >= 0,  xl <= x <= xu
(Section 1, problem (1); equality-free form as in the paper).

    f(x) = c'x + 1/2 x'Qx + sum_i q4_i x_i^4 / 4
    g(x) = A x - b - W (x * x)
    J(x) = A - 2 W diag(x)                      (Jacobian of g)
    H(x, lam) = Q + diag(3 q4 x^2) + 2 diag(W' lam)
              = Hessian of the Lagrangian f - lam'(g - s)
                (the (1,1) block of eq. kkt_system, Section 3)

Plain scipy.sparse arithmetic in FP64; ``problem`` is any object with the
attributes n, m, c, b, A, Q, q4, W, xl, xu (CSR parts rowptr/colind/val).
"""
import numpy as np
import scipy.sparse as sp


def csr(mat, nrows, ncols):
    if mat is None:
        return sp.csr_matrix((nrows, ncols))
    return sp.csr_matrix((np.asarray(mat.val, float), np.asarray(mat.colind),
                          np.asarray(mat.rowptr)), shape=(nrows, ncols))


def q_full(problem):
    """Symmetric Q from its lower triangle."""
    L = csr(problem.Q, problem.n, problem.n)
    d = L.diagonal()
    return (L + L.T - sp.diags(d)).tocsr()


def parts(problem):
    n, m = problem.n, problem.m
    A = csr(problem.A, m, n)
    W = csr(problem.W, m, n)
    Q = q_full(problem)
    q4 = np.zeros(n) if problem.q4 is None else np.asarray(problem.q4, float)
    return A, W, Q, q4


def objective(problem, x):
    A, W, Q, q4 = parts(problem)
    return float(problem.c @ x + 0.5 * x @ (Q @ x) + np.sum(q4 * x ** 4) / 4.0)


def gradient(problem, x):
    A, W, Q, q4 = parts(problem)
    return problem.c + Q @ x + q4 * x ** 3


def constraints(problem, x):
    A, W, Q, q4 = parts(problem)
    return A @ x - problem.b - W @ (x * x)


def jacobian(problem, x):
    """J = A - 2 W diag(x), as a scipy CSR matrix."""
    A, W, Q, q4 = parts(problem)
    return (A - 2.0 * W @ sp.diags(x)).tocsr()


def jacobian_pattern(problem):
    """CSR structure (row pointers, column indices) of J's fixed pattern: the
    union of the patterns of A and W, whatever the values of x (Section 4:
    derivatives live on fixed sparsity patterns; Section 2: the symbolic
    analysis is done once on that pattern).  Taken from the values of J at
    one point instead, entries of W that vanish there (x_j = 0) would be
    missing from the pattern."""
    n, m = problem.n, problem.m
    S = sp.csr_matrix((m, n))
    for M in (problem.A, problem.W):
        if M is not None and int(M.rowptr[-1]) > 0:
            S = S + sp.csr_matrix((np.ones(int(M.rowptr[-1])), np.asarray(M.colind), np.asarray(M.rowptr)),
                                  shape=(m, n))
    S = S.tocsr()
    S.sort_indices()
    return S.indptr, S.indices


def hessian_lower_pattern(problem):
    """CSR structure of the lower triangle of H's fixed pattern: Q's lower
    triangle plus the full diagonal (the q4 and W' lambda terms)."""
    n = problem.n
    S = sp.eye(n, format="csr")
    if problem.Q is not None and int(problem.Q.rowptr[-1]) > 0:
        Q = problem.Q
        S = S + sp.csr_matrix((np.ones(int(Q.rowptr[-1])), np.asarray(Q.colind), np.asarray(Q.rowptr)),
                              shape=(n, n))
    S = sp.tril(S).tocsr()
    S.sort_indices()
    return S.indptr, S.indices


def hessian(problem, x, lam):
    """Symmetric Lagrangian Hessian Q + diag(3 q4 x^2 + 2 W' lam)."""
    A, W, Q, q4 = parts(problem)
    return (Q + sp.diags(3.0 * q4 * x ** 2 + 2.0 * (W.T @ lam))).tocsr()


def bounds(problem):
    n = problem.n
    xl = np.full(n, -np.inf) if problem.xl is None else np.asarray(problem.xl, float)
    xu = np.full(n, np.inf) if problem.xu is None else np.asarray(problem.xu, float)
    return xl, xu


def kind(problem):
    A, W, Q, q4 = parts(problem)
    if W.nnz > 0 or np.any(q4 != 0):
        return "nlp"
    if Q.nnz > 0:
        return "qp"
    return "lp"
