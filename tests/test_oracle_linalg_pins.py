"""Pins of the oracle's linear algebra and derivatives (test infrastructure).

P4 factor identity ||P'KP - LL'||_F / ||K||_F <= 1e-12, positive pivots, and
   agreement with numpy's dense Cholesky (a third reference)
P5 the condensed step equals the step of the full regularised KKT system
   (Section 3, eq. kkt_system, with bound rows), solved densely by LU
P8 derivatives by central finite differences; J_kj = -2 x_j / 5 on the grid
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cholesky as chol
from oracle import kkt, model, symbolic
from paper_2508_16094_amd import workloads as w


def _random_spd_pattern(n, seed, deg=4):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, n, size=n * deg)
    cols = rng.integers(0, n, size=n * deg)
    B = sp.csr_matrix((rng.standard_normal(n * deg), (rows, cols)), shape=(n, n))
    return (B @ B.T + sp.eye(n) * 0.5).tocsr()


@pytest.mark.parametrize("n,seed", [(50, 1), (300, 2), (1200, 3)])
def test_p4_sparse_factor_identity(n, seed):
    K = _random_spd_pattern(n, seed)
    Kl = sp.tril(K).tocsr()
    adj = symbolic.pattern_from_lower_csr(n, Kl.indptr, Kl.indices)
    sym = symbolic.analyze(adj, n)
    F = chol.SparseFactor(sym["perm"], sym["structs"]).factor(K)
    L = F.to_dense()
    Kp = K.toarray()[np.ix_(sym["perm"], sym["perm"])]
    assert np.linalg.norm(Kp - L @ L.T) / np.linalg.norm(Kp) <= 1e-12
    assert np.all(np.diag(L) > 0)
    assert np.max(np.abs(L - np.linalg.cholesky(Kp))) <= 1e-10 * np.max(np.abs(L))
    b = np.random.default_rng(seed).standard_normal(n)
    x = F.solve(b)
    assert np.linalg.norm(K @ x - b) <= 1e-10 * np.linalg.norm(b) * max(1, np.linalg.norm(K.toarray(), 2))


def test_p4_dense_factor_and_not_pd():
    K = _random_spd_pattern(80, 9).toarray()
    L = chol.dense_cholesky(K)
    assert np.linalg.norm(K - L @ L.T) / np.linalg.norm(K) <= 1e-12
    K2 = K.copy()
    K2[10, 10] = -1.0
    with pytest.raises(chol.NotPositiveDefinite):
        chol.dense_cholesky(K2)
    Ksp = sp.csr_matrix(K2)
    Kl = sp.tril(Ksp).tocsr()
    adj = symbolic.pattern_from_lower_csr(80, Kl.indptr, Kl.indices)
    sym = symbolic.analyze(adj, 80)
    with pytest.raises(chol.NotPositiveDefinite):
        chol.SparseFactor(sym["perm"], sym["structs"]).factor(Ksp)


def _full_kkt_step(p, x, s, lam, zl, zu, t_s, t_l, t_u, dp, dd):
    """Dense Newton system in (dx, ds, dlam, dzl, dzu) from eq. kkt_system
    (rows: stationarity, complementarity S lam, regularised feasibility)
    plus the bound complementarity rows; solved by partial-pivot LU."""
    n, m = p.n, p.m
    xl, xu = model.bounds(p)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    L_idx, U_idx = np.nonzero(il)[0], np.nonzero(iu)[0]
    nl, nu = len(L_idx), len(U_idx)
    J = model.jacobian(p, x).toarray()
    H = model.hessian(p, x, lam).toarray()
    gf = model.gradient(p, x)
    g = model.constraints(p, x)
    zl_full = np.where(il, zl, 0); zu_full = np.where(iu, zu, 0)
    r_d = gf - J.T @ lam - zl_full + zu_full
    N = n + 2 * m + nl + nu
    M = np.zeros((N, N)); r = np.zeros(N)
    ix, isl, ilm = slice(0, n), slice(n, n + m), slice(n + m, n + 2 * m)
    izl, izu = slice(n + 2 * m, n + 2 * m + nl), slice(n + 2 * m + nl, N)
    M[ix, ix] = H + dp * np.eye(n); M[ix, ilm] = -J.T
    M[ix, izl] = -np.eye(n)[:, L_idx]; M[ix, izu] = np.eye(n)[:, U_idx]
    r[ix] = -r_d
    M[isl, isl] = np.diag(lam); M[isl, ilm] = np.diag(s); r[isl] = t_s - s * lam
    M[ilm, ix] = J; M[ilm, isl] = -np.eye(m); M[ilm, ilm] = dd * np.eye(m); r[ilm] = -(g - s)
    for k, i in enumerate(L_idx):
        M[n + 2 * m + k, i] = zl[i]; M[n + 2 * m + k, n + 2 * m + k] = x[i] - xl[i]
        r[n + 2 * m + k] = t_l[i] - (x[i] - xl[i]) * zl[i]
    for k, i in enumerate(U_idx):
        M[n + 2 * m + nl + k, i] = -zu[i]; M[n + 2 * m + nl + k, n + 2 * m + nl + k] = xu[i] - x[i]
        r[n + 2 * m + nl + k] = t_u[i] - (xu[i] - x[i]) * zu[i]
    import scipy.linalg
    d = scipy.linalg.lu_solve(scipy.linalg.lu_factor(M), r)
    dzl = np.zeros(n); dzu = np.zeros(n)
    dzl[L_idx] = d[izl]; dzu[U_idx] = d[izu]
    return d[ix], d[isl], d[ilm], dzl, dzu


def _condensed_step(p, x, s, lam, zl, zu, t_s, t_l, t_u, dp, dd):
    xl, xu = model.bounds(p)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    J = model.jacobian(p, x); H = model.hessian(p, x, lam)
    gf = model.gradient(p, x); g = model.constraints(p, x)
    r_d = gf - J.T @ lam - zl + zu
    sig_s, sig_x = kkt.sigmas(x, s, lam, zl, zu, xl, xu, il, iu, dd)
    K = kkt.condensed_matrix(H, J, sig_s, sig_x, dp)
    rhs = kkt.condensed_rhs(J, r_d, g, lam, sig_s, x, zl, zu, xl, xu, il, iu, t_s, t_l, t_u)
    dx = np.linalg.solve(K.toarray(), rhs)
    return (dx,) + kkt.recover(J, dx, g, g - s, lam, sig_s, x, zl, zu, xl, xu, il, iu,
                               t_s, t_l, t_u, dd)


@pytest.mark.parametrize("which", ["lp", "qp", "nlp", "halfbounds"])
def test_p5_condensed_equals_full_kkt(which):
    rng = np.random.default_rng(5)
    if which == "lp":
        p = w.random_lp(12, 7, 3, 11)
    elif which == "qp":
        p = w.qp_instance(14, 3)
    elif which == "nlp":
        p = w.nlp_grid(4, 4)
    else:
        p = w.random_lp(10, 6, 3, 12)
        p.xl = np.where(np.arange(10) % 3 == 0, -np.inf, 0.0)
        p.xu = np.where(np.arange(10) % 3 == 1, np.inf, 10.0)
    n, m = p.n, p.m
    xl, xu = model.bounds(p)
    lo = np.where(np.isfinite(xl), xl, -5.0); hi = np.where(np.isfinite(xu), xu, 5.0)
    x = lo + rng.uniform(0.2, 0.8, n) * (hi - lo)
    s = rng.uniform(0.5, 2.0, m); lam = rng.uniform(0.5, 2.0, m)
    zl = np.where(np.isfinite(xl), rng.uniform(0.5, 2, n), 0.0)
    zu = np.where(np.isfinite(xu), rng.uniform(0.5, 2, n), 0.0)
    t_s = rng.uniform(0, 0.3, m)
    t_l = np.where(np.isfinite(xl), rng.uniform(0, 0.3, n), 0.0)
    t_u = np.where(np.isfinite(xu), rng.uniform(0, 0.3, n), 0.0)
    for dp, dd in [(1e-8, 1e-8), (0.3, 0.2)]:
        a = _full_kkt_step(p, x, s, lam, zl, zu, t_s, t_l, t_u, dp, dd)
        b = _condensed_step(p, x, s, lam, zl, zu, t_s, t_l, t_u, dp, dd)
        for u, v in zip(a, b):
            assert np.max(np.abs(u - v)) <= 1e-10 * max(1.0, np.max(np.abs(u)))


@pytest.mark.parametrize("which", ["nlp", "qp"])
def test_p8_derivatives_finite_differences(which):
    p = w.nlp_grid(5, 6) if which == "nlp" else w.qp_instance(20, 4)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, p.n); lam = rng.uniform(0.1, 1, p.m)
    gf = model.gradient(p, x)
    J = model.jacobian(p, x).toarray()
    H = model.hessian(p, x, lam).toarray()
    for j in range(p.n):
        h = 1e-6 * max(1.0, abs(x[j]))
        e = np.zeros(p.n); e[j] = h
        fd_f = (model.objective(p, x + e) - model.objective(p, x - e)) / (2 * h)
        assert abs(fd_f - gf[j]) <= 1e-6 * max(1.0, abs(gf[j]))
        fd_g = (model.constraints(p, x + e) - model.constraints(p, x - e)) / (2 * h)
        assert np.max(np.abs(fd_g - J[:, j])) <= 1e-6 * max(1.0, np.max(np.abs(J[:, j])))
        lag = lambda xx: model.gradient(p, xx) - model.jacobian(p, xx).T @ lam
        fd_h = (lag(x + e) - lag(x - e)) / (2 * h)
        assert np.max(np.abs(fd_h - H[:, j])) <= 1e-6 * max(1.0, np.max(np.abs(H[:, j])))


def test_p8_grid_jacobian_exact_form():
    p = w.nlp_grid(6, 7)
    x = np.random.default_rng(1).uniform(-1, 1, p.n)
    J = model.jacobian(p, x).tocoo()
    assert np.allclose(J.data, -2.0 * x[J.col] / 5.0, rtol=0, atol=1e-15)


def _dual_step(p, x, s, lam, zl, zu, t_s, t_l, t_u, dp, dd):
    """Step through the dual condensed system (eq. kkt_dual), solved densely."""
    xl, xu = model.bounds(p)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    J = model.jacobian(p, x); H = model.hessian(p, x, lam)
    gf = model.gradient(p, x); g = model.constraints(p, x)
    r_d = gf - J.T @ lam - zl + zu
    _, sig_x = kkt.sigmas(x, s, lam, zl, zu, xl, xu, il, iu, dd)
    d = kkt.dual_scaling(H, sig_x, dp)
    M = kkt.dual_matrix(J, d, s, lam, dd)
    rt = kkt.reduced_dual_residual(r_d, x, zl, zu, xl, xu, il, iu, t_l, t_u)
    dlam = np.linalg.solve(M.toarray(), kkt.dual_rhs(J, d, rt, g, lam, t_s))
    dx = kkt.dual_dx(J, d, dlam, rt)
    ds = J @ dx + (g - s) + dd * dlam
    dzl, dzu = kkt.bound_steps(dx, x, zl, zu, xl, xu, il, iu, t_l, t_u)
    return dx, ds, dlam, dzl, dzu


def _random_point(p, rng):
    xl, xu = model.bounds(p)
    n, m = p.n, p.m
    lo = np.where(np.isfinite(xl), xl, -5.0); hi = np.where(np.isfinite(xu), xu, 5.0)
    x = lo + rng.uniform(0.2, 0.8, n) * (hi - lo)
    s = rng.uniform(0.5, 2.0, m); lam = rng.uniform(0.5, 2.0, m)
    zl = np.where(np.isfinite(xl), rng.uniform(0.5, 2, n), 0.0)
    zu = np.where(np.isfinite(xu), rng.uniform(0.5, 2, n), 0.0)
    t_s = rng.uniform(0, 0.3, m)
    t_l = np.where(np.isfinite(xl), rng.uniform(0, 0.3, n), 0.0)
    t_u = np.where(np.isfinite(xu), rng.uniform(0, 0.3, n), 0.0)
    return x, s, lam, zl, zu, t_s, t_l, t_u


@pytest.mark.parametrize("which", ["lp", "qp", "halfbounds", "more_rows"])
def test_p5_dual_condensed_equals_full_kkt(which):
    """eq. kkt_dual: the normal-equations step equals the Newton step of the
    full regularised system (dense partial-pivot LU) component by component."""
    rng = np.random.default_rng(8)
    if which == "lp":
        p = w.random_lp(12, 7, 3, 11)
    elif which == "qp":
        p = w.qp_instance(14, 3)
    elif which == "more_rows":
        p = w.random_lp(8, 13, 4, 19)
    else:
        p = w.random_lp(10, 6, 3, 12)
        p.xl = np.where(np.arange(10) % 3 == 0, -np.inf, 0.0)
        p.xu = np.where(np.arange(10) % 3 == 1, np.inf, 10.0)
    pt = _random_point(p, rng)
    for dp, dd in [(1e-8, 1e-8), (0.3, 0.2)]:
        a = _full_kkt_step(p, *pt, dp, dd)
        b = _dual_step(p, *pt, dp, dd)
        for u, v in zip(a, b):
            assert np.max(np.abs(u - v)) <= 1e-9 * max(1.0, np.max(np.abs(u)))


def test_dual_condensed_needs_a_diagonal_hessian():
    p = w.nlp_grid(4, 4)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.1, 0.5, p.n)
    with pytest.raises(kkt.NotDiagonal):
        kkt.dual_scaling(model.hessian(p, x, np.ones(p.m)), np.zeros(p.n), 1e-8)


@pytest.mark.parametrize("seed", [1, 2])
def test_dual_pattern_is_the_structure_of_j_jt(seed):
    p = w.random_lp(30, 18, 3, seed)
    J = model.jacobian(p, np.ones(p.n)).tocsr()
    adj = symbolic.dual_pattern(p.m, p.n, J.indptr, J.indices)
    B = (J.toarray() != 0).astype(int)
    S = (B @ B.T) > 0
    for v in range(p.m):
        assert adj[v] == [u for u in range(p.m) if S[v, u] and u != v]


def _augmented_step(p, x, s, lam, zl, zu, t_s, t_l, t_u, dp, dd):
    """Step through the augmented SQD system (eq. augmentedKKT), factored by
    the oracle's signed LDL' under its symbolic ordering."""
    xl, xu = model.bounds(p)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    J = model.jacobian(p, x).tocsr(); H = model.hessian(p, x, lam)
    gf = model.gradient(p, x); g = model.constraints(p, x)
    r_d = gf - J.T @ lam - zl + zu
    _, sig_x = kkt.sigmas(x, s, lam, zl, zu, xl, xu, il, iu, dd)
    A = kkt.augmented_matrix(H, J, s, lam, sig_x, dp, dd)
    Hl = sp.tril(H).tocsr()
    sym = symbolic.analyze(symbolic.augmented_pattern(p.n, p.m, J.indptr, J.indices, Hl.indptr, Hl.indices),
                           p.n + p.m)
    F = chol.SparseFactor(sym["perm"], sym["structs"]).factor_ldlt(A)
    rt = kkt.reduced_dual_residual(r_d, x, zl, zu, xl, xu, il, iu, t_l, t_u)
    dx, dlam = kkt.augmented_split(F.solve_ldlt(kkt.augmented_rhs(rt, g, lam, t_s)), p.n)
    ds = J @ dx + (g - s) + dd * dlam
    dzl, dzu = kkt.bound_steps(dx, x, zl, zu, xl, xu, il, iu, t_l, t_u)
    return dx, ds, dlam, dzl, dzu


@pytest.mark.parametrize("which", ["lp", "qp", "nlp", "halfbounds"])
def test_p5_augmented_equals_full_kkt(which):
    """eq. augmentedKKT through a signed LDL': the step equals the Newton
    step of the full regularised system (dense partial-pivot LU)."""
    rng = np.random.default_rng(9)
    if which == "lp":
        p = w.random_lp(12, 7, 3, 11)
    elif which == "qp":
        p = w.qp_instance(14, 3)
    elif which == "nlp":
        p = w.nlp_grid(4, 4)
    else:
        p = w.random_lp(10, 6, 3, 12)
        p.xl = np.where(np.arange(10) % 3 == 0, -np.inf, 0.0)
        p.xu = np.where(np.arange(10) % 3 == 1, np.inf, 10.0)
    pt = _random_point(p, rng)
    for dp, dd in [(1e-8, 1e-8), (0.3, 0.2)]:
        a = _full_kkt_step(p, *pt, dp, dd)
        b = _augmented_step(p, *pt, dp, dd)
        for u, v in zip(a, b):
            assert np.max(np.abs(u - v)) <= 1e-9 * max(1.0, np.max(np.abs(u)))


@pytest.mark.parametrize("seed", range(5))
def test_sqd_strong_factorisability_and_pivot_signs(seed):
    """Section 2: an SQD matrix [E A'; A -F] (E, F SPD) has P'KP = LDL' for
    every permutation P, and each pivot carries the sign of its block
    (positive for E's variables, negative for F's): inertia (n, m, 0).
    Checked under random permutations with the oracle's LDL' (dense
    structure, so any order is a valid symbolic structure); the factor
    reproduces P'KP to 1e-12."""
    rng = np.random.default_rng(seed)
    n, m = 9 + seed, 6 + seed
    Bn = rng.standard_normal((n, n)); E = Bn @ Bn.T / n + 0.1 * np.eye(n)
    Bm = rng.standard_normal((m, m)); F = Bm @ Bm.T / m + 0.1 * np.eye(m)
    A = rng.standard_normal((m, n))
    K = np.block([[E, A.T], [A, -F]])
    N = n + m
    structs = [np.arange(j + 1, N) for j in range(N)]
    sign = np.concatenate([np.ones(n), -np.ones(m)])
    for _ in range(6):
        perm = rng.permutation(N)
        Fc = chol.SparseFactor(perm, structs).factor_ldlt(sp.csr_matrix(K))
        assert np.array_equal(np.sign(Fc.D), sign[perm])
        Ld = Fc.to_dense()
        Kp = K[np.ix_(perm, perm)]
        assert np.linalg.norm(Kp - Ld @ np.diag(Fc.D) @ Ld.T) / np.linalg.norm(Kp) <= 1e-12
        b = rng.standard_normal(N)
        assert np.max(np.abs(K @ Fc.solve_ldlt(b) - b)) <= 1e-10 * np.max(np.abs(b)) * np.linalg.cond(K)


def test_augmented_pattern_is_the_structure_of_the_block_matrix():
    p = w.nlp_grid(5, 4)
    x = np.linspace(0.1, 0.9, p.n)
    J = model.jacobian(p, x).tocsr()
    Hl = sp.tril(model.hessian(p, x, np.ones(p.m))).tocsr()
    adj = symbolic.augmented_pattern(p.n, p.m, J.indptr, J.indices, Hl.indptr, Hl.indices)
    Jd = J.toarray() != 0
    Hd = (Hl + Hl.T).toarray() != 0
    S = np.block([[Hd, Jd.T], [Jd, np.zeros((p.m, p.m), bool)]])
    for v in range(p.n + p.m):
        assert adj[v] == [u for u in range(p.n + p.m) if S[v, u] and u != v]
