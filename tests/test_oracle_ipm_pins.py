"""Pins of the oracle's interior-point solver against results the
mathematics fixes independently of it (test infrastructure).

P1 vertex enumeration of tiny LPs (an LP optimum is attained at a vertex)
P1b LP optima against an independent LP solver (HiGHS through scipy), at
    sizes past enumeration, including the block-angular structure
P2 closed-form QP optima (separable box QP; one-constraint diagonal QP)
P2b QP optima against scipy's trust-region constrained method, with Q
    written out in the test (diagonal instances of the batch workload and a
    grid-Laplacian Q)
P3 NLP special cases (c = 0 gives x* = 0; small c leaves constraints
   inactive so x* solves x^3 + c + Lx = 0)
P3b NLP optima with active quadratic constraints against scipy's trust-region
    constrained method, objective and constraints written out in the test
P7 duality gap and interior invariants along the iteration
"""
import itertools

import numpy as np
import pytest

from oracle import checker, ipm, model
from paper_2508_16094_amd import workloads as w


def _vertex_enumeration_lp(p):
    """min c'x over {Ax >= b, l <= x <= u} by enumerating every basis."""
    A = p.A.to_scipy().toarray()
    n = p.n
    G = np.vstack([A, np.eye(n), -np.eye(n)])
    h = np.concatenate([p.b, p.xl, -p.xu])
    best = np.inf
    for rows in itertools.combinations(range(G.shape[0]), n):
        M = G[list(rows)]
        if abs(np.linalg.det(M)) < 1e-10:
            continue
        x = np.linalg.solve(M, h[list(rows)])
        if np.all(G @ x >= h - 1e-9):
            best = min(best, float(p.c @ x))
    return best


@pytest.mark.parametrize("form", ["primal", "dual", "augmented"])
@pytest.mark.parametrize("seed", range(6))
def test_p1_tiny_lp_vertex_enumeration(seed, form):
    n, m = 4 + seed % 3, 3 + seed % 4
    p = w.random_lp(n, m, min(3, m), 777 + seed)
    f_star = _vertex_enumeration_lp(p)
    r = ipm.solve(p, tol=1e-10, form=form)
    assert r["status"] == ipm.OK
    assert abs(r["f"] - f_star) <= 1e-7 * max(1.0, abs(f_star))


def _highs_lp(p):
    """min c'x over {Ax >= b, l <= x <= u} by HiGHS (scipy's linprog)."""
    from scipy.optimize import linprog
    r = linprog(p.c, A_ub=-p.A.to_scipy(), b_ub=-p.b, bounds=list(zip(p.xl, p.xu)), method="highs")
    assert r.status == 0, r.message
    return float(r.fun)


_P1B_CASES = ([("random", s) for s in range(3)] + [("block", s) for s in range(2)]
              + [("one_sided", s) for s in range(3)])


@pytest.mark.parametrize("form", ["primal", "dual", "augmented"])
@pytest.mark.parametrize("case", _P1B_CASES, ids=[f"{k}{s}" for k, s in _P1B_CASES])
def test_p1b_lp_against_highs(case, form):
    kind, seed = case
    if kind == "random":
        p = w.random_lp(60, 25, 4, 900 + seed)
    elif kind == "one_sided":   # every other variable has no upper bound (and a cost >= 0)
        p = w.random_lp(60, 25, 4, 950 + seed)
        up_free = np.arange(p.n) % 2 == 0
        p.xu = np.where(up_free, np.inf, p.xu)
        p.c = np.where(up_free, np.abs(p.c), p.c)
    else:   # 4 blocks of 10 x 20 with 3 linking rows, the benchmark LP's shape
        p = w.lp_block(4, 10, 20, nnz_per_col=3, n_link_rows=3, link_nnz=3, link_cols_per_block=5,
                       instance=seed)
    f_star = _highs_lp(p)
    r = ipm.solve(p, tol=1e-10, form=form)
    assert r["status"] == ipm.OK
    assert abs(r["f"] - f_star) <= 1e-8 * max(1.0, abs(f_star))


def _trust_constr_qp(p, Q):
    """min c'x + x'Qx/2 over {Ax >= b, l <= x <= u} by scipy's trust-region
    constrained method, Q dense."""
    from scipy.optimize import Bounds, LinearConstraint, minimize
    A = p.A.to_scipy().toarray()
    x0 = (p.xl + np.minimum(p.xu, p.xl + 1.0)) / 2
    r = minimize(lambda x: p.c @ x + 0.5 * x @ Q @ x, x0, jac=lambda x: p.c + Q @ x, hess=lambda x: Q,
                 method="trust-constr", constraints=[LinearConstraint(A, p.b, np.inf)],
                 bounds=Bounds(p.xl, p.xu), options={"gtol": 1e-12, "xtol": 1e-14, "maxiter": 5000})
    assert r.status in (1, 2), r.message
    return float(r.fun)


def _grid_q_dense(nx, ny, shift):
    """4-neighbour grid Laplacian plus shift I, entry by entry (node (i, j) is
    i ny + j)."""
    n = nx * ny
    Q = np.zeros((n, n))
    for i in range(nx):
        for j in range(ny):
            k = i * ny + j
            Q[k, k] = shift
            for a, b in ((i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)):
                if 0 <= a < nx and 0 <= b < ny:
                    Q[k, k] += 1.0
                    Q[k, a * ny + b] = -1.0
    return Q


@pytest.mark.parametrize("case", ["diag0", "diag1", "diag2", "grid"])
def test_p2b_qp_against_trust_constr(case):
    if case == "grid":
        p = w.random_lp(30, 15, 3, 4242)
        p.Q = w.grid_laplacian_lower(5, 6, shift=0.5)
        Q = _grid_q_dense(5, 6, 0.5)
        forms = ["primal", "augmented"]          # the dual system needs a diagonal Hessian
    else:
        p = w.qp_instance(30, int(case[-1]))
        assert np.array_equal(p.Q.colind, np.arange(30))
        Q = np.diag(p.Q.val)
        forms = ["primal", "dual", "augmented"]
    f_star = _trust_constr_qp(p, Q)
    for form in forms:
        r = ipm.solve(p, tol=1e-10, form=form)
        assert r["status"] == ipm.OK, form
        assert abs(r["f"] - f_star) <= 1e-7 * max(1.0, abs(f_star)), form


def _grid_stencil_rows(nx, ny):
    """Rows of the grid NLP's constraint weights: for every node (i, j) with
    i + j even, 1/5 on the node and its in-grid 4-neighbours."""
    rows = []
    for i in range(nx):
        for j in range(ny):
            if (i + j) % 2 == 0:
                rows.append([a * ny + b for a, b in ((i, j), (i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1))
                             if 0 <= a < nx and 0 <= b < ny])
    S = np.zeros((len(rows), nx * ny))
    for k, r in enumerate(rows):
        S[k, r] = 0.2
    return S


@pytest.mark.parametrize("form", ["primal", "augmented"])
@pytest.mark.parametrize("nx,ny,scale,inst", [(5, 6, 4.0, 0), (5, 6, 4.0, 1), (6, 6, 6.0, 2)])
def test_p3b_nlp_active_constraints_against_trust_constr(nx, ny, scale, inst, form):
    """min sum(x^4/4 + c x) + x'Lx/2 s.t. 1 - S (x o x) >= 0, with c scaled so
    that some constraints are active at the optimum."""
    from scipy.optimize import NonlinearConstraint, minimize
    p = w.nlp_grid(nx, ny, inst)
    p.c = p.c * scale
    L = _grid_q_dense(nx, ny, 0.0)
    S = _grid_stencil_rows(nx, ny)
    con = NonlinearConstraint(lambda x: 1 - S @ (x * x), 0, np.inf, jac=lambda x: -2 * S * x[None, :],
                              hess=lambda x, v: -2 * np.diag(S.T @ v))
    ref = minimize(lambda x: np.sum(x ** 4) / 4 + p.c @ x + 0.5 * x @ L @ x, np.zeros(nx * ny),
                   jac=lambda x: p.c + x ** 3 + L @ x, hess=lambda x: L + np.diag(3 * x ** 2),
                   method="trust-constr", constraints=[con], options={"gtol": 1e-12, "xtol": 1e-14, "maxiter": 5000})
    assert ref.status in (1, 2), ref.message
    assert np.sum(1 - S @ (ref.x * ref.x) < 1e-6) >= 2      # constraints active at the optimum
    r = ipm.solve(p, tol=1e-10, form=form)
    assert r["status"] == ipm.OK
    assert abs(r["f"] - ref.fun) <= 1e-7 * max(1.0, abs(ref.fun))


class _P:
    pass


def _box_qp(n, seed, with_constraint):
    rng = np.random.default_rng(seed)
    p = _P()
    p.n = n
    q = rng.uniform(0.5, 2.0, n)
    p.c = rng.standard_normal(n) * 3
    p.Q = w.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), q)
    p.q4 = None
    p.W = None
    p.xl = rng.uniform(-2, 0, n)
    p.xu = p.xl + rng.uniform(0.5, 3.0, n)
    if with_constraint:
        a = rng.uniform(0.2, 1.0, n)
        p.m = 1
        p.A = w.CSR(1, n, np.array([0, n], dtype=np.int64), np.arange(n, dtype=np.int32), a)
        x_free = np.clip(-p.c / q, p.xl, p.xu)
        # choose beta so that the constraint is active at the optimum
        beta = float(a @ x_free) + 0.3 * float(a @ (p.xu - x_free))
        p.b = np.array([beta])
    else:
        p.m = 0
        p.A = None
        p.b = np.zeros(0)
    return p, q


@pytest.mark.parametrize("seed", range(4))
def test_p2_separable_box_qp_closed_form(seed):
    p, q = _box_qp(12, 100 + seed, False)
    x_star = np.clip(-p.c / q, p.xl, p.xu)
    r = ipm.solve(p, tol=1e-10)
    assert r["status"] == ipm.OK
    assert np.max(np.abs(r["x"] - x_star)) <= 1e-6


@pytest.mark.parametrize("form", ["primal", "dual", "augmented"])
@pytest.mark.parametrize("seed", range(4))
def test_p2_one_constraint_qp_bisection(seed, form):
    p, q = _box_qp(15, 200 + seed, True)
    a = p.A.val
    beta = p.b[0]

    def x_of(nu):
        return np.clip((a * nu - p.c) / q, p.xl, p.xu)

    lo, hi = 0.0, 1.0
    while a @ x_of(hi) < beta:
        hi *= 2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if a @ x_of(mid) < beta:
            lo = mid
        else:
            hi = mid
    nu = 0.5 * (lo + hi)
    x_star = x_of(nu)
    r = ipm.solve(p, tol=1e-10, form=form)
    assert r["status"] == ipm.OK
    assert np.max(np.abs(r["x"] - x_star)) <= 1e-6
    assert abs(r["lam"][0] - nu) <= 1e-5 * max(1.0, nu)


def test_p3_nlp_zero_linear_term():
    p = w.nlp_grid(12, 12)
    p.c = np.zeros(p.n)
    r = ipm.solve(p, tol=1e-10)
    assert r["status"] == ipm.OK
    assert np.max(np.abs(r["x"])) <= 1e-5
    assert abs(r["f"]) <= 1e-9
    assert np.max(np.abs(r["lam"])) <= 1e-6


def test_p3_nlp_inactive_constraints_newton_root():
    p = w.nlp_grid(14, 10)
    p.c = 1e-2 * p.c
    L = model.q_full(p)
    # independent damped Newton on x^3 + c + Lx = 0
    x = np.zeros(p.n)
    for _ in range(100):
        F = x ** 3 + p.c + L @ x
        Jm = (L + np.diag(3 * x ** 2)) if False else (L.toarray() + np.diag(3 * x ** 2))
        dx = np.linalg.solve(Jm, -F)
        x = x + dx
        if np.max(np.abs(dx)) < 1e-15:
            break
    assert np.all(model.constraints(p, x) > 0)
    r = ipm.solve(p, tol=1e-10)
    assert r["status"] == ipm.OK
    assert np.max(np.abs(r["x"] - x)) <= 1e-6


@pytest.mark.parametrize("maker", ["lp", "qp"])
def test_p7_duality_and_invariants(maker):
    p = w.lp_small() if maker == "lp" else w.qp_instance(200, 5)
    r = ipm.solve(p, tol=1e-9)
    assert r["status"] == ipm.OK
    d = checker.lp_qp_dual_objective(p, r["x"], r["lam"], r["zl"], r["zu"])
    assert abs(r["f"] - d) <= 1e-7 * (1 + abs(r["f"]))
    for h in r["history"]:
        assert h["min_s"] > 0 and h["min_lam"] > 0 and h["min_z"] > 0
        assert h["min_xl"] > 0 and h["min_xu"] > 0
    chk = checker.check(p, r["x"], r["s"], r["lam"], r["zl"], r["zu"])
    assert chk["P"] <= 1e-9 and chk["D"] <= 1e-9 and chk["C"] <= 1e-9


def test_p7_fraction_to_boundary():
    """s_new >= (1 - tau) s_old componentwise, tau >= 0.99."""
    p = w.lp_small(1)
    r = ipm.solve(p, tol=1e-8)
    assert r["status"] == ipm.OK
    assert all(0 < h["alpha_p"] <= 1 and 0 < h["alpha_d"] <= 1 for h in r["history"])


def test_inertia_correction_path_forced():
    """A forced non-positive pivot runs the regularisation loop and the
    solve still converges (delta_w enlarges K's diagonal)."""
    p = w.qp_instance(120, 2)
    r = ipm.solve(p, tol=1e-8, force_inertia=True)
    assert r["status"] == ipm.OK
    assert all(h["delta_w"] > 0 for h in r["history"])


def test_max_iter_status():
    r = ipm.solve(w.lp_small(), max_iter=2)
    assert r["status"] == ipm.MAX_ITER and r["iterations"] == 2


def test_warm_start_from_solution_converges_fast():
    p = w.qp_instance(200, 7)
    cold = ipm.solve(p, tol=1e-8)
    warm = ipm.solve(p, tol=1e-8, start=(cold["x"], cold["lam"]))
    assert warm["status"] == ipm.OK
    assert abs(warm["f"] - cold["f"]) <= 1e-6 * (1 + abs(cold["f"]))
    assert warm["iterations"] <= cold["iterations"]


def _push_case(m_rows=True):
    """3 variables: x0 in [0, 10], x1 in [0, 1], x2 <= 100 (no lower bound);
    rows g1 = x0 + x1 - 0.5, g2 = -x2 + 90 (none when m_rows is False)."""
    xl = np.array([0.0, 0.0, -np.inf])
    xu = np.array([10.0, 1.0, 100.0])
    if m_rows:
        A = w.csr_from_coo(2, 3, [0, 0, 1], [0, 1, 2], [1.0, 1.0, -1.0])
        b = np.array([0.5, -90.0])
    else:
        A, b = None, np.zeros(0)
    return w.Problem(n=3, m=2 if m_rows else 0, c=np.zeros(3), b=b, A=A, xl=xl, xu=xu)


def test_push_start_hand_computed():
    """Bound push of a predicted point, values worked out by hand:
    x0 = -5 -> 0 + min(1e-2 max(1, 0), 1e-2 * 10) = 0.01;
    x1 = 0.9999 -> 1 - min(1e-2 max(1, 1), 1e-2 * 1) = 0.99;
    x2 = 150 -> 100 - 1e-2 max(1, 100) = 99 (no lower bound, width infinite);
    g = (0.01 + 0.99 - 0.5, -99 + 90) = (0.5, -9);
    s = max(g, 1e-2 max(1, |g|)) = (0.5, 0.09); lambda = max((1e-3, 2e-3), 1e-2) = (0.01, 0.01);
    mu_w = max(1e-4, s'lambda / m) = (0.005 + 0.0009) / 2 = 0.00295;
    z_l = mu_w / (x - l) = (0.295, 0.00295 / 0.99, 0); z_u = mu_w / (u - x) = (0.00295 / 9.99, 0.295, 0.00295)."""
    p = _push_case()
    xl, xu = model.bounds(p)
    x, s, lam, zl, zu = ipm.push_start(p, np.array([-5.0, 0.9999, 150.0]), np.array([1e-3, 2e-3]), xl, xu)
    mu_w = 0.00295
    np.testing.assert_allclose(x, [0.01, 0.99, 99.0], rtol=1e-14)
    np.testing.assert_allclose(s, [0.5, 0.09], rtol=1e-12)
    np.testing.assert_allclose(lam, [0.01, 0.01], rtol=1e-15)
    np.testing.assert_allclose(zl, [0.295, mu_w / 0.99, 0.0], rtol=1e-12)
    np.testing.assert_allclose(zu, [mu_w / 9.99, 0.295, mu_w], rtol=1e-12)


def test_push_start_floor_without_rows():
    """With no rows s'lambda / max(1, m) = 0, so mu_w is its floor 1e-4:
    interior x = (5, 0.5, 3) stays, z_l = (1e-4/5, 1e-4/0.5, 0),
    z_u = (1e-4/5, 1e-4/0.5, 1e-4/97)."""
    p = _push_case(m_rows=False)
    xl, xu = model.bounds(p)
    x, s, lam, zl, zu = ipm.push_start(p, np.array([5.0, 0.5, 3.0]), np.zeros(0), xl, xu)
    np.testing.assert_allclose(x, [5.0, 0.5, 3.0], rtol=0)
    assert s.size == 0 and lam.size == 0
    np.testing.assert_allclose(zl, [2e-5, 2e-4, 0.0], rtol=1e-14)
    np.testing.assert_allclose(zu, [2e-5, 2e-4, 1e-4 / 97.0], rtol=1e-14)


@pytest.mark.parametrize("maker", [lambda: w.lp_small(2), lambda: w.qp_instance(300, 5),
                                   lambda: w.lp_block(nblocks=3, block_rows=150, block_cols=300,
                                                      link_cols_per_block=10)])
def test_dual_form_invariants_and_same_optimum(maker):
    """P7 for the dual form: interior iterates, fraction to the boundary and
    the LP/QP dual objective; its optimum is the primal form's."""
    p = maker()
    r = ipm.solve(p, tol=1e-9, form="dual", dense_max=0)
    ref = ipm.solve(p, tol=1e-9)
    assert r["status"] == ipm.OK and ref["status"] == ipm.OK
    assert abs(r["f"] - ref["f"]) <= 1e-7 * max(1.0, abs(ref["f"]))
    for h in r["history"]:
        assert h["min_s"] > 0 and h["min_lam"] > 0 and h["min_z"] > 0
    chk = checker.check(p, r["x"], r["s"], r["lam"], r["zl"], r["zu"])
    assert max(chk["P"], chk["D"], chk["C"]) <= 1e-9


def test_nonconvex_grid_reaches_a_local_minimiser():
    """Nonconvex grid NLP (mixed-sign stencil weights): the oracle needs the
    inertia correction, ends at a KKT point with active constraints, and
    that point satisfies the second-order condition of a local minimiser:
    the Lagrangian Hessian on the null space of the active constraints'
    gradients is positive definite (strict complementarity holds: every
    active multiplier is bounded away from zero)."""
    import scipy.linalg
    p = w.nlp_grid_nonconvex(20, 20, 0, 0.5, 0.2, 5.0)
    r = ipm.solve(p, tol=1e-10)
    assert r["status"] == ipm.OK
    assert sum(1 for h in r["history"] if h["delta_w"] > 0) > 0
    chk = checker.check(p, r["x"], r["s"], r["lam"], r["zl"], r["zu"])
    assert max(chk["P"], chk["D"], chk["C"]) <= 1e-9
    active = r["lam"] > 1e-6
    assert active.sum() > 0 and np.min(r["lam"][active]) > 1e-3
    JA = model.jacobian(p, r["x"]).toarray()[active]
    Z = scipy.linalg.null_space(JA)
    Hr = Z.T @ model.hessian(p, r["x"], r["lam"]).toarray() @ Z
    assert np.min(np.linalg.eigvalsh(0.5 * (Hr + Hr.T))) > 1e-6
    # and the Hessian itself is indefinite somewhere on the path (at the
    # start x = 0, lambda = 1), which is why the correction was needed
    H0 = model.hessian(p, np.zeros(p.n), np.ones(p.m)).toarray()
    assert np.min(np.linalg.eigvalsh(H0)) < 0


@pytest.mark.parametrize("maker", [lambda: w.nlp_grid(24, 20), lambda: w.qp_param(12, 15).base,
                                   lambda: w.lp_block(nblocks=3, block_rows=150, block_cols=300,
                                                      link_cols_per_block=10)])
def test_augmented_form_same_optimum(maker):
    """The augmented SQD form reaches the primal form's optimum (NLP and a
    QP with a non-diagonal Hessian included) with interior iterates."""
    p = maker()
    r = ipm.solve(p, tol=1e-9, form="augmented")
    ref = ipm.solve(p, tol=1e-9)
    assert r["status"] == ipm.OK and ref["status"] == ipm.OK
    assert abs(r["f"] - ref["f"]) <= 1e-7 * max(1.0, abs(ref["f"]))
    for h in r["history"]:
        assert h["min_lam"] > 0 and h["min_s"] > 0


def test_augmented_form_stops_on_an_indefinite_hessian():
    """A nonconvex Hessian breaks the SQD structure: a pivot takes the wrong
    sign and the augmented form ends with NUMERICAL (the paper's reason to
    use the primal condensed form with inertia correction there)."""
    r = ipm.solve(w.nlp_grid_nonconvex(20, 20, 0, 0.5, 0.2, 5.0), tol=1e-9, form="augmented")
    assert r["status"] == ipm.NUMERICAL
