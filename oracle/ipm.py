"""Predictor-corrector primal-dual interior-point method (test
infrastructure only).

The paper describes the IPM only through its barrier KKT conditions
(Section 3, eq. kkt), the regularised Newton system (eq. kkt_system) and its
primal condensation (eq. kkt_primal), with fixed regularisation
delta_p = delta_d = 1e-8 as in the MadIPM options (Appendix, solver options)
and inertia correction on failure (Section 3, Regularization).  Every other
component is an elementwise map or a reduction (Section 1).  The iteration below is the
Mehrotra predictor-corrector scheme of the IPM literature the paper cites
(Nocedal & Wright), in this order:

 0 start: x from the bounds, s = max(g(x), 1), lambda = 1, z = 1
   (warm start: the supplied point pushed into the interior)
 1 evaluate f, grad f, g, J, H                            (model)
 2 r_d = grad f - J'lambda - z_l + z_u, r_p = g - s,
   mu = (s'lambda + (x-l)'z_l + (u-x)'z_u) / N_c
 3 stop when P, D, C <= tol (checker.measures)
 4 K = H + diag(Sigma_x + delta_p) + J' Sigma_s J           (kkt)
 5 factor K = LL' (inertia correction on a non-positive pivot)
 6-7 predictor: targets 0; affine step lengths; sigma = (mu_aff/mu)^3
 8 corrector: targets sigma mu - (second-order products)
 9 fraction to boundary tau = max(0.99, 1 - mu); LP: separate primal/dual
   steps, QP/NLP: the common minimum
10 NLP: backtracking on the residual norm phi
11 update
"""
import time

import numpy as np
import scipy.sparse as sp

from . import checker, kkt, model
from . import cholesky as chol
from . import symbolic

OK, MAX_ITER, TIME_LIMIT, STALLED = 0, 1, 2, 3
NUMERICAL = -4
STATUS_NAMES = {OK: "optimal", MAX_ITER: "max_iter", TIME_LIMIT: "time_limit",
                STALLED: "stalled", NUMERICAL: "numerical"}


class Factorizer:
    """Dense (small order) or sparse (fixed symbolic structure) Cholesky of
    the condensed matrix; pattern() gives the adjacency lists of its
    structure, used for the symbolic analysis of the sparse path."""

    def __init__(self, order, pattern, dense_max=1500):
        self.n = order
        self.dense = self.n <= dense_max
        self.count = 0
        if not self.dense:
            self.sym = symbolic.analyze(pattern(), self.n)

    def factor(self, K):
        self.count += 1
        if self.dense:
            self.L = chol.dense_cholesky(K.toarray())
        else:
            self.F = chol.SparseFactor(self.sym["perm"], self.sym["structs"]).factor(K)

    def solve(self, b):
        if self.dense:
            return chol.dense_solve(self.L, b)
        return self.F.solve(b)


def initial_point(xl, xu):
    x = np.zeros_like(xl)
    fl, fu = np.isfinite(xl), np.isfinite(xu)
    both = fl & fu
    x[both] = 0.5 * (xl[both] + xu[both])
    x[fl & ~fu] = xl[fl & ~fu] + 1.0
    x[~fl & fu] = xu[~fl & fu] - 1.0
    return x


def push_start(problem, x_hat, lam_hat, xl, xu):
    """Interior push of a predicted point (bound-push rule of Waechter and
    Biegler, cited in the paper's Section 3)."""
    x = np.array(x_hat, dtype=float, copy=True)
    fl, fu = np.isfinite(xl), np.isfinite(xu)
    width = np.where(fl & fu, xu - xl, np.inf)
    pl = np.minimum(1e-2 * np.maximum(1.0, np.abs(np.where(fl, xl, 0))), 1e-2 * width)
    pu = np.minimum(1e-2 * np.maximum(1.0, np.abs(np.where(fu, xu, 0))), 1e-2 * width)
    x = np.where(fl, np.maximum(x, xl + pl), x)
    x = np.where(fu, np.minimum(x, xu - pu), x)
    g = model.constraints(problem, x)
    s = np.maximum(g, 1e-2 * np.maximum(1.0, np.abs(g)))
    lam = np.maximum(np.asarray(lam_hat, dtype=float), 1e-2)
    mu_w = max(1e-4, float(s @ lam) / max(1, problem.m))
    zl = np.where(fl, mu_w / np.where(fl, x - xl, 1.0), 0.0)
    zu = np.where(fu, mu_w / np.where(fu, xu - x, 1.0), 0.0)
    return x, s, lam, zl, zu


def _max_step(v, dv):
    neg = dv < 0
    if not np.any(neg):
        return np.inf
    return float(np.min(-v[neg] / dv[neg]))


def solve(problem, tol=1e-6, max_iter=500, delta_p=1e-8, delta_d=1e-8,
          max_wall_time=900.0, start=None, dense_max=1500, log=None,
          force_inertia=False, form="primal"):
    """Returns a dict: status, iterations, f, P, D, C, x, s, lam, zl, zu,
    history (per-iteration mu, alphas, invariants) and factorizations.

    form "primal" solves each Newton step through the primal condensed
    system (eq. kkt_primal), "dual" through the dual condensed system
    (eq. kkt_dual, the normal equations; needs a diagonal Hessian),
    "augmented" through the SQD augmented system (eq. augmentedKKT) with a
    signed LDL' factorisation.  The inertia correction of step 5 applies to
    the primal form; in the other forms a factorisation failure (or, in the
    augmented form, a pivot whose sign is not its block's) ends the solve
    with status NUMERICAL."""
    if form not in ("primal", "dual", "augmented"):
        raise ValueError(form)
    t0 = time.time()
    n, m = problem.n, problem.m
    xl, xu = model.bounds(problem)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    nc = m + int(il.sum()) + int(iu.sum())
    kind = model.kind(problem)
    if start is None:
        x = initial_point(xl, xu)
        s = np.maximum(model.constraints(problem, x), 1.0)
        lam = np.ones(m)
        zl = np.where(il, 1.0, 0.0)
        zu = np.where(iu, 1.0, 0.0)
    else:
        x, s, lam, zl, zu = push_start(problem, start[0], start[1], xl, xu)
    fac = None
    delta_w_last = 0.0
    hist = []
    status = MAX_ITER
    it = 0
    while True:
        f = model.objective(problem, x)
        gf = model.gradient(problem, x)
        g = model.constraints(problem, x)
        J = model.jacobian(problem, x)
        H = model.hessian(problem, x, lam)
        r_d = gf - J.T @ lam - zl + zu
        r_p = g - s
        P, D, C, comp = checker.measures_from(f, gf, g, r_d, r_p, s, lam, x, zl, zu, xl, xu, il, iu)
        mu = comp / nc if nc else 0.0
        if log:
            log(f"it {it:3d} f {f:+.10e} P {P:.2e} D {D:.2e} C {C:.2e} mu {mu:.2e}")
        if P <= tol and D <= tol and C <= tol:
            status = OK
            break
        if it >= max_iter:
            status = MAX_ITER
            break
        if time.time() - t0 > max_wall_time:
            status = TIME_LIMIT
            break
        if fac is None:
            # symbolic analysis once, on the fixed patterns of J and H
            j_rp, j_ci = model.jacobian_pattern(problem)
            h_rp, h_ci = model.hessian_lower_pattern(problem)
            if form == "augmented":
                aug_sym = symbolic.analyze(symbolic.augmented_pattern(n, m, j_rp, j_ci, h_rp, h_ci), n + m)
                fac = chol.SparseFactor(aug_sym["perm"], aug_sym["structs"])
                fac.count = 0
                block_sign = np.concatenate([np.ones(n), -np.ones(m)])[aug_sym["perm"]]
            elif form == "dual":
                fac = Factorizer(m, lambda: symbolic.dual_pattern(m, n, j_rp, j_ci), dense_max)
            else:
                fac = Factorizer(n, lambda: symbolic.kkt_pattern(n, j_rp, j_ci, h_rp, h_ci), dense_max)
        sig_s, sig_x = kkt.sigmas(x, s, lam, zl, zu, xl, xu, il, iu, delta_d)
        delta_w = 0.0
        if form == "augmented":
            # eq. augmentedKKT: signed LDL' of the SQD matrix
            fac.count += 1
            try:
                fac.factor_ldlt(kkt.augmented_matrix(H, J, s, lam, sig_x, delta_p, delta_d))
            except chol.SingularPivot:
                status = NUMERICAL
                break
            if np.any(np.sign(fac.D) != block_sign):
                status = NUMERICAL
                break

            def direction(t_s, t_l, t_u):
                rt = kkt.reduced_dual_residual(r_d, x, zl, zu, xl, xu, il, iu, t_l, t_u)
                dx, dlam = kkt.augmented_split(fac.solve_ldlt(kkt.augmented_rhs(rt, g, lam, t_s)), n)
                ds = J @ dx + r_p + delta_d * dlam
                dzl, dzu = kkt.bound_steps(dx, x, zl, zu, xl, xu, il, iu, t_l, t_u)
                return dx, ds, dlam, dzl, dzu
        elif form == "dual":
            # eq. kkt_dual: factor M, d_lambda from M, then d_x
            dD = kkt.dual_scaling(H, sig_x, delta_p)
            try:
                fac.factor(kkt.dual_matrix(J, dD, s, lam, delta_d))
            except chol.NotPositiveDefinite:
                status = NUMERICAL
                break

            def direction(t_s, t_l, t_u):
                rt = kkt.reduced_dual_residual(r_d, x, zl, zu, xl, xu, il, iu, t_l, t_u)
                dlam = fac.solve(kkt.dual_rhs(J, dD, rt, g, lam, t_s))
                dx = kkt.dual_dx(J, dD, dlam, rt)
                ds = J @ dx + r_p + delta_d * dlam
                dzl, dzu = kkt.bound_steps(dx, x, zl, zu, xl, xu, il, iu, t_l, t_u)
                return dx, ds, dlam, dzl, dzu
        else:
            # eq. kkt_primal; step 5: inertia correction on failure
            K = kkt.condensed_matrix(H, J, sig_s, sig_x, delta_p)
            try:
                if force_inertia:
                    raise chol.NotPositiveDefinite(0)
                fac.factor(K)
            except chol.NotPositiveDefinite:
                delta_w = 1e-4 if delta_w_last == 0.0 else max(1e-20, delta_w_last / 3.0)
                first = delta_w_last == 0.0
                while True:
                    try:
                        fac.factor(K + delta_w * sp.eye(n))
                        delta_w_last = delta_w
                        break
                    except chol.NotPositiveDefinite:
                        delta_w *= 100.0 if first else 8.0
                        if delta_w > 1e40:
                            status = NUMERICAL
                            break
                if status == NUMERICAL:
                    break

            def direction(t_s, t_l, t_u):
                rhs = kkt.condensed_rhs(J, r_d, g, lam, sig_s, x, zl, zu, xl, xu, il, iu, t_s, t_l, t_u)
                dx = fac.solve(rhs)
                ds, dlam, dzl, dzu = kkt.recover(J, dx, g, r_p, lam, sig_s, x, zl, zu, xl, xu, il, iu,
                                                 t_s, t_l, t_u, delta_d)
                return dx, ds, dlam, dzl, dzu

        def step_limits(dx, ds, dlam, dzl, dzu):
            ap = min(_max_step(s, ds), _max_step((x - xl)[il], dx[il]),
                     _max_step((xu - x)[iu], -dx[iu]))
            ad = min(_max_step(lam, dlam), _max_step(zl[il], dzl[il]), _max_step(zu[iu], dzu[iu]))
            return ap, ad

        zero_m, zero_n = np.zeros(m), np.zeros(n)
        dxa, dsa, dla, dzla, dzua = direction(zero_m, zero_n, zero_n)
        apa, ada = step_limits(dxa, dsa, dla, dzla, dzua)
        apa, ada = min(1.0, apa), min(1.0, ada)
        if kind != "lp":
            apa = ada = min(apa, ada)
        mu_aff = (float((s + apa * dsa) @ (lam + ada * dla))
                  + float(((x - xl + apa * dxa)[il] * (zl + ada * dzla)[il]).sum())
                  + float(((xu - x - apa * dxa)[iu] * (zu + ada * dzua)[iu]).sum())) / nc
        sigma = min(1.0, (mu_aff / mu) ** 3) if mu > 0 else 0.0
        smu = sigma * mu
        t_s = smu - dsa * dla
        t_l = np.where(il, smu - dxa * dzla, 0.0)
        t_u = np.where(iu, smu + dxa * dzua, 0.0)
        dx, ds, dlam, dzl, dzu = direction(t_s, t_l, t_u)
        ap_max, ad_max = step_limits(dx, ds, dlam, dzl, dzu)
        tau = max(0.99, 1.0 - mu)
        ap, ad = min(1.0, tau * ap_max), min(1.0, tau * ad_max)
        if kind != "lp":
            ap = ad = min(ap, ad)
        if kind == "nlp":
            def phi(xx, ss, ll, zzl, zzu):
                gg = model.constraints(problem, xx)
                rd = model.gradient(problem, xx) - model.jacobian(problem, xx).T @ ll - zzl + zzu
                parts = [rd, gg - ss, ss * ll - smu, (xx - xl)[il] * zzl[il] - smu,
                         (xu - xx)[iu] * zzu[iu] - smu]
                return float(np.sqrt(sum(float(p @ p) for p in parts)))
            phi0 = phi(x, s, lam, zl, zu)
            a = ap
            ok = False
            for _ in range(31):
                if phi(x + a * dx, s + a * ds, lam + a * dlam, zl + a * dzl, zu + a * dzu) \
                        <= (1.0 - 1e-4 * a) * phi0:
                    ok = True
                    break
                a *= 0.5
            if not ok:
                status = STALLED
                break
            ap = ad = a
        x = x + ap * dx
        s = s + ap * ds
        lam = lam + ad * dlam
        zl = zl + ad * dzl
        zu = zu + ad * dzu
        hist.append(dict(mu=mu, sigma=sigma, alpha_p=ap, alpha_d=ad, delta_w=delta_w,
                         min_s=float(s.min()) if m else np.inf,
                         min_lam=float(lam.min()) if m else np.inf,
                         min_z=float(min(zl[il].min() if il.any() else np.inf,
                                         zu[iu].min() if iu.any() else np.inf)),
                         min_xl=float((x - xl)[il].min()) if il.any() else np.inf,
                         min_xu=float((xu - x)[iu].min()) if iu.any() else np.inf))
        it += 1
    f = model.objective(problem, x)
    return dict(status=status, iterations=it, f=f, P=P, D=D, C=C, x=x, s=s, lam=lam,
                zl=zl, zu=zu, history=hist, factorizations=fac.count if fac else 0,
                time=time.time() - t0)
