"""Scaled optimality measures of a primal-dual point (test infrastructure
only).  From the barrier KKT conditions (Section 3, eq. kkt) at mu = 0 with
bound multipliers:

  P = ||g - s||_inf / (1 + ||g||_inf)
  D = ||grad f - J'lambda - z_l + z_u||_inf / (1 + ||grad f||_inf)
  C = (s'lambda + (x-l)'z_l + (u-x)'z_u) / (1 + |f|)
"""
import numpy as np

from . import model


def _inf(v):
    return float(np.max(np.abs(v))) if len(v) else 0.0


def measures_from(f, gf, g, r_d, r_p, s, lam, x, zl, zu, xl, xu, il, iu):
    comp = (float(s @ lam) + float(((x - xl)[il] * zl[il]).sum())
            + float(((xu - x)[iu] * zu[iu]).sum()))
    P = _inf(r_p) / (1.0 + _inf(g))
    D = _inf(r_d) / (1.0 + _inf(gf))
    C = comp / (1.0 + abs(f))
    return P, D, C, comp


def check(problem, x, s, lam, zl, zu):
    """Recompute f, P, D, C and the true violations from a returned point."""
    xl, xu = model.bounds(problem)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    f = model.objective(problem, x)
    gf = model.gradient(problem, x)
    g = model.constraints(problem, x)
    J = model.jacobian(problem, x)
    zl = np.where(il, zl, 0.0)
    zu = np.where(iu, zu, 0.0)
    r_d = gf - J.T @ lam - zl + zu
    P, D, C, comp = measures_from(f, gf, g, r_d, g - s, s, lam, x, zl, zu, xl, xu, il, iu)
    viol = max(_inf(np.maximum(0.0, -g)),
               _inf(np.maximum(0.0, (xl - x)[il])), _inf(np.maximum(0.0, (x - xu)[iu])))
    return dict(f=f, P=P, D=D, C=C, violation=viol,
                min_s=float(np.min(s)) if len(s) else np.inf,
                min_lam=float(np.min(lam)) if len(lam) else np.inf)


def lp_qp_dual_objective(problem, x, lam, zl, zu):
    """Wolfe dual objective for f = c'x + 1/2 x'Qx, g = Ax - b (no W, q4):
    d = -1/2 x'Qx + b'lambda + l'z_l - u'z_u (finite bounds only).  Equal to
    f at a KKT point (duality invariant)."""
    xl, xu = model.bounds(problem)
    il, iu = np.isfinite(xl), np.isfinite(xu)
    Q = model.q_full(problem)
    return float(-0.5 * x @ (Q @ x) + problem.b @ lam + (xl * zl)[il].sum() - (xu * zu)[iu].sum())
