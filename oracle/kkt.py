"""Condensed KKT system of the pivoting-free IPM (test infrastructure only).

Section 3 (eq. kkt_system) gives the regularised Newton system in
(d_x, d_s, -d_lambda); eliminating d_s gives the augmented system
(eq. augmentedKKT) and eliminating d_lambda the primal condensed system
(eq. kkt_primal):  (H + delta_p I + J' (delta_d I + Lambda^{-1} S)^{-1} J) d_x
= -r.  The paper leaves the right-hand side unstated ("an appropriate
right-hand side"); with variable bounds and general complementarity
targets (t_s, t_l, t_u) the elimination gives

  Sigma_s = lambda / (s + delta_d lambda)        (= (delta_d I + S/Lambda)^-1)
  Sigma_x = z_l/(x - l) + z_u/(u - x)
  K       = H + diag(Sigma_x + delta_p) + J' diag(Sigma_s) J
  r~_d    = r_d - t_l/(x-l) + z_l + t_u/(u-x) - z_u
  rhs     = -r~_d - J' [Sigma_s (g - t_s/lambda)]
  d_lam   = Sigma_s (t_s/lambda - g - J d_x)
  d_s     = J d_x + r_p + delta_d d_lam
  d_zl    = t_l/(x-l) - z_l - (z_l/(x-l)) d_x
  d_zu    = t_u/(u-x) - z_u + (z_u/(u-x)) d_x
Bound terms only exist on finite bounds (masks il, iu).

Dual condensed system (eq. kkt_dual, the normal equations): when the (1,1)
block H + Sigma_x + delta_p I is diagonal (LP, QP with diagonal Q), it is
inverted, D = (H + Sigma_x + delta_p I)^-1, and the augmented system in
(d_x, d_lambda)
    (H + Sigma_x + delta_p I) d_x - J' d_lambda = -r~_d
    J d_x + (delta_d I + S/Lambda) d_lambda     = t_s/lambda - g
gives
  M        = delta_d I + S/Lambda + J D J'              (m x m, SPD)
  M d_lam  = t_s/lambda - g + J D r~_d
  d_x      = D (J' d_lam - r~_d)
  d_s      = J d_x + r_p + delta_d d_lam,  d_z as above.

Augmented system (eq. augmentedKKT) with the bound term folded into the
(1,1) block, in the unknowns (d_x, -d_lambda):
  [ H + Sigma_x + delta_p I    J'                   ] [ d_x      ]   [ -r~_d          ]
  [ J                          -(delta_d I + S/Lam) ] [ -d_lam   ] = [ t_s/lambda - g ]
For convex problems the matrix is symmetric quasi-definite (SQD): it has
P'AP = L D L' for every permutation P, with D positive on the x block and
negative on the lambda block (Section 2, strong factorisability).
"""
import numpy as np
import scipy.sparse as sp


def sigmas(x, s, lam, zl, zu, xl, xu, il, iu, delta_d):
    sig_s = lam / (s + delta_d * lam)
    sig_x = np.zeros_like(x)
    sig_x[il] += zl[il] / (x[il] - xl[il])
    sig_x[iu] += zu[iu] / (xu[iu] - x[iu])
    return sig_s, sig_x


def condensed_matrix(H, J, sig_s, sig_x, delta_p):
    n = H.shape[0]
    return (H + sp.diags(sig_x + delta_p) + J.T @ sp.diags(sig_s) @ J).tocsr()


def condensed_rhs(J, r_d, g, lam, sig_s, x, zl, zu, xl, xu, il, iu, t_s, t_l, t_u):
    rt = r_d.copy()
    rt[il] += -t_l[il] / (x[il] - xl[il]) + zl[il]
    rt[iu] += t_u[iu] / (xu[iu] - x[iu]) - zu[iu]
    return -rt - J.T @ (sig_s * (g - t_s / lam))


def bound_steps(dx, x, zl, zu, xl, xu, il, iu, t_l, t_u):
    dzl = np.zeros_like(x)
    dzu = np.zeros_like(x)
    dzl[il] = t_l[il] / (x[il] - xl[il]) - zl[il] - zl[il] / (x[il] - xl[il]) * dx[il]
    dzu[iu] = t_u[iu] / (xu[iu] - x[iu]) - zu[iu] + zu[iu] / (xu[iu] - x[iu]) * dx[iu]
    return dzl, dzu


def recover(J, dx, g, r_p, lam, sig_s, x, zl, zu, xl, xu, il, iu, t_s, t_l, t_u, delta_d):
    Jdx = J @ dx
    dlam = sig_s * (t_s / lam - g - Jdx)
    ds = Jdx + r_p + delta_d * dlam
    dzl, dzu = bound_steps(dx, x, zl, zu, xl, xu, il, iu, t_l, t_u)
    return ds, dlam, dzl, dzu


class NotDiagonal(ValueError):
    """The dual condensed system needs a diagonal (1,1) block."""


def dual_scaling(H, sig_x, delta_p):
    """D = (H + Sigma_x + delta_p I)^-1 for a diagonal H (NotDiagonal
    otherwise).  Entries that are not positive are returned as they are
    (1 / value): M is then not positive definite and its factorisation
    reports it."""
    Hc = H.tocsr()
    if (Hc - sp.diags(Hc.diagonal())).count_nonzero():
        raise NotDiagonal("the dual condensed system needs a diagonal Hessian")
    return 1.0 / (Hc.diagonal() + sig_x + delta_p)


def dual_matrix(J, d, s, lam, delta_d):
    """M = delta_d I + S/Lambda + J D J' (eq. kkt_dual)."""
    return (sp.diags(delta_d + s / lam) + J @ sp.diags(d) @ J.T).tocsr()


def reduced_dual_residual(r_d, x, zl, zu, xl, xu, il, iu, t_l, t_u):
    """r~_d: r_d with the bound complementarity targets folded in."""
    rt = r_d.copy()
    rt[il] += -t_l[il] / (x[il] - xl[il]) + zl[il]
    rt[iu] += t_u[iu] / (xu[iu] - x[iu]) - zu[iu]
    return rt


def dual_rhs(J, d, rt, g, lam, t_s):
    """Right-hand side of M d_lambda: t_s/lambda - g + J D r~_d."""
    return t_s / lam - g + J @ (d * rt)


def dual_dx(J, d, dlam, rt):
    """d_x = D (J' d_lambda - r~_d)."""
    return d * (J.T @ dlam - rt)


def augmented_matrix(H, J, s, lam, sig_x, delta_p, delta_d):
    """The SQD matrix of eq. augmentedKKT (x block first, then lambda)."""
    n, m = H.shape[0], J.shape[0]
    A11 = (H + sp.diags(sig_x + delta_p)).tocsr()
    A22 = sp.diags(-(delta_d + s / lam))
    return sp.bmat([[A11, J.T], [J, A22]], format="csr")


def augmented_rhs(rt, g, lam, t_s):
    """[-r~_d; t_s/lambda - g]."""
    return np.concatenate([-rt, t_s / lam - g])


def augmented_split(v, n):
    """(d_x, d_lambda) from the solution (d_x, -d_lambda)."""
    return v[:n], -v[n:]
