"""Plain FP64 CPU oracle for the FETI dual operator and its consumers.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  Every function follows
the paper's definitions directly with dense LAPACK factorisations; there is
no blocking, sparsity exploitation or reordering beyond what those library
routines do internally.  Precision: float64 throughout (the paper states no
precision; FP64 is the FETI norm).

Notation (paper Sec. II): K_i subdomain stiffness, K_i^+ = K_reg,i^{-1}
(Sec. III), B~_i the rows of B that touch subdomain i (one +-1 per row),
D_i the dual-index map of subdomain i (local multiplier -> global), R_i the
kernel basis, F = B K^+ B^T, G = B R, d = B K^+ f - c, e = R^T f,
P = I - G (G^T G)^{-1} G^T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


# --------------------------------------------------------------------------
# generalised inverse through the regularised matrix (Sec. III)
# --------------------------------------------------------------------------


class RegInverse:
    """K_reg^{-1} applied through a dense Cholesky factor (LAPACK potrf),
    with one step of iterative refinement whose residual is formed in
    extended precision, so the solve error is near FP64 rounding."""

    def __init__(self, Kreg):
        self.K = sp.csr_matrix(Kreg)
        self.Kl = self.K.astype(np.longdouble)
        self.cf = sla.cho_factor(self.K.toarray(), lower=True, check_finite=False)

    def solve(self, rhs, refine=True):
        rhs = np.asarray(rhs, dtype=np.float64)
        x = sla.cho_solve(self.cf, rhs, check_finite=False)
        if refine:
            r = rhs.astype(np.longdouble) - self.Kl @ x.astype(np.longdouble)
            x = x + sla.cho_solve(self.cf, np.asarray(r, dtype=np.float64),
                                  check_finite=False)
        return x


def Bt_dense(n, b_dof, b_sign):
    """B~_i^T as a dense n x m matrix: column j is sign_j * e_{dof_j}."""
    m = len(b_dof)
    Bt = np.zeros((n, m))
    Bt[np.asarray(b_dof), np.arange(m)] = np.asarray(b_sign, dtype=np.float64)
    return Bt


def local_dual_operator(Kreg, b_dof, b_sign, inv=None):
    """F~_i = B~_i K_reg,i^{-1} B~_i^T  (eq. localdualoperator with K^+ =
    K_reg^{-1}).  Computed as Z = K_reg^{-1} B~^T, F = B~ Z, then the two
    triangles are averaged (F is symmetric in exact arithmetic)."""
    inv = inv or RegInverse(Kreg)
    n = Kreg.shape[0]
    Z = inv.solve(Bt_dense(n, b_dof, b_sign))
    F = np.asarray(b_sign, dtype=np.float64)[:, None] * Z[np.asarray(b_dof), :]
    return 0.5 * (F + F.T)


# --------------------------------------------------------------------------
# application of F (eqs. dualop_apply_impl / dualop_apply_expl)
# --------------------------------------------------------------------------


def apply_explicit(F_list, dual_maps, lam, n_lambda):
    """q = sum_i D_i^T F~_i (D_i lam): scatter, dense matvec, gather."""
    q = np.zeros(n_lambda)
    for F, D in zip(F_list, dual_maps):
        np.add.at(q, D, F @ lam[D])
    return q


def apply_implicit(invs, subs, lam, n_lambda):
    """q = sum_i D_i^T B~_i K_reg,i^{-1} B~_i^T D_i lam, right to left."""
    q = np.zeros(n_lambda)
    for inv, s in zip(invs, subs):
        p = lam[s.dual_map]
        v = np.zeros(s.n)
        np.add.at(v, s.b_dof, s.b_sign * p)
        u = inv.solve(v)
        np.add.at(q, s.dual_map, s.b_sign * u[s.b_dof])
    return q


# --------------------------------------------------------------------------
# coarse space, projector, PCPG (Sec. II, Alg. 1)
# --------------------------------------------------------------------------


def G_matrix(prob):
    """G = B R, dense n_lambda x (sum_i dim Ker K_i); block i is D_i^T B~_i R_i."""
    nk = [s.R.shape[1] for s in prob.subs]
    G = np.zeros((prob.n_lambda, sum(nk)))
    col = 0
    for s, k in zip(prob.subs, nk):
        G[s.dual_map, col:col + k] += s.b_sign[:, None] * s.R[s.b_dof, :]
        col += k
    return G


def lumped_preconditioner(prob):
    """The lumped preconditioner of Alg. 1, M = sum_i D_i^T B~_i K_i B~_i^T D_i,
    with K_i taken as the regularised stiffness K_reg,i the solver works with.
    Returns a function w -> M w."""
    blocks = []
    for s in prob.subs:
        Bt = Bt_dense(s.n, s.b_dof, s.b_sign)
        blocks.append((s.dual_map, Bt.T @ (s.Kreg @ Bt)))

    def apply(w):
        y = np.zeros(prob.n_lambda)
        for dmap, Mi in blocks:
            y[dmap] += Mi @ w[dmap]
        return y

    return apply


def scaled_jump_operator(prob, scaling="stiffness", K="K"):
    """The scaled jump operator B_D = (B W B^T)^{-1} B W (dense, n_lambda x
    sum n_i, subdomain blocks side by side) with W diagonal per subdomain
    DOF: 1 / K_i[d, d] (stiffness scaling) or 1 (multiplicity scaling).
    Alg. 1 leaves M open; with the non-redundant chain gluing a node shared
    by k subdomains carries k - 1 multipliers, so weights applied row by row
    cannot satisfy B_D B^T = I there, while this B_D does for any diagonal
    W > 0 (B has full row rank).  Also returns B."""
    nn = [s.n for s in prob.subs]
    off = np.concatenate([[0], np.cumsum(nn)])
    B = np.zeros((prob.n_lambda, off[-1]))
    wv = np.zeros(off[-1])
    for i, sub in enumerate(prob.subs):
        B[sub.dual_map, off[i] + sub.b_dof] = sub.b_sign
        Ki = sub.K if K == "K" else sub.Kreg
        wv[off[i]:off[i + 1]] = 1.0 / Ki.diagonal() if scaling == "stiffness" else 1.0
    A = (B * wv[None, :]) @ B.T
    return np.linalg.solve(A, B * wv[None, :]), B


def scaled_lumped_preconditioner(prob, scaling="stiffness", K="K"):
    """The lumped preconditioner with the scaled jump operator,
    M = B_D blockdiag(K_i) B_D^T (B_D from scaled_jump_operator; K_i the
    unregularised stiffness, or K_reg,i).  Returns a function w -> M w."""
    BD, _ = scaled_jump_operator(prob, scaling, K)
    Kb = sp.block_diag([(sub.K if K == "K" else sub.Kreg) for sub in prob.subs], format="csr")
    M = BD @ (Kb @ BD.T)

    def apply(w):
        return M @ w

    return apply


def e_vector(prob):
    """e = R^T f."""
    return np.concatenate([s.R.T @ s.f for s in prob.subs])


def d_vector(prob, invs):
    """d = B K^+ f - c."""
    d = -prob.c.copy()
    for inv, s in zip(invs, prob.subs):
        u = inv.solve(s.f)
        np.add.at(d, s.dual_map, s.b_sign * u[s.b_dof])
    return d


class Projector:
    """P x = x - G (G^T G)^{-1} G^T x, with (G^T G) factored densely."""

    def __init__(self, G):
        self.G = G
        self.cf = sla.cho_factor(G.T @ G, lower=True)

    def coarse_solve(self, y):
        return sla.cho_solve(self.cf, y)

    def __call__(self, x):
        return x - self.G @ self.coarse_solve(self.G.T @ x)


def pcpg(apply_F, d, G, e, tol=1e-9, maxit=1000, M=None, fixed_iters=None):
    """Preconditioned conjugate projected gradient, Alg. 1.

    lambda_I = G (G^T G)^{-1} e (so G^T lambda_I = e); M = identity unless
    given.  Stops when ||w_k|| <= tol ||w_0||, or after exactly fixed_iters
    iterations if that is given.  Returns (lambda, iterations, history of
    ||w_k||/||w_0||)."""
    P = Projector(G)
    Mop = M or (lambda x: x)
    lam = G @ P.coarse_solve(e)
    r = d - apply_F(lam)
    w = P(r)
    y = P(Mop(w))
    p = y.copy()
    wy = w @ y
    w0 = np.linalg.norm(w)
    hist = [1.0]
    k = 0
    while True:
        if fixed_iters is not None:
            if k >= fixed_iters:
                break
        elif hist[-1] <= tol or k >= maxit:
            break
        q = apply_F(p)
        delta = wy / (p @ q)
        lam = lam + delta * p
        r = r - delta * q
        w = P(r)
        y = P(Mop(w))
        wy_new = w @ y
        beta = wy_new / wy
        wy = wy_new
        p = y + beta * p
        k += 1
        hist.append(np.linalg.norm(w) / w0 if w0 > 0 else 0.0)
    return lam, k, np.array(hist)


def alpha_from_lambda(G, d, Flam):
    """alpha = -(G^T G)^{-1} G^T (d - F lambda)  (eq. alphacompute)."""
    P = Projector(G)
    return -P.coarse_solve(G.T @ (d - Flam))


def primal_solution(prob, invs, lam, alpha):
    """u_i = K_i^+ (f_i - B~_i^T lambda_i) + R_i alpha_i  (eq. solutionUeval)."""
    us = []
    col = 0
    for inv, s in zip(invs, prob.subs):
        k = s.R.shape[1]
        v = s.f.copy()
        np.add.at(v, s.b_dof, -s.b_sign * lam[s.dual_map])
        us.append(inv.solve(v) + s.R @ alpha[col:col + k])
        col += k
    return us


# --------------------------------------------------------------------------
# derivatives of J = mu^T F(theta) lambda
# --------------------------------------------------------------------------


def primal_from_dual(inv, sub, x):
    """u_x,i = K_reg,i^{-1} B~_i^T D_i x."""
    v = np.zeros(sub.n)
    np.add.at(v, sub.b_dof, sub.b_sign * x[sub.dual_map])
    return inv.solve(v)


def grad_theta(inv, sub, mu, lam):
    """dJ/dtheta_e for the elements of one subdomain.

    With K_reg(theta) = sum_e theta_e K_e0 + rho Rt Rt^T (rho frozen),
    dF/dtheta_e = -B K^{-1} K_e0 K^{-1} B^T, so
    dJ/dtheta_e = -u_mu|_e^T K_e0 u_lam|_e  (K_e0: the element's own
    unit-coefficient matrix)."""
    um = primal_from_dual(inv, sub, mu)
    ul = primal_from_dual(inv, sub, lam)
    ed = sub.elem_dofs()
    Ke = np.broadcast_to(sub.elem_matrices(), (ed.shape[0],) + sub.Ke_ref.shape[-2:])
    return -np.einsum("ea,eab,eb->e", um[ed], Ke, ul[ed])
