"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
a brute-force dense inverse, the Moore-Penrose route, the global FEM solve the
torn system is equivalent to (Sec. II, eq. femsystem vs eq. fetisystem),
central finite differences, and exact identities.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth import make_problem, config_problem, element_matrix, simplex_element_matrix, kuhn_simplices
from synth.problems import assemble_stiffness, regularise
from oracle import feti
from oracle import implicit as orc_impl


# ---------------------------------------------------------------- helpers

def dense_B(sub):
    B = np.zeros((sub.m, sub.n))
    for j in range(sub.m):
        B[j, sub.b_dof[j]] = sub.b_sign[j]
    return B


def global_fem_solve(prob):
    """Direct solve of the untorn FEM system with Dirichlet dofs eliminated."""
    dpn = prob.dpn
    nn = int(np.prod([e + 1 for e in prob.n_elems]))
    N = nn * dpn
    rows, cols, vals = [], [], []
    f = np.zeros(N)
    for s in prob.subs:
        g = (s.gnode[:, None] * dpn + np.arange(dpn)[None, :]).ravel()
        K = s.K.tocoo()
        rows.append(g[K.row]); cols.append(g[K.col]); vals.append(K.data)
        np.add.at(f, g, s.f)
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    coords = np.stack(np.unravel_index(np.arange(nn), [e + 1 for e in prob.n_elems][::-1])[::-1],
                      axis=-1)
    fixed = np.zeros(N, dtype=bool)
    if prob.dirichlet_axis is not None:
        fixed = np.repeat(coords[:, prob.dirichlet_axis] == 0, dpn)
    free = ~fixed
    u = np.zeros(N)
    u[free] = spla.spsolve(K[free][:, free].tocsc(), f[free])
    return u


def solve_feti(prob, tol=1e-12):
    invs = [feti.RegInverse(s.Kreg) for s in prob.subs]
    Fs = [feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign, inv)
          for s, inv in zip(prob.subs, invs)]
    Ds = [s.dual_map for s in prob.subs]
    applyF = lambda x: feti.apply_explicit(Fs, Ds, x, prob.n_lambda)
    G = feti.G_matrix(prob)
    e = feti.e_vector(prob)
    d = feti.d_vector(prob, invs)
    lam, it, hist = feti.pcpg(applyF, d, G, e, tol=tol, maxit=5000)
    alpha = feti.alpha_from_lambda(G, d, applyF(lam))
    us = feti.primal_solution(prob, invs, lam, alpha)
    return dict(invs=invs, Fs=Fs, G=G, e=e, d=d, lam=lam, it=it, alpha=alpha, us=us,
                applyF=applyF)


def tiny(kind, seed=7):
    if kind == "heat2d":
        return make_problem(2, "heat", [[3, 4], [4, 3]], 0.5, dirichlet_axis=0, seed=seed)
    if kind == "heat3d":
        return make_problem(3, "heat", [[3, 2], [2, 3], [3, 2]], 0.5, dirichlet_axis=2, seed=seed)
    if kind == "elast3d":
        return make_problem(3, "elasticity", [[2, 3], [2, 2], [3, 2]], 0.3, dirichlet_axis=2,
                            seed=seed)
    if kind == "elast2d":
        return make_problem(2, "elasticity", [[3, 2, 3], [3, 2]], 0.3, dirichlet_axis=0,
                            seed=seed)
    # linear simplices on the same kind of grids (the paper's element type)
    if kind == "heat2d_tri":
        return make_problem(2, "heat", [[3, 4], [4, 3]], 0.5, dirichlet_axis=0, seed=seed,
                            elem="simplex")
    if kind == "heat3d_tet":
        return make_problem(3, "heat", [[3, 2], [2, 3], [2, 2]], 0.5, dirichlet_axis=2, seed=seed,
                            elem="simplex")
    if kind == "elast3d_tet":
        return make_problem(3, "elasticity", [[2, 2], [2, 2], [2, 2]], 0.3, dirichlet_axis=2,
                            seed=seed, elem="simplex")
    raise ValueError(kind)


KINDS = ["heat2d", "heat3d", "elast3d", "elast2d", "heat2d_tri", "heat3d_tet", "elast3d_tet"]


# ---------------------------------------------------------------- element matrices

def test_element_matrices_closed_form():
    K2 = element_matrix(2, "heat")
    # bilinear unit square: 2/3 on the diagonal, -1/6 along edges, -1/3 across
    assert np.allclose(np.diag(K2), 2 / 3)
    assert np.isclose(K2[0, 1], -1 / 6) and np.isclose(K2[0, 2], -1 / 6)
    assert np.isclose(K2[0, 3], -1 / 3)
    K3 = element_matrix(3, "heat", h=0.25)
    # trilinear cube of edge h: h/3 diagonal, 0 along edges, -h/12 face and body diagonals
    assert np.allclose(np.diag(K3), 0.25 / 3)
    assert np.isclose(K3[0, 1], 0.0, atol=1e-15)
    assert np.isclose(K3[0, 3], -0.25 / 12) and np.isclose(K3[0, 7], -0.25 / 12)
    for K in (K2, K3):
        assert np.allclose(K.sum(axis=1), 0.0, atol=1e-15)
    Ke = element_matrix(3, "elasticity", h=1.0, E=1.0, nu=0.3)
    assert np.allclose(Ke, Ke.T)
    ev = np.linalg.eigvalsh(Ke)
    assert np.sum(ev < 1e-10) == 6  # six rigid-body modes
    # rigid-body modes of one cube are in its null space
    corners = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], float)
    for t in np.eye(3):
        assert np.allclose(Ke @ np.tile(t, 8), 0, atol=1e-14)
    rot = np.zeros(24)
    rot[0::3] = -corners[:, 1]
    rot[1::3] = corners[:, 0]
    assert np.allclose(Ke @ rot, 0, atol=1e-14)


def test_simplex_element_matrices_closed_form():
    """Linear simplices of the Kuhn subdivision: the barycentric gradients of
    (0,0),(1,0),(1,1) are (-1,0),(1,-1),(0,1) (area 1/2), those of
    (0,0,0),(1,0,0),(1,1,0),(1,1,1) are -e_x, e_x-e_y, e_y-e_z, e_z (volume
    1/6): tridiagonal [1,-1; -1,2,-1; ...; -1,1] scaled by the measure."""
    T2 = np.array([[1, -1, 0], [-1, 2, -1], [0, -1, 1]], float) / 2
    assert np.allclose(simplex_element_matrix(2, "heat", kuhn_simplices(2)[0]), T2)
    T3 = np.array([[1, -1, 0, 0], [-1, 2, -1, 0], [0, -1, 2, -1], [0, 0, -1, 1]], float) / 6
    for v in kuhn_simplices(3):       # every Kuhn simplex, vertices in Kuhn order
        assert np.allclose(simplex_element_matrix(3, "heat", v, h=0.5), 0.5 * T3)
    # the six tetrahedra tile the cube: a linear field a.x has energy |a|^2 h^3
    h = 0.25
    a = np.array([0.3, -1.1, 0.7])
    cube = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)])
    E = 0.0
    for v in kuhn_simplices(3):
        u = (v * h) @ a
        E += u @ simplex_element_matrix(3, "heat", v, h=h) @ u
    assert np.isclose(E, a @ a * h ** 3)
    assert len(kuhn_simplices(3)) == 6 and {tuple(c) for v in kuhn_simplices(3) for c in v} <= {tuple(c) for c in cube}
    # elasticity: rigid motions in the kernel (rank 12 - 6), and a uniform
    # strain eps has energy eps:D:eps times the volume
    for v in kuhn_simplices(3):
        Ke = simplex_element_matrix(3, "elasticity", v, h=1.0, E=1.0, nu=0.3)
        assert np.allclose(Ke, Ke.T)
        assert np.sum(np.linalg.eigvalsh(Ke) < 1e-12) == 6
    nu, Ey = 0.3, 1.0
    lam_, mu_ = Ey * nu / ((1 + nu) * (1 - 2 * nu)), Ey / (2 * (1 + nu))
    Gd = np.array([[0.2, 0.1, 0.0], [0.1, -0.3, 0.05], [0.0, 0.05, 0.4]])  # symmetric displacement gradient
    Etot = 0.0
    for v in kuhn_simplices(3):
        u = (v.astype(float) @ Gd.T).ravel()
        Etot += u @ simplex_element_matrix(3, "elasticity", v, h=1.0, E=Ey, nu=nu) @ u
    eps_energy = lam_ * np.trace(Gd) ** 2 + 2 * mu_ * np.sum(Gd * Gd)
    assert np.isclose(Etot, eps_energy)


# ---------------------------------------------------------------- 1D closed form

@pytest.mark.parametrize("nsub,nel", [(2, 5), (3, 4)])
def test_local_dual_operator_1d_closed_form(nsub, nel):
    """1D bar, nodes 0..n, unit conductivity, edge h, K_reg = K + rho e0 e0^T:
    (K_reg^{-1})_{ij} = 1/rho + h*min(i,j).  With the chain gluing and the
    Dirichlet row at x=0 this fixes every F~_i entry."""
    P = make_problem(1, "heat", [[nel] * nsub], 0.0, dirichlet_axis=0, seed=1)
    h = P.h
    for s in P.subs:
        rho = s.rho
        Ginv = lambda i, j: 1.0 / rho + h * min(i, j)
        expect = np.array([[s.b_sign[a] * s.b_sign[b] * Ginv(s.b_dof[a], s.b_dof[b])
                            for b in range(s.m)] for a in range(s.m)])
        F = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)
        assert np.allclose(F, expect, rtol=1e-14, atol=0)
    # explicit structure of the first two subdomains
    s0, s1 = P.subs[0], P.subs[1]
    F0 = feti.local_dual_operator(s0.Kreg, s0.b_dof, s0.b_sign)
    r = 1.0 / s0.rho
    assert np.allclose(F0, [[r, r], [r, r + nel * h]], rtol=1e-14)
    F1 = feti.local_dual_operator(s1.Kreg, s1.b_dof, s1.b_sign)
    r1 = 1.0 / s1.rho
    if nsub == 2:
        assert np.allclose(F1, [[r1]], rtol=1e-14)
    else:  # middle subdomain: -1 at its left end, +1 at its right end
        assert np.allclose(F1, [[r1, -r1], [-r1, r1 + nel * h]], rtol=1e-14)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("kind", KINDS)
def test_local_dual_operator_brute_force(kind):
    P = tiny(kind)
    for s in P.subs:
        F = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)
        B = dense_B(s)
        Fb = B @ np.linalg.inv(s.Kreg.toarray()) @ B.T
        assert np.allclose(F, Fb, rtol=0, atol=1e-11 * np.abs(Fb).max())
        assert np.array_equal(F, F.T)
        ev = np.linalg.eigvalsh(F)
        assert ev.min() >= -1e-12 * ev.max()


@pytest.mark.parametrize("kind", KINDS)
def test_generalized_inverse(kind):
    """K K_reg^{-1} K = K (the defining property of K^+, Sec. II)."""
    P = tiny(kind)
    for s in P.subs:
        K = s.K.toarray()
        X = feti.RegInverse(s.Kreg).solve(K)
        assert np.linalg.norm(K @ X - K) <= 1e-12 * np.linalg.norm(K)


@pytest.mark.parametrize("kind", KINDS)
def test_projected_operator_matches_moore_penrose(kind):
    """P F P does not depend on the generalised inverse: it equals the value
    obtained with the Moore-Penrose pseudo-inverse of K."""
    P = tiny(kind)
    G = feti.G_matrix(P)
    Pr = feti.Projector(G)
    nl = P.n_lambda
    F = np.zeros((nl, nl))
    Fmp = np.zeros((nl, nl))
    for s in P.subs:
        Fi = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)
        F[np.ix_(s.dual_map, s.dual_map)] += Fi
        B = dense_B(s)
        Fmp[np.ix_(s.dual_map, s.dual_map)] += B @ np.linalg.pinv(s.K.toarray(), rcond=1e-12,
                                                                 hermitian=True) @ B.T
    PF = np.stack([Pr(Pr(F[:, j])) for j in range(nl)], 1)
    PF = np.stack([Pr(PF[i, :]) for i in range(nl)], 0)
    PM = np.stack([Pr(Fmp[:, j]) for j in range(nl)], 1)
    PM = np.stack([Pr(PM[i, :]) for i in range(nl)], 0)
    assert np.abs(PF - PM).max() <= 1e-9 * np.abs(PM).max()


def test_F_additivity_and_apply_routes():
    """sum_i D_i^T F~_i D_i equals B K^+ B^T assembled globally (Sec. II-A),
    and explicit application equals the implicit right-to-left one (Sec. III)."""
    P = tiny("heat3d")
    nl = P.n_lambda
    Fsum = np.zeros((nl, nl))
    Bg = np.zeros((nl, sum(s.n for s in P.subs)))
    Kinv = []
    off = 0
    for s in P.subs:
        Fsum[np.ix_(s.dual_map, s.dual_map)] += feti.local_dual_operator(
            s.Kreg, s.b_dof, s.b_sign)
        Bg[s.dual_map, off + s.b_dof] = s.b_sign
        Kinv.append(np.linalg.inv(s.Kreg.toarray()))
        off += s.n
    from scipy.linalg import block_diag
    Fglob = Bg @ block_diag(*Kinv) @ Bg.T
    assert np.abs(Fsum - Fglob).max() <= 1e-11 * np.abs(Fglob).max()
    invs = [feti.RegInverse(s.Kreg) for s in P.subs]
    Fs = [feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign, i) for s, i in zip(P.subs, invs)]
    qe = feti.apply_explicit(Fs, [s.dual_map for s in P.subs], P.lam, nl)
    qi = feti.apply_implicit(invs, P.subs, P.lam, nl)
    assert np.abs(qe - qi).max() <= 1e-13 * np.abs(qi).max()
    assert np.allclose(qe, Fglob @ P.lam, rtol=0, atol=1e-11 * np.abs(qe).max())


# ---------------------------------------------------------------- whole FETI

@pytest.mark.parametrize("kind", ["C1", "heat3d", "elast3d", "elast2d", "heat2d_tri", "heat3d_tet",
                                  "elast3d_tet"])
def test_feti_solution_equals_global_fem(kind):
    """The torn system is equivalent to the FEM system: PCPG (Alg. 1) + alpha
    (eq. alphacompute) + u recovery (eq. solutionUeval) reproduce the global
    direct solve, and the constraints G^T lambda = e, B u = c hold."""
    P = config_problem(1) if kind == "C1" else tiny(kind)
    r = solve_feti(P, tol=1e-13)
    ug = global_fem_solve(P)
    dpn = P.dpn
    err = 0.0
    for s, u in zip(P.subs, r["us"]):
        g = (s.gnode[:, None] * dpn + np.arange(dpn)[None, :]).ravel()
        err = max(err, np.abs(u - ug[g]).max())
    assert err <= 1e-8 * np.abs(ug).max()
    assert np.abs(r["G"].T @ r["lam"] - r["e"]).max() <= 1e-10 * max(1, np.abs(r["e"]).max())
    Bu = np.zeros(P.n_lambda)
    for s, u in zip(P.subs, r["us"]):
        np.add.at(Bu, s.dual_map, s.b_sign * u[s.b_dof])
    assert np.abs(Bu - P.c).max() <= 1e-8 * np.abs(ug).max()


def test_pcpg_fixed_iterations_and_lambda_uniqueness():
    """lambda does not depend on rho (a different valid generalised inverse)."""
    P = tiny("heat2d")
    r1 = solve_feti(P)
    for s in P.subs:
        s.Kreg = regularise(s.K, s.R, s.fix_dofs, 7.5 * s.rho)
    r2 = solve_feti(P)
    assert np.abs(r1["lam"] - r2["lam"]).max() <= 1e-8 * np.abs(r1["lam"]).max()
    # fixed iteration count is honoured
    lam, it, hist = feti.pcpg(r1["applyF"], r1["d"], r1["G"], r1["e"], fixed_iters=3)
    assert it == 3 and len(hist) == 4


# ---------------------------------------------------------------- derivatives

def _J(sub, theta, mu, lam):
    K = assemble_stiffness(sub, theta)
    Kr = regularise(K, sub.R, sub.fix_dofs, sub.rho)
    F = feti.local_dual_operator(Kr, sub.b_dof, sub.b_sign)
    return mu[sub.dual_map] @ F @ lam[sub.dual_map]


@pytest.mark.parametrize("elem,physics", [("box", "heat"), ("simplex", "heat"), ("simplex", "elasticity")])
def test_gradient_central_differences(elem, physics):
    w = [[3, 3]] * 3 if physics == "heat" else [[2, 2]] * 3
    P = make_problem(3, physics, w, 0.3, dirichlet_axis=2, seed=11, elem=elem)
    rng = np.random.default_rng(0)
    eps = np.finfo(float).eps
    for s in P.subs[:3]:
        inv = feti.RegInverse(s.Kreg)
        g = feti.grad_theta(inv, s, P.mu, P.lam)
        J0 = abs(_J(s, s.theta, P.mu, P.lam))
        for e in rng.choice(len(s.theta), 6, replace=False):
            h = 1e-6
            tp = s.theta.copy(); tp[e] += h
            tm = s.theta.copy(); tm[e] -= h
            fd = (_J(s, tp, P.mu, P.lam) - _J(s, tm, P.mu, P.lam)) / (2 * h)
            # truncation O(h^2) plus the rounding of the two J values (eps |J| / h)
            assert abs(fd - g[e]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()) + 50 * eps * J0 / h


def test_gradient_euler_identity():
    """P F P is homogeneous of degree -1 in theta (heat), so with projected
    mu, lambda: sum_e theta_e dJ/dtheta_e = -J exactly."""
    P = make_problem(3, "heat", [[3, 2], [2, 3], [2, 2]], 0.3, dirichlet_axis=2, seed=5)
    Pr = feti.Projector(feti.G_matrix(P))
    mu, lam = Pr(P.mu), Pr(P.lam)
    J, S = 0.0, 0.0
    for s in P.subs:
        inv = feti.RegInverse(s.Kreg)
        F = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign, inv)
        J += mu[s.dual_map] @ F @ lam[s.dual_map]
        S += s.theta @ feti.grad_theta(inv, s, mu, lam)
    assert abs(S + J) <= 1e-10 * abs(J)


# ---------------------------------------------------------------- C oracle

@pytest.mark.parametrize("kind", ["heat3d", "elast3d"])
def test_c_implicit_apply_matches_python_oracle(kind):
    P = tiny(kind)
    invs = [feti.RegInverse(s.Kreg) for s in P.subs]
    q = feti.apply_implicit(invs, P.subs, P.lam, P.n_lambda)
    for perms in (None, [np.arange(s.n, dtype=np.int32) for s in P.subs]):
        I = orc_impl.ImplicitCPU(P.subs, P.n_lambda, nthreads=3, perms=perms)
        I.factor()
        qc = I.apply(P.lam)
        assert np.abs(qc - q).max() <= 1e-11 * np.abs(q).max()


@pytest.mark.parametrize("kind", ["heat2d", "elast3d"])
def test_lumped_preconditioner_matches_global_product(kind):
    """The oracle's lumped preconditioner, assembled subdomain by subdomain
    through the dual maps, equals the global product B blockdiag(K_reg,i) B^T
    built from one sparse B over all subdomain DOFs (an independent route:
    every row of B carries the +-1 of each subdomain it glues); it is
    symmetric positive semi-definite."""
    P = tiny(kind)
    from oracle.feti import lumped_preconditioner
    offs = np.cumsum([0] + [s.n for s in P.subs])
    rows, cols, vals = [], [], []
    for i, s in enumerate(P.subs):
        rows += list(s.dual_map)
        cols += list(offs[i] + np.asarray(s.b_dof))
        vals += list(np.asarray(s.b_sign, dtype=float))
    B = sp.csr_matrix((vals, (rows, cols)), shape=(P.n_lambda, offs[-1]))
    K = sp.block_diag([s.Kreg for s in P.subs], format="csr")
    Mg = (B @ K @ B.T).toarray()
    Mo = lumped_preconditioner(P)
    I = np.eye(P.n_lambda)
    Mcols = np.column_stack([Mo(I[:, k]) for k in range(P.n_lambda)])
    assert np.allclose(Mcols, Mg, rtol=1e-13, atol=1e-13 * np.abs(Mg).max())
    assert np.allclose(Mcols, Mcols.T, atol=1e-13 * np.abs(Mg).max())
    assert np.linalg.eigvalsh(0.5 * (Mcols + Mcols.T)).min() >= -1e-10 * np.abs(Mg).max()


@pytest.mark.parametrize("kind", ["heat3d", "elast3d", "heat3d_tet"])
def test_c_explicit_assembly_matches_python_oracle(kind):
    """The C oracle's explicit F~_i (one unit solve per column with its own
    sparse factor) equals the dense-LAPACK F~_i; its dense explicit apply
    equals the Python explicit apply and the implicit one."""
    P = tiny(kind)
    I = orc_impl.ImplicitCPU(P.subs, P.n_lambda, nthreads=3)
    I.factor()
    I.assemble()
    Fs = []
    for i, s in enumerate(P.subs):
        F = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)
        Fc = I.dual_operator(i)
        assert np.abs(Fc - F).max() <= 1e-12 * np.abs(F).max()
        Fs.append(F)
    q = feti.apply_explicit(Fs, [s.dual_map for s in P.subs], P.lam, P.n_lambda)
    qe = I.apply_explicit(P.lam)
    qi = I.apply(P.lam)
    assert np.abs(qe - q).max() <= 1e-12 * np.abs(q).max()
    assert np.abs(qi - q).max() <= 1e-12 * np.abs(q).max()


def test_c_explicit_assembly_1d_closed_form():
    """The C oracle's explicit F~_i of the 1D bar equal (K_reg^{-1})_{ij} =
    1/rho + h min(i, j) entry by entry (m = 2 and m = 1 subdomains)."""
    P = make_problem(1, "heat", [[6, 6]], 0.0, dirichlet_axis=0, seed=1)
    I = orc_impl.ImplicitCPU(P.subs, P.n_lambda, nthreads=2)
    I.factor()
    I.assemble()
    s0, s1 = P.subs
    r0, r1 = 1.0 / s0.rho, 1.0 / s1.rho
    assert np.allclose(I.dual_operator(0), [[r0, r0], [r0, r0 + 6 * P.h]], rtol=1e-14, atol=0)
    assert np.allclose(I.dual_operator(1), [[r1]], rtol=1e-14, atol=0)


@pytest.mark.parametrize("kind", ["heat3d", "elast3d"])
def test_c_norm_and_condition_estimates(kind):
    """||F~_i||_2 (power iteration) against the largest singular value of the
    dense F~_i, and cond(K_reg,i) (power + inverse iteration) against the
    ratio of the extreme eigenvalues of the dense K_reg,i (LAPACK)."""
    P = tiny(kind)
    I = orc_impl.ImplicitCPU(P.subs, P.n_lambda, nthreads=2)
    I.factor()
    nrm = I.opnorms(iters=300)
    kap = I.kappas(iters=300)
    for i, s in enumerate(P.subs):
        F = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)
        assert abs(nrm[i] - np.linalg.norm(F, 2)) <= 1e-6 * np.linalg.norm(F, 2)
        ev = np.linalg.eigvalsh(s.Kreg.toarray())
        # the largest eigenvalues of a stiffness matrix cluster, so the
        # power iteration is slow there: an estimate within 1 %
        assert abs(kap[i] - ev[-1] / ev[0]) <= 1e-2 * ev[-1] / ev[0]


@pytest.mark.parametrize("kind", ["heat3d", "elast3d", "heat2d_tri"])
def test_nd_order_is_a_permutation_with_the_same_operator(kind):
    """The oracle's geometric nested-dissection order is a permutation of
    the DOFs, keeps each node's DOFs together, and the implicit apply with
    it equals the one with SuperLU's minimum-degree order."""
    P = tiny(kind)
    for s in P.subs:
        p = orc_impl.nd_order(s.coords, s.dpn, leaf=4)
        assert np.array_equal(np.sort(p), np.arange(s.n))
        assert np.all(p.reshape(-1, s.dpn) // s.dpn == (p.reshape(-1, s.dpn) // s.dpn)[:, :1])
    qs = []
    for order in ("nd", "mmd"):
        I = orc_impl.ImplicitCPU(P.subs, P.n_lambda, nthreads=2, order=order)
        I.factor()
        qs.append(I.apply(P.lam))
    assert np.abs(qs[0] - qs[1]).max() <= 1e-12 * np.abs(qs[1]).max()


@pytest.mark.parametrize("kind", ["heat3d", "elast3d", "heat2d_tri"])
def test_sparse_reg_inverse_matches_dense(kind):
    """The oracle's sparse K_reg^{-1} (its own Cholesky, nested-dissection
    order, refined) solves like the dense LAPACK one and satisfies
    K K_reg^{-1} K = K (the generalised-inverse property, Sec. III)."""
    P = tiny(kind)
    rng = np.random.default_rng(3)
    for s in P.subs:
        inv = orc_impl.SparseRegInverse(s.Kreg, s.coords, s.dpn)
        ref = feti.RegInverse(s.Kreg)
        b = rng.standard_normal(s.n)
        x, xr = inv.solve(b), ref.solve(b)
        assert np.abs(x - xr).max() <= 1e-13 * np.abs(xr).max()
        K = s.K.toarray()
        KXK = K @ np.column_stack([inv.solve(K[:, j]) for j in range(s.n)])
        assert np.abs(KXK - K).max() <= 1e-10 * np.abs(K).max()


# ---------------------------------------------------------------- scaled lumped preconditioner

@pytest.mark.parametrize("kind,scaling", [("heat3d", "stiffness"), ("elast3d", "stiffness"),
                                          ("heat3d_tet", "multiplicity")])
def test_scaled_jump_operator_is_a_right_inverse(kind, scaling):
    """B_D = (B W B^T)^{-1} B W satisfies B_D B^T = I for any diagonal W > 0
    (B of full row rank): checked against B assembled from the subdomain
    rows directly (not through the oracle's B)."""
    P = tiny(kind)
    BD, _ = feti.scaled_jump_operator(P, scaling)
    off = np.concatenate([[0], np.cumsum([s.n for s in P.subs])])
    Bt = np.zeros((off[-1], P.n_lambda))
    for i, s in enumerate(P.subs):
        for j in range(s.m):
            Bt[off[i] + s.b_dof[j], s.dual_map[j]] = s.b_sign[j]
    assert np.abs(BD @ Bt - np.eye(P.n_lambda)).max() <= 1e-12


def test_scaled_jump_operator_two_subdomains_closed_form():
    """Without cross points (two subdomains, every node on one gluing row)
    B W B^T is diagonal and B_D reduces to row weights: on a gluing row
    between i and j the entry of subdomain i is its sign times
    k_j / (k_i + k_j) (k = diagonal stiffness at the glued DOF, stiffness
    scaling), on a Dirichlet row its sign."""
    P = make_problem(2, "heat", [[4, 5], [6]], 1.0, dirichlet_axis=0, seed=3)
    assert P.nsub == 2
    BD, _ = feti.scaled_jump_operator(P, "stiffness")
    off = [0, P.subs[0].n]
    carriers = {}
    for i, s in enumerate(P.subs):
        for j in range(s.m):
            carriers.setdefault(int(s.dual_map[j]), []).append((i, j))
    expect = np.zeros_like(BD)
    for g, cs in carriers.items():
        if len(cs) == 1:
            i, j = cs[0]
            expect[g, off[i] + P.subs[i].b_dof[j]] = P.subs[i].b_sign[j]
        else:
            (i, a), (k, b) = cs
            ki = P.subs[i].K.diagonal()[P.subs[i].b_dof[a]]
            kk = P.subs[k].K.diagonal()[P.subs[k].b_dof[b]]
            expect[g, off[i] + P.subs[i].b_dof[a]] = P.subs[i].b_sign[a] * kk / (ki + kk)
            expect[g, off[k] + P.subs[k].b_dof[b]] = P.subs[k].b_sign[b] * ki / (ki + kk)
    assert np.abs(BD - expect).max() <= 1e-14


@pytest.mark.parametrize("kind", ["heat3d", "elast3d"])
def test_scaled_lumped_pcpg_reaches_the_same_solution(kind):
    """Alg. 1 with M = B_D K B_D^T converges to the lambda of M = I (the
    solution does not depend on the preconditioner) in fewer iterations on
    a lognormal-coefficient problem; M is symmetric positive semi-definite."""
    P = tiny(kind)
    r = solve_feti(P, tol=1e-13)
    M = feti.scaled_lumped_preconditioner(P)
    Md = np.stack([M(e) for e in np.eye(P.n_lambda)], axis=1)
    assert np.abs(Md - Md.T).max() <= 1e-12 * np.abs(Md).max()
    assert np.linalg.eigvalsh(0.5 * (Md + Md.T)).min() >= -1e-10 * np.abs(Md).max()
    lam, it, _ = feti.pcpg(r["applyF"], r["d"], r["G"], r["e"], tol=1e-13, maxit=5000, M=M)
    assert np.abs(lam - r["lam"]).max() <= 1e-8 * np.abs(r["lam"]).max()
    assert it < r["it"]
