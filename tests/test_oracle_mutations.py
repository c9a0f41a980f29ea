"""Mistakes planted in the oracle, on the CPU, are caught by its pins.

Each case replaces one oracle function by a copy carrying a plausible
mistake (a flipped sign, a dropped term, a transposed or shifted index, a
wrong operand) and runs the pins of tests/test_oracle_pins.py that should
reject it; the test passes when they fail.  This shows that the pins are
not satisfied by the oracle's own structure alone.  Nothing here touches a
GPU or the library.
"""
import numpy as np
import pytest

from oracle import feti
import tests.test_oracle_pins as pins

_ORIG_LDO = feti.local_dual_operator
_ORIG_APPLY_EXPL = feti.apply_explicit
_ORIG_APPLY_IMPL = feti.apply_implicit
_ORIG_PROJ_CALL = feti.Projector.__call__
_ORIG_GRAD = feti.grad_theta
_ORIG_SOLVE = feti.RegInverse.solve
_ORIG_SJO = feti.scaled_jump_operator
_ORIG_PCPG = feti.pcpg


def ldo_offdiag_sign(Kreg, b_dof, b_sign, inv=None):
    F = _ORIG_LDO(Kreg, b_dof, b_sign, inv)
    if F.shape[0] > 1:
        F = F.copy()
        F[0, 1] = -F[0, 1]
        F[1, 0] = -F[1, 0]
    return F


def ldo_no_signs(Kreg, b_dof, b_sign, inv=None):
    return _ORIG_LDO(Kreg, b_dof, np.abs(np.asarray(b_sign)), inv)


def ldo_shifted_dof(Kreg, b_dof, b_sign, inv=None):
    d = np.asarray(b_dof).copy()
    d[-1] = (d[-1] + 1) % Kreg.shape[0]
    return _ORIG_LDO(Kreg, d, b_sign, inv)


def solve_dropped_refinement_and_scaled(self, rhs, refine=True):
    return 1.001 * _ORIG_SOLVE(self, rhs, refine)


def apply_expl_drops_last(F_list, dual_maps, lam, n_lambda):
    return _ORIG_APPLY_EXPL(F_list[:-1], dual_maps[:-1], lam, n_lambda)


def apply_expl_transposed_map(F_list, dual_maps, lam, n_lambda):
    q = np.zeros(n_lambda)
    for F, D in zip(F_list, dual_maps):
        np.add.at(q, D[::-1], F @ lam[D])
    return q


def apply_impl_sign_dropped(invs, subs, lam, n_lambda):
    q = np.zeros(n_lambda)
    for inv, s in zip(invs, subs):
        p = lam[s.dual_map]
        v = np.zeros(s.n)
        np.add.at(v, s.b_dof, p)
        u = inv.solve(v)
        np.add.at(q, s.dual_map, s.b_sign * u[s.b_dof])
    return q


def projector_plus(self, x):
    return x + self.G @ self.coarse_solve(self.G.T @ x)


def grad_sign(inv, sub, mu, lam):
    return -_ORIG_GRAD(inv, sub, mu, lam)


def grad_swapped_operands(inv, sub, mu, lam):
    um = feti.primal_from_dual(inv, sub, mu)
    ul = feti.primal_from_dual(inv, sub, lam)
    ed = sub.elem_dofs()
    Ke = np.broadcast_to(sub.elem_matrices(), (ed.shape[0],) + sub.Ke_ref.shape[-2:])
    return -np.einsum("ea,eab,eb->e", um[ed], Ke, um[ed])


def sjo_one_sided_weights(prob, scaling="stiffness", K="K"):
    BD, B = _ORIG_SJO(prob, scaling, K)
    # (B W B^T)^{-1} B instead of (B W B^T)^{-1} B W
    nn = [s.n for s in prob.subs]
    off = np.concatenate([[0], np.cumsum(nn)])
    wv = np.concatenate([1.0 / (s.K if K == "K" else s.Kreg).diagonal() for s in prob.subs])
    A = (B * wv[None, :]) @ B.T
    return np.linalg.solve(A, B), B


def pcpg_beta_sign(apply_F, d, G, e, tol=1e-9, maxit=1000, M=None, fixed_iters=None):
    P = feti.Projector(G)
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
    while (fixed_iters is not None and k < fixed_iters) or (fixed_iters is None and hist[-1] > tol and k < maxit):
        q = apply_F(p)
        delta = wy / (p @ q)
        lam = lam + delta * p
        r = r - delta * q
        w = P(r)
        y = P(Mop(w))
        wy_new = w @ y
        p = y - (wy_new / wy) * p
        wy = wy_new
        k += 1
        hist.append(np.linalg.norm(w) / w0)
    return lam, k, np.array(hist)


CASES = [
    ("local_dual_operator: off-diagonal sign", (feti, "local_dual_operator", ldo_offdiag_sign),
     [lambda: pins.test_local_dual_operator_1d_closed_form(3, 4),
      lambda: pins.test_local_dual_operator_brute_force("heat3d")]),
    ("local_dual_operator: signs of B~ dropped", (feti, "local_dual_operator", ldo_no_signs),
     [lambda: pins.test_local_dual_operator_1d_closed_form(3, 4),
      lambda: pins.test_local_dual_operator_brute_force("elast3d")]),
    ("local_dual_operator: a multiplier on the wrong DOF", (feti, "local_dual_operator", ldo_shifted_dof),
     [lambda: pins.test_local_dual_operator_brute_force("heat2d"),
      lambda: pins.test_F_additivity_and_apply_routes()]),
    ("RegInverse.solve: a stray factor", (feti.RegInverse, "solve", solve_dropped_refinement_and_scaled),
     [lambda: pins.test_generalized_inverse("heat3d"),
      lambda: pins.test_local_dual_operator_1d_closed_form(2, 5)]),
    ("apply_explicit: last subdomain dropped", (feti, "apply_explicit", apply_expl_drops_last),
     [lambda: pins.test_F_additivity_and_apply_routes(),
      lambda: pins.test_feti_solution_equals_global_fem("heat3d")]),
    ("apply_explicit: gather through a reversed map", (feti, "apply_explicit", apply_expl_transposed_map),
     [lambda: pins.test_F_additivity_and_apply_routes()]),
    ("apply_implicit: sign of the scatter dropped", (feti, "apply_implicit", apply_impl_sign_dropped),
     [lambda: pins.test_F_additivity_and_apply_routes()]),
    ("Projector: I + G (G^T G)^{-1} G^T", (feti.Projector, "__call__", projector_plus),
     [lambda: pins.test_feti_solution_equals_global_fem("heat3d"),
      lambda: pins.test_projected_operator_matches_moore_penrose("heat2d")]),
    ("pcpg: sign of beta", (feti, "pcpg", pcpg_beta_sign),
     [lambda: pins.test_feti_solution_equals_global_fem("elast3d")]),
    ("grad_theta: sign", (feti, "grad_theta", grad_sign),
     [lambda: pins.test_gradient_central_differences("box", "heat"),
      lambda: pins.test_gradient_euler_identity()]),
    ("grad_theta: u_mu used twice", (feti, "grad_theta", grad_swapped_operands),
     [lambda: pins.test_gradient_central_differences("simplex", "elasticity")]),
    ("scaled_jump_operator: W on one side only", (feti, "scaled_jump_operator", sjo_one_sided_weights),
     [lambda: pins.test_scaled_jump_operator_is_a_right_inverse("heat3d", "stiffness"),
      lambda: pins.test_scaled_jump_operator_two_subdomains_closed_form()]),
]


@pytest.mark.parametrize("name,patch,checks", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, name, patch, checks):
    owner, attr, bad = patch
    monkeypatch.setattr(owner, attr, bad)
    for check in checks:
        with pytest.raises((AssertionError, np.linalg.LinAlgError)):
            check()


def test_unmutated_pins_pass():
    """The same checks pass on the oracle as it is."""
    for _, _, checks in CASES:
        for check in checks:
            check()
