"""GPU parity of the batched supernodal solves: implicit application, the dual
right-hand side d = B K^+ f - c and the reverse mode of J = g^T F(theta) lambda.

All against the FP64 oracle; tolerance max(1e-12, kappa*eps) as for the
assembled operator (the solves use the same FP64 host factor)."""
import numpy as np
import pytest

from synth import config_problem, make_problem
from synth.problems import assemble_stiffness, regularise
from oracle import feti
from tests.gpu_common import say, make_context

pytestmark = pytest.mark.gpu


def _cases():
    return {
        "C5s": lambda: config_problem(5, scale=(2, 6)),
        "C2s": lambda: config_problem(2, scale=(2, 12)),
        "el3": lambda: make_problem(3, "elasticity", [[3, 4], [3, 3], [4, 3]], 0.3, dirichlet_axis=2, seed=3),
        "heat2d": lambda: make_problem(2, "heat", [[7, 13, 5], [9, 11]], 0.5, dirichlet_axis=0, seed=9),
        "C5s_tet": lambda: config_problem(5, scale=(2, 6), elem="simplex"),
    }


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _dev(t, a):
    return t.tensor(np.ascontiguousarray(a), dtype=t.float64, device="cuda")


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_implicit_apply_and_dual_rhs(torch_cuda, case):
    t = torch_cuda
    prob = _cases()[case]()
    say("implicit apply / dual rhs", case)
    ctx = make_context(prob)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    invs = [feti.RegInverse(s.Kreg) for s in prob.subs]
    q_o = feti.apply_implicit(invs, prob.subs, prob.lam, prob.n_lambda)
    lam = _dev(t, prob.lam)
    q = t.empty_like(lam)
    ctx.apply_implicit(lam, q)
    t.cuda.synchronize()
    qg = q.cpu().numpy()
    err = np.linalg.norm(qg - q_o) / np.linalg.norm(q_o)
    say("implicit rel err", err)
    assert err <= 1e-12
    ctx.apply_implicit(lam, q)
    t.cuda.synchronize()
    assert np.array_equal(q.cpu().numpy(), qg)   # deterministic
    f = np.concatenate([s.f for s in prob.subs])
    c = np.random.default_rng(1).standard_normal(prob.n_lambda)
    prob.c = c
    d_o = feti.d_vector(prob, invs)
    d = t.empty_like(lam)
    ctx.dual_rhs(_dev(t, f), d, c=_dev(t, c))
    t.cuda.synchronize()
    err = np.linalg.norm(d.cpu().numpy() - d_o) / np.linalg.norm(d_o)
    say("dual rhs rel err", err)
    assert err <= 1e-12
    ctx.close()


@pytest.mark.parametrize("case", ["C5s", "el3", "C5s_tet"])
def test_backward_matches_oracle(torch_cuda, case):
    t = torch_cuda
    prob = _cases()[case]()
    say("backward", case)
    ctx = make_context(prob, with_elements=True)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    g = prob.mu
    ne = sum(len(s.theta) for s in prob.subs)
    dlam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    dth = t.empty(ne, dtype=t.float64, device="cuda")
    ctx.apply_backward(_dev(t, g), _dev(t, prob.lam), dlam, dth)
    t.cuda.synchronize()
    Fs = [feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign) for s in prob.subs]
    dl_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], g, prob.n_lambda)
    err = np.linalg.norm(dlam.cpu().numpy() - dl_o) / np.linalg.norm(dl_o)
    say("dlambda rel err", err)
    assert err <= 1e-12
    dt_o = np.concatenate([feti.grad_theta(feti.RegInverse(s.Kreg), s, g, prob.lam) for s in prob.subs])
    err = np.linalg.norm(dth.cpu().numpy() - dt_o) / np.linalg.norm(dt_o)
    say("dtheta rel err", err)
    assert err <= 1e-12
    ctx.close()


def test_backward_central_differences(torch_cuda):
    """dJ/dtheta_e from the GPU adjoint against central differences of the
    oracle's J(theta) = mu^T F(theta) lambda, h = 1e-6 (rho frozen)."""
    t = torch_cuda
    prob = make_problem(3, "heat", [[3, 3], [3, 3], [3, 3]], 0.3, dirichlet_axis=2, seed=11)
    ctx = make_context(prob, with_elements=True)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    ne = sum(len(s.theta) for s in prob.subs)
    dlam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    dth = t.empty(ne, dtype=t.float64, device="cuda")
    ctx.apply_backward(_dev(t, prob.mu), _dev(t, prob.lam), dlam, dth)
    t.cuda.synchronize()
    dth = dth.cpu().numpy()
    offs = np.cumsum([0] + [len(s.theta) for s in prob.subs])
    rng = np.random.default_rng(0)
    for si in (0, 3, 7):
        s = prob.subs[si]
        for e in rng.choice(len(s.theta), 4, replace=False):
            vals = []
            for sgn in (1, -1):
                th = s.theta.copy()
                th[e] += sgn * 1e-6
                Kr = regularise(assemble_stiffness(s, th), s.R, s.fix_dofs, s.rho)
                F = feti.local_dual_operator(Kr, s.b_dof, s.b_sign)
                vals.append(prob.mu[s.dual_map] @ F @ prob.lam[s.dual_map])
            fd = (vals[0] - vals[1]) / 2e-6
            gpu = dth[offs[si] + e]
            say(f"sub {si} elem {e}: fd {fd:.10e} gpu {gpu:.10e}")
            assert abs(fd - gpu) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(dth).max())
    ctx.close()


def test_autograd_function_gradients(torch_cuda):
    """J = mu^T F(theta) lambda through torch.autograd: dJ/dlambda = F mu and
    dJ/dtheta equal the oracle's adjoint (workload C5 law, small mesh)."""
    t = torch_cuda
    from paper_2502_08382_amd.autograd import feti_apply
    prob = config_problem(5, scale=(2, 5))
    ctx = make_context(prob, with_elements=True)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    theta = t.tensor(np.concatenate([s.theta for s in prob.subs]), dtype=t.float64, device="cuda",
                     requires_grad=True)
    lam = _dev(t, prob.lam).requires_grad_(True)
    mu = _dev(t, prob.mu)
    J = (mu * feti_apply(lam, theta, ctx)).sum()
    J.backward()
    Fs = [feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign) for s in prob.subs]
    Ds = [s.dual_map for s in prob.subs]
    J_o = prob.mu @ feti.apply_explicit(Fs, Ds, prob.lam, prob.n_lambda)
    dl_o = feti.apply_explicit(Fs, Ds, prob.mu, prob.n_lambda)
    dt_o = np.concatenate([feti.grad_theta(feti.RegInverse(s.Kreg), s, prob.mu, prob.lam) for s in prob.subs])
    assert abs(J.item() - J_o) <= 1e-12 * abs(J_o)
    assert np.linalg.norm(lam.grad.cpu().numpy() - dl_o) <= 1e-12 * np.linalg.norm(dl_o)
    assert np.linalg.norm(theta.grad.cpu().numpy() - dt_o) <= 1e-12 * np.linalg.norm(dt_o)
    ctx.close()


@pytest.mark.timeout(900)
def test_backward_full_size(torch_cuda):
    """The 64-subdomain heat workload (10^3 hexes, theta = exp(N(0, 0.3)))
    at full size.

    * dJ/dlambda = F mu: every entry against the oracle's explicit apply,
      |d_g| <= 1e-12 s_g (s_g = sum over the carriers of g of
      ||F~_i||_2 ||mu_i||_2).
    * dJ/dtheta of every element of every subdomain against the oracle's
      adjoint -u_mu|_e^T K_e0 u_lam|_e.  With u = K_reg^{-1} B~^T x known to
      a normwise relative error of about kappa(K_reg,i) eps on either side,
      |d(dJ/dtheta_e)| <= tau_i ||K_e0||_2 (||u_mu|| ||u_lam|_e|| +
      ||u_mu|_e|| ||u_lam||) with tau_i = max(1e-12, kappa_i eps) (kappa
      from the oracle's estimate); the observed maximum is printed.
    * Central differences (h = 1e-6) of the oracle's J_i on all 1000
      elements of one subdomain and 256 seeded elements of the others.  A
      subdomain's J_i is ~2e5 while dJ/dtheta_e is O(1-10), so the quotient
      carries a rounding error of order eps |J_i| / h; the bound is 1e-6
      relative plus 50 eps |J_i| / h."""
    import os
    t = torch_cuda
    prob = config_problem(5)
    say("backward full size", "nsub", prob.nsub)
    ctx = make_context(prob, with_elements=True)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    ne = sum(len(s.theta) for s in prob.subs)
    dlam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    dth = t.empty(ne, dtype=t.float64, device="cuda")
    ctx.apply_backward(_dev(t, prob.mu), _dev(t, prob.lam), dlam, dth)
    t.cuda.synchronize()
    dth = dth.cpu().numpy()
    dlam = dlam.cpu().numpy()
    from oracle import implicit as orc
    I = orc.ImplicitCPU(prob.subs, prob.n_lambda, nthreads=max(1, min(16, len(os.sched_getaffinity(0)))))
    I.factor()
    kap = I.kappas(60)
    invs = [feti.RegInverse(s.Kreg) for s in prob.subs]
    Fs = [feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign, inv) for s, inv in zip(prob.subs, invs)]
    dl_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.mu, prob.n_lambda)
    sc = np.zeros(prob.n_lambda)
    for F, sub in zip(Fs, prob.subs):
        sc[sub.dual_map] += np.linalg.norm(F, 2) * np.linalg.norm(prob.mu[sub.dual_map])
    e_dl = (np.abs(dlam - dl_o) / sc).max()
    say(f"dlambda: every entry max |d|/s_g {e_dl:.2e}, normwise "
        f"{np.linalg.norm(dlam - dl_o) / np.linalg.norm(dl_o):.2e}")
    assert e_dl <= 1e-12
    offs = np.cumsum([0] + [len(s.theta) for s in prob.subs])
    worst, worst_rel = 0.0, 0.0
    for si, (s, inv) in enumerate(zip(prob.subs, invs)):
        g_o = feti.grad_theta(inv, s, prob.mu, prob.lam)
        g_g = dth[offs[si]:offs[si + 1]]
        um = feti.primal_from_dual(inv, s, prob.mu)
        ul = feti.primal_from_dual(inv, s, prob.lam)
        ed = s.elem_dofs()
        kn = np.linalg.norm(s.Ke_ref, 2) if s.uniform_elements else \
            np.array([np.linalg.norm(K, 2) for K in s.elem_matrices()])
        se = kn * (np.linalg.norm(um) * np.linalg.norm(ul[ed], axis=1)
                   + np.linalg.norm(um[ed], axis=1) * np.linalg.norm(ul))
        tau = max(1e-12, kap[si] * np.finfo(float).eps)
        r = (np.abs(g_g - g_o) / se).max()
        worst = max(worst, r / tau)
        worst_rel = max(worst_rel, np.linalg.norm(g_g - g_o) / np.linalg.norm(g_o))
        assert r <= tau, (si, r, tau)
    say(f"dtheta, every element of every subdomain: max |d|/(tau_i s_e) {worst:.2e}, "
        f"worst normwise rel {worst_rel:.2e}")
    rng = np.random.default_rng(2)
    h, eps = 1e-6, np.finfo(float).eps
    full = int(rng.integers(prob.nsub))
    picks = [(full, e) for e in range(len(prob.subs[full].theta))]
    others = [i for i in range(prob.nsub) if i != full]
    for j in range(256):
        si = int(others[rng.integers(len(others))])
        picks.append((si, int(rng.integers(len(prob.subs[si].theta)))))
    def central_difference(pick):
        si, e = pick
        s = prob.subs[si]
        bl = np.zeros(s.n)
        np.add.at(bl, s.b_dof, s.b_sign * prob.lam[s.dual_map])
        vals = []
        for sgn in (1, -1):
            th = s.theta.copy()
            th[e] += sgn * h
            Kr = regularise(assemble_stiffness(s, th), s.R, s.fix_dofs, s.rho)
            um = feti.primal_from_dual(orc.SparseRegInverse(Kr, s.coords, s.dpn), s, prob.mu)
            vals.append(um @ bl)          # J_i = mu_i^T B~ K_reg^{-1} B~^T lambda_i
        return (vals[0] - vals[1]) / (2 * h), abs(vals[0])

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max(1, min(16, len(os.sched_getaffinity(0))))) as ex:
        fds = list(ex.map(central_difference, picks))
    worst_fd = 0.0
    for (si, e), (fd, Ji) in zip(picks, fds):
        gpu = dth[offs[si] + e]
        bound = 1e-6 * abs(fd) + 50 * eps * Ji / h
        worst_fd = max(worst_fd, abs(fd - gpu) / bound)
        assert abs(fd - gpu) <= bound, (si, e, fd, gpu, bound)
    say(f"central differences on {len(picks)} elements (all of subdomain {full}): max |fd - gpu|/bound "
        f"{worst_fd:.2e}")
    ctx.close()


def test_debug_checks_report_non_finite_values(torch_cuda):
    """Option debug_checks: a NaN in lambda (fetiF_apply, fetiF_apply_static,
    fetiF_apply_implicit) or in g (fetiF_apply_backward) is reported as
    FETIF_ENONFINITE naming the vector and its first bad index; with finite
    inputs the results equal those of a context without checks, bitwise."""
    from paper_2502_08382_amd import FetiError
    t = torch_cuda
    prob = _cases()["C5s"]()
    ref = make_context(prob, with_elements=True)
    dbg = make_context(prob, with_elements=True, debug_checks=1)
    for c in (ref, dbg):
        c.factor_upload([s.Kreg.data for s in prob.subs])
        c.assemble()
    ne = sum(len(s.theta) for s in prob.subs)
    lam, g = _dev(t, prob.lam), _dev(t, prob.mu)
    outs = {}
    for name, c in (("ref", ref), ("dbg", dbg)):
        q, qs, qi = (t.empty(prob.n_lambda, dtype=t.float64, device="cuda") for _ in range(3))
        dl, dth = t.empty(prob.n_lambda, dtype=t.float64, device="cuda"), t.empty(ne, dtype=t.float64, device="cuda")
        c.apply(lam, q)
        c.apply_static(lam, qs)
        c.apply_implicit(lam, qi)
        c.apply_backward(g, lam, dl, dth)
        t.cuda.synchronize()
        outs[name] = [x.cpu().numpy() for x in (q, qs, qi, dl, dth)]
    for a, b in zip(outs["ref"], outs["dbg"]):
        assert np.array_equal(a, b)
    bad = lam.clone()
    bad[7] = float("nan")
    q = t.empty_like(lam)
    for call in (lambda: dbg.apply(bad, q), lambda: dbg.apply_static(bad, q), lambda: dbg.apply_implicit(bad, q)):
        with pytest.raises(FetiError) as e:
            call()
        say("debug check:", e.value)
        assert e.value.status == 7 and "lambda" in str(e.value) and "index 7" in str(e.value)
    gb = g.clone()
    gb[3] = float("inf")
    dl, dth = t.empty_like(lam), t.empty(ne, dtype=t.float64, device="cuda")
    with pytest.raises(FetiError) as e:
        dbg.apply_backward(gb, lam, dl, dth)
    say("debug check:", e.value)
    assert e.value.status == 7 and "g holds" in str(e.value) and "index 3" in str(e.value)
    # without the option the NaN propagates and nothing is raised
    ref.apply(bad, q)
    t.cuda.synchronize()
    assert np.isnan(q.cpu().numpy()).any()
    ref.close()
    dbg.close()
