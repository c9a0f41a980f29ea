"""GPU parity of the dual solver (Alg. 1) and the primal recovery.

Pins: a fixed number of PCPG iterations reproduces the oracle's iterates of
the same algorithm; the converged lambda equals the oracle's; u equals the
global FEM direct solve (the torn system is equivalent to the FEM system);
graph replay is bitwise identical to direct launches; FP32/BF16 operators
with FP64 refinement reach the FP64 solution."""
import numpy as np
import pytest

from synth import config_problem, make_problem
from oracle import feti
from tests.gpu_common import say, make_context
from tests.test_oracle_pins import global_fem_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _dev(t, a):
    return t.tensor(np.ascontiguousarray(a), dtype=t.float64, device="cuda")


def _cases():
    return {
        "C1": lambda: config_problem(1),
        "heat3d": lambda: make_problem(3, "heat", [[3, 4], [4, 3], [3, 3]], 0.5, dirichlet_axis=2, seed=4),
        "elast3d": lambda: make_problem(3, "elasticity", [[3, 3], [3, 4], [4, 3]], 0.2, dirichlet_axis=2, seed=6),
        "heat3d_tet": lambda: make_problem(3, "heat", [[4, 3], [3, 4], [3, 3]], 0.5, dirichlet_axis=2, seed=8,
                                           elem="simplex"),
    }


def _oracle(prob):
    invs = [feti.RegInverse(s.Kreg) for s in prob.subs]
    Fs = [feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign, i) for s, i in zip(prob.subs, invs)]
    Ds = [s.dual_map for s in prob.subs]
    applyF = lambda x: feti.apply_explicit(Fs, Ds, x, prob.n_lambda)
    return invs, applyF, feti.G_matrix(prob), feti.e_vector(prob), feti.d_vector(prob, invs)


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_pcpg_and_primal_match_oracle_and_fem(torch_cuda, case):
    t = torch_cuda
    prob = _cases()[case]()
    say("pcpg", case, "n_lambda", prob.n_lambda)
    invs, applyF, G, e_o, d_o = _oracle(prob)
    ctx = make_context(prob)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    f = _dev(t, np.concatenate([s.f for s in prob.subs]))
    nk = G.shape[1]
    e = t.empty(nk, dtype=t.float64, device="cuda")
    d = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    ctx.coarse_rhs(f, e)
    ctx.dual_rhs(f, d)
    t.cuda.synchronize()
    assert np.abs(e.cpu().numpy() - e_o).max() <= 1e-12 * max(1.0, np.abs(e_o).max())
    assert np.linalg.norm(d.cpu().numpy() - d_o) <= 1e-12 * np.linalg.norm(d_o)
    # a fixed number of iterations reproduces the oracle's iterates
    lam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    stream = t.cuda.Stream()
    with t.cuda.stream(stream):
        r5 = ctx.pcpg(d, e, lam, fixed_iters=5, stream=stream)
    stream.synchronize()
    lam5_o, it5, _ = feti.pcpg(applyF, d_o, G, e_o, fixed_iters=5)
    err5 = np.linalg.norm(lam.cpu().numpy() - lam5_o) / np.linalg.norm(lam5_o)
    say("5 iterations: rel diff", err5, r5)
    assert r5["iters"] == 5 and err5 <= 1e-10
    # converged solution
    with t.cuda.stream(stream):
        r = ctx.pcpg(d, e, lam, tol=1e-12, max_iters=3000, stream=stream)
    stream.synchronize()
    lam_o, it_o, _ = feti.pcpg(applyF, d_o, G, e_o, tol=1e-12, maxit=3000)
    err = np.linalg.norm(lam.cpu().numpy() - lam_o) / np.linalg.norm(lam_o)
    say(f"converged: gpu iters {r['iters']} oracle iters {it_o} rel err {err:.2e} res {r['rel_residual']:.2e}")
    assert r["rel_residual"] <= 1e-12 and err <= 1e-8
    assert abs(r["iters"] - it_o) <= 10
    # primal recovery against the global FEM solve
    alpha = t.empty(nk, dtype=t.float64, device="cuda")
    u = t.empty(sum(s.n for s in prob.subs), dtype=t.float64, device="cuda")
    ctx.primal(f, d, lam, alpha, u)
    t.cuda.synchronize()
    ug = global_fem_solve(prob)
    uu = u.cpu().numpy()
    off, worst = 0, 0.0
    for s in prob.subs:
        gd = (s.gnode[:, None] * prob.dpn + np.arange(prob.dpn)[None, :]).ravel()
        worst = max(worst, np.abs(uu[off:off + s.n] - ug[gd]).max())
        off += s.n
    say("u vs FEM max abs err", worst, "scale", np.abs(ug).max())
    assert worst <= 1e-8 * np.abs(ug).max()
    ctx.close()


def test_pcpg_graph_replay_is_bitwise_identical(torch_cuda):
    t = torch_cuda
    prob = config_problem(5, scale=(2, 5))
    ctx = make_context(prob)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    f = _dev(t, np.concatenate([s.f for s in prob.subs]))
    e = t.empty(prob.nsub, dtype=t.float64, device="cuda")
    d = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    ctx.coarse_rhs(f, e)
    ctx.dual_rhs(f, d)
    stream = t.cuda.Stream()
    outs = []
    for graph in (False, True, True):
        lam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
        with t.cuda.stream(stream):
            r = ctx.pcpg(d, e, lam, fixed_iters=40, check_every=10, use_graph=graph, stream=stream)
        stream.synchronize()
        # eager work between replays
        _ = (lam * 2).sum().item()
        outs.append(lam.cpu().numpy())
        say("graph" if graph else "direct", r)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_pcpg_refinement_reaches_fp64_solution(torch_cuda, prec):
    t = torch_cuda
    prob = config_problem(4, scale=(2, 8))
    invs, applyF, G, e_o, d_o = _oracle(prob)
    lam_o, it_o, _ = feti.pcpg(applyF, d_o, G, e_o, tol=1e-12, maxit=3000)
    ctx = make_context(prob, f_storage=prec)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    f = _dev(t, np.concatenate([s.f for s in prob.subs]))
    e = t.empty(prob.nsub, dtype=t.float64, device="cuda")
    d = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    ctx.coarse_rhs(f, e)
    ctx.dual_rhs(f, d)
    lam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    stream = t.cuda.Stream()
    with t.cuda.stream(stream):
        r = ctx.pcpg(d, e, lam, tol=1e-9, refine=True, inner_tol=1e-4 if prec == "f32" else 1e-2,
                     max_iters=5000, stream=stream)
    stream.synchronize()
    err = np.linalg.norm(lam.cpu().numpy() - lam_o) / np.linalg.norm(lam_o)
    say(prec, "refined:", r, "lambda rel err", err, "fp64 oracle iters", it_o)
    assert r["rel_residual"] <= 1e-9
    assert err <= 1e-6
    ctx.close()


@pytest.mark.parametrize("case", ["heat3d", "elast3d"])
def test_pcpg_lumped_preconditioner(torch_cuda, case):
    """PCPG with the lumped preconditioner M = sum_i D_i^T B~_i K_reg,i B~_i^T
    D_i: five iterations reproduce the oracle's preconditioned iterates, the
    converged lambda equals the oracle's and the unpreconditioned solution,
    the primal solution equals the global FEM solve, and graph replay is
    bitwise equal to direct launches."""
    t = torch_cuda
    prob = _cases()[case]()
    say("lumped pcpg", case, "n_lambda", prob.n_lambda)
    invs, applyF, G, e_o, d_o = _oracle(prob)
    M = feti.lumped_preconditioner(prob)
    ctx = make_context(prob)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    f = _dev(t, np.concatenate([s.f for s in prob.subs]))
    nk = G.shape[1]
    e = t.empty(nk, dtype=t.float64, device="cuda")
    d = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    ctx.coarse_rhs(f, e)
    ctx.dual_rhs(f, d)
    stream = t.cuda.Stream()
    lam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    with t.cuda.stream(stream):
        r5 = ctx.pcpg(d, e, lam, fixed_iters=5, precond=1, use_graph=False, stream=stream)
    stream.synchronize()
    lam5 = lam.cpu().numpy()
    lam5_o, _, _ = feti.pcpg(applyF, d_o, G, e_o, fixed_iters=5, M=M)
    err5 = np.linalg.norm(lam5 - lam5_o) / np.linalg.norm(lam5_o)
    say("5 preconditioned iterations: rel diff", err5, r5)
    assert err5 <= 1e-10
    with t.cuda.stream(stream):
        ctx.pcpg(d, e, lam, fixed_iters=5, precond=1, use_graph=True, check_every=5, stream=stream)
    stream.synchronize()
    assert np.array_equal(lam.cpu().numpy(), lam5)
    with t.cuda.stream(stream):
        r = ctx.pcpg(d, e, lam, tol=1e-12, max_iters=3000, precond=1, stream=stream)
    stream.synchronize()
    lam_o, it_o, _ = feti.pcpg(applyF, d_o, G, e_o, tol=1e-12, maxit=3000, M=M)
    lam_i, it_i, _ = feti.pcpg(applyF, d_o, G, e_o, tol=1e-12, maxit=3000)
    err = np.linalg.norm(lam.cpu().numpy() - lam_o) / np.linalg.norm(lam_o)
    say(f"converged: gpu iters {r['iters']} oracle {it_o} (unpreconditioned {it_i}) rel err {err:.2e}")
    assert r["rel_residual"] <= 1e-12 and err <= 1e-8
    assert np.linalg.norm(lam_o - lam_i) <= 1e-8 * np.linalg.norm(lam_i)
    alpha = t.empty(nk, dtype=t.float64, device="cuda")
    u = t.empty(sum(s.n for s in prob.subs), dtype=t.float64, device="cuda")
    ctx.primal(f, d, lam, alpha, u)
    t.cuda.synchronize()
    ug = global_fem_solve(prob)
    uu = u.cpu().numpy()
    off, worst = 0, 0.0
    for s in prob.subs:
        gd = (s.gnode[:, None] * prob.dpn + np.arange(prob.dpn)[None, :]).ravel()
        worst = max(worst, np.abs(uu[off:off + s.n] - ug[gd]).max())
        off += s.n
    assert worst <= 1e-8 * np.abs(ug).max()
    ctx.close()


@pytest.mark.parametrize("case", ["heat3d", "elast3d", "C4s"])
def test_pcpg_scaled_lumped_preconditioner(torch_cuda, case):
    """PCPG with the lumped preconditioner on the scaled jump operator,
    M = B_D K B_D^T with B_D = (B W B^T)^{-1} B W, W = diag(K_i)^{-1}
    (fetiF_precond_values given the unregularised K_i): five iterations
    reproduce the oracle's preconditioned iterates, the converged lambda
    equals the unpreconditioned solution, in fewer iterations, and graph
    replay is bitwise equal to direct launches."""
    from paper_2502_08382_amd import values_in_pattern
    t = torch_cuda
    prob = config_problem(4, scale=(3, 6)) if case == "C4s" else _cases()[case]()
    say("scaled lumped pcpg", case, "n_lambda", prob.n_lambda)
    invs, applyF, G, e_o, d_o = _oracle(prob)
    M = feti.scaled_lumped_preconditioner(prob, "stiffness", "K")
    ctx = make_context(prob)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    ctx.precond_values([values_in_pattern(s.K, s.Kreg) for s in prob.subs])
    f = _dev(t, np.concatenate([s.f for s in prob.subs]))
    e = t.empty(G.shape[1], dtype=t.float64, device="cuda")
    d = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    ctx.coarse_rhs(f, e)
    ctx.dual_rhs(f, d)
    stream = t.cuda.Stream()
    lam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    with t.cuda.stream(stream):
        ctx.pcpg(d, e, lam, fixed_iters=5, precond=2, use_graph=False, stream=stream)
    stream.synchronize()
    lam5 = lam.cpu().numpy()
    lam5_o, _, _ = feti.pcpg(applyF, d_o, G, e_o, fixed_iters=5, M=M)
    err5 = np.linalg.norm(lam5 - lam5_o) / np.linalg.norm(lam5_o)
    say(f"  5 preconditioned iterations: rel diff {err5:.2e}")
    assert err5 <= 1e-10
    with t.cuda.stream(stream):
        ctx.pcpg(d, e, lam, fixed_iters=5, precond=2, use_graph=True, check_every=5, stream=stream)
    stream.synchronize()
    assert np.array_equal(lam.cpu().numpy(), lam5)
    with t.cuda.stream(stream):
        r = ctx.pcpg(d, e, lam, tol=1e-12, max_iters=3000, precond=2, stream=stream)
        r0 = ctx.pcpg(d, e, lam, tol=1e-12, max_iters=3000, precond=0, stream=stream)
    stream.synchronize()
    lam_i, it_i, _ = feti.pcpg(applyF, d_o, G, e_o, tol=1e-12, maxit=3000)
    with t.cuda.stream(stream):
        ctx.pcpg(d, e, lam, tol=1e-12, max_iters=3000, precond=2, stream=stream)
    stream.synchronize()
    err = np.linalg.norm(lam.cpu().numpy() - lam_i) / np.linalg.norm(lam_i)
    say(f"  converged: gpu iters {r['iters']} (M = I: {r0['iters']}, oracle M = I: {it_i}) rel err vs M = I "
        f"solution {err:.2e}")
    assert r["rel_residual"] <= 1e-12 and err <= 1e-8
    assert r["iters"] < r0["iters"]
    ctx.close()


@pytest.mark.parametrize("refine", [False, True])
def test_pcpg_reports_nan_for_non_finite_input(torch_cuda, refine):
    """A NaN in d makes the projected residual NaN: the solver reports
    rel_residual (and w0) as NaN, not as a converged 0, and the same context
    solves a finite right-hand side normally afterwards."""
    t = torch_cuda
    prob = _cases()["heat3d"]()
    ctx = make_context(prob)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    f = _dev(t, np.concatenate([s.f for s in prob.subs]))
    e = t.empty(ctx.n_coarse, dtype=t.float64, device="cuda")
    d = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    lam = t.empty(prob.n_lambda, dtype=t.float64, device="cuda")
    ctx.coarse_rhs(f, e)
    ctx.dual_rhs(f, d)
    d[3] = float("nan")
    r = ctx.pcpg(d, e, lam, tol=1e-9, max_iters=200, refine=refine)
    t.cuda.synchronize()
    say("NaN in d, refine", refine, r)
    assert np.isnan(r["rel_residual"]) and np.isnan(r["w0"]), r
    ctx.dual_rhs(f, d)
    r2 = ctx.pcpg(d, e, lam, tol=1e-9, max_iters=3000, refine=refine)
    t.cuda.synchronize()
    say("finite d afterwards", r2)
    assert r2["rel_residual"] <= 1e-9 and np.isfinite(lam.cpu().numpy()).all(), r2
