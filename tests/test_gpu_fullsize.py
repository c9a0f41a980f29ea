"""Full-size parity of the assembled operator and its application, element by
element, in the launch configuration the benchmark times.

Workloads: the 512-subdomain heat problem (12^3 hexes, lognormal(0, 0.5)),
the 729 uneven elasticity subdomains (m up to 3438) and the 216-subdomain
heat problem (16^3 hexes, lognormal(0, 1)) with F~ stored in FP64, FP32 and
BF16.  Launch configuration: the TRSM shape the assembly tuner picks and the
stored apply shape of the workload (as bench.py installs them).

Every entry of q = sum_i D_i^T F~_i D_i lambda is checked against the
oracle's implicit apply (plain C sparse Cholesky, eq. dualop_apply_impl);
normwise against ||q|| the bound is 1e-12, or kappa_max eps where the
conditioning of K_reg allows no better (observed: 4.5e-11 on the uneven
elasticity workload, kappa up to 8.5e6).
The per-entry bound is tau * s_g with the normwise scale
    s_g = sum over the (subdomain i, row a) carrying multiplier g of
          ||F~_i||_2 ||lambda_i||_2     (>= sum_b |F~_i[a,b]| |lambda_b|),
||F~_i||_2 from the oracle (power iteration), and
 * FP64: tau = 1e-12 (the FP64 parity target);
 * FP32 / BF16 storage: tau = u_s + u_32 + gamma_d with u_s the storage
   rounding unit (2^-24, 2^-8), u_32 = 2^-24 for lambda rounded to FP32, and
   gamma_d = d u_32 / (1 - d u_32) for FP32 sums no deeper than
   d = ceil(m_max / 4) + 64 additions (a lane adds the column terms of the
   rows its wavefront takes, a quarter of a band, plus its row-dot and
   reduction chains); this is a worst-case bound.
F~_i is compared element-wise on 16 subdomains per workload (the largest
and smallest m, the largest n, 13 seeded ones) against the refined dense
oracle: |F_gpu[a,b] - F[a,b]| <= tol sqrt(F[a,a] F[b,b]) with tol = 1e-12,
or the conditioning bound kappa(K_reg,i) eps when that is larger (kappa
from the oracle's estimate).  FP32/BF16 storage is pinned bitwise on every
subdomain: it equals the round-to-nearest-even of the FP64 context's F~_i
built from the same factor with the same TRSM shape.  Observed maxima are
printed.
"""
import numpy as np
import pytest

from synth import config_problem
from oracle import feti
from oracle import implicit as orc
from tests.gpu_common import say, make_context, rne_f32, rne_bf16, reduced_apply_bound

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

EPS = np.finfo(float).eps

_CACHE = {}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _workload(k):
    """Problem, oracle (factored), ||F~_i||_2 and kappa(K_reg,i) estimates
    of workload k, built once per session."""
    if k not in _CACHE:
        import os
        prob = config_problem(k)
        nt = max(1, min(16, len(os.sched_getaffinity(0))))
        I = orc.ImplicitCPU(prob.subs, prob.n_lambda, nthreads=nt)
        I.factor()
        q_o = I.apply(prob.lam)
        nrm = I.opnorms(60)
        kap = I.kappas(60)
        _CACHE[k] = (prob, I, q_o, nrm, kap)
        say(f"workload {k}: nsub {prob.nsub} n_lambda {prob.n_lambda} m {min(s.m for s in prob.subs)}.."
            f"{max(s.m for s in prob.subs)} kappa {kap.min():.2e}..{kap.max():.2e}")
    return _CACHE[k]


def _scale(prob, nrm, lam):
    """s_g = sum over the carriers of g of ||F~_i||_2 ||lambda_i||_2."""
    s = np.zeros(prob.n_lambda)
    for i, sub in enumerate(prob.subs):
        s[sub.dual_map] += nrm[i] * np.linalg.norm(lam[sub.dual_map])
    return s


def _sample(prob, k=16):
    ms = [s.m for s in prob.subs]
    ns = [s.n for s in prob.subs]
    pick = [int(np.argmax(ms)), int(np.argmin(ms)), int(np.argmax(ns))]
    rng = np.random.default_rng(31)
    for i in rng.permutation(prob.nsub):
        if len(set(pick)) >= k:
            break
        pick.append(int(i))
    return sorted(set(pick))


def _bench_context(prob, prec, torch_cuda, trsm=None):
    """Context assembled in the benchmark's launch configuration."""
    from paper_2502_08382_amd.autotune import tune_assembly, install_stored_apply_shape
    ctx = make_context(prob, f_storage=prec)
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    if trsm is None:
        trsm = tune_assembly(ctx)
        trsm = (trsm["panel"], trsm["chunk"])
    ctx.set_assembly(*trsm)
    ctx.assemble()
    torch_cuda.cuda.synchronize()
    shape = install_stored_apply_shape(ctx)
    say(f"  launch configuration: trsm {trsm}, apply {shape}")
    return ctx, trsm


def _gpu_apply(t, ctx, lam):
    lam_d = t.tensor(lam, dtype=t.float64, device="cuda")
    q_d = t.empty_like(lam_d)
    ctx.apply(lam_d, q_d)
    t.cuda.synchronize()
    return q_d.cpu().numpy()


def _check_q(prob, q_g, q_o, scale, tau, label):
    err = np.abs(q_g - q_o)
    ratio = err / scale
    g = int(np.argmax(ratio))
    rel = np.linalg.norm(q_g - q_o) / np.linalg.norm(q_o)
    say(f"  {label}: every q entry: max |dq|/s_g {ratio.max():.3e} at {g} (bound {tau:.3e}), "
        f"max |dq|/|q| {np.max(err / np.maximum(np.abs(q_o), 1e-300)):.3e}, normwise {rel:.3e}")
    assert np.all(np.isfinite(q_g))
    assert ratio.max() <= tau, (g, q_g[g], q_o[g], scale[g])
    return rel


@pytest.mark.timeout(900)
@pytest.mark.parametrize("k", [2, 3, 4])
def test_full_size_fp64(torch_cuda, k):
    t = torch_cuda
    prob, I, q_o, nrm, kap = _workload(k)
    say(f"full size fp64 workload {k}")
    ctx, _ = _bench_context(prob, "f64", t)
    q_g = _gpu_apply(t, ctx, prob.lam)
    rel = _check_q(prob, q_g, q_o, _scale(prob, nrm, prob.lam), 1e-12, "fp64")
    # normwise against ||q||, which cancellation between the two carriers of
    # a gluing multiplier makes far smaller than the scales above: 1e-12, or
    # the conditioning bound of any FP64 Cholesky-based operator when that is
    # larger (the uneven elasticity workload: kappa up to ~1e7)
    tol_n = max(1e-12, kap.max() * EPS)
    say(f"  normwise |dq|/|q| {rel:.3e} (bound {tol_n:.2e})")
    assert rel <= tol_n
    worst = 0.0
    for i in _sample(prob):
        s = prob.subs[i]
        Fo = feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)
        Fg = ctx.download_F(i)
        d = np.sqrt(np.diag(Fo))
        E = np.abs(Fg - Fo) / np.outer(d, d)
        tol = max(1e-12, kap[i] * EPS)
        worst = max(worst, E.max())
        say(f"  sub {i} n {s.n} m {s.m}: max |dF_ab|/sqrt(F_aa F_bb) {E.max():.3e} "
            f"(tol {tol:.2e}, kappa {kap[i]:.2e})")
        assert np.array_equal(Fg, Fg.T)
        assert E.max() <= tol
    say(f"  workload {k}: worst element-wise F error {worst:.3e}")
    ctx.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_full_size_reduced_precision(torch_cuda, prec):
    """The 216-subdomain heat workload with F~ stored in FP32 / BF16: the
    stored values are bitwise the round-to-nearest-even of the FP64 F~_i of
    the same factor (every subdomain); every q entry within the derived
    bound of the FP64 oracle; FP32 normwise within 1e-5."""
    t = torch_cuda
    prob, I, q_o, nrm, kap = _workload(4)
    say(f"full size {prec} workload 4")
    ctx, trsm = _bench_context(prob, prec, t)
    ref = make_context(prob, f_storage="f64")
    ref.factor_upload([s.Kreg.data for s in prob.subs])
    ref.set_assembly(*trsm)
    ref.assemble()
    t.cuda.synchronize()
    rnd = rne_f32 if prec == "f32" else rne_bf16
    for i in range(prob.nsub):
        F64 = ref.download_F(i)
        assert np.abs(F64).max() < 3e38 and np.abs(F64[F64 != 0]).min() > 1.2e-38
        assert np.array_equal(ctx.download_F(i), rnd(F64)), i
    say(f"  stored {prec} F~ equals RNE(FP64 F~) bitwise on all {prob.nsub} subdomains")
    ref.close()
    q_g = _gpu_apply(t, ctx, prob.lam)
    tau = reduced_apply_bound(prec, max(s.m for s in prob.subs))
    rel = _check_q(prob, q_g, q_o, _scale(prob, nrm, prob.lam), tau, prec)
    if prec == "f32":
        assert rel <= 1e-5
    ctx.close()
