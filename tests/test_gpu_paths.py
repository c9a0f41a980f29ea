"""The paper's other assembly routes through the same library, against the
oracle (eq. localdualoperator) element by element.

* TRSM path (Sec. IV-C: two TRSMs and an SpMM): the forward solve
  X = L^{-1} P B~^T, the backward solve Z = L^{-T} X (dense, FP64 MFMA),
  then F~ = B~ P^T Z.  It reaches the same F~_i as the SYRK path up to
  rounding: checked against the oracle's refined dense F~_i at
  max(1e-12, kappa(K_reg) eps) per element (scaled by sqrt(F_aa F_bb)) and
  against the SYRK path of the same factor at 1e-13.
* Schur-complement route (Sec. III, the augmented matrix eq.
  matrix_for_sc): the multiplier nodes ordered last, so the factor's
  trailing block is the Cholesky factor of the interior's Schur complement
  and X lives in it; same kernels, same bounds.
The applied operator (every q entry) and FP32/BF16 storage (bitwise RNE of
the FP64 result of the same route) are checked as well.
"""
import numpy as np
import pytest

from synth import config_problem, make_problem
from oracle import feti
from tests.gpu_common import (say, make_context, upload_and_assemble, oracle_F, gpu_apply, elem_err, q_entry_err,
                              rne_f32, rne_bf16)

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps


def _cases():
    return {
        "C5s": lambda: config_problem(5, scale=(2, 6)),
        "C2s": lambda: config_problem(2, scale=(2, 12)),
        "el3": lambda: make_problem(3, "elasticity", [[3, 4], [3, 3], [4, 3]], 0.3, dirichlet_axis=2, seed=3),
        "el8": lambda: make_problem(3, "elasticity", [[8, 7], [8, 8], [7, 8]], 0.3, dirichlet_axis=2, seed=5),
        "heat2d_ragged": lambda: make_problem(2, "heat", [[7, 13, 5], [9, 11]], 0.5, dirichlet_axis=0, seed=9),
        "C2s_tet": lambda: config_problem(2, scale=(2, 12), elem="simplex"),
        "heat1d": lambda: make_problem(1, "heat", [[9, 6, 11]], 0.5, dirichlet_axis=0, seed=5),
    }


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _kappas(prob):
    out = []
    for s in prob.subs:
        w = np.linalg.eigvalsh(s.Kreg.toarray())
        out.append(float(w[-1] / w[0]))
    return out


def _check_F(prob, ctx, label, kap, ref=None):
    """Element-wise against the oracle at max(1e-12, kappa eps); against the
    SYRK path of the same factor at max(1e-13, 8 sqrt(kappa) eps) (the two
    routes share X = L^{-1} P B~^T; the TRSM path's backward solve adds an
    error of order cond(L) eps = sqrt(kappa) eps)."""
    worst = worst_ref = 0.0
    for i, s in enumerate(prob.subs):
        Fo = oracle_F(prob, i)
        Fg = ctx.download_F(i)
        tol = max(1e-12, kap[i] * EPS)
        e = elem_err(Fg, Fo)
        worst = max(worst, e)
        assert e <= tol, (i, e, tol)
        if ref is not None:
            er = elem_err(Fg, ref.download_F(i))
            worst_ref = max(worst_ref, er)
            assert er <= max(1e-13, 8 * np.sqrt(kap[i]) * EPS), (i, er)
    say(f"  {label}: max element-wise error vs oracle {worst:.2e}" +
        ("" if ref is None else f", vs the SYRK path of the same factor {worst_ref:.2e}"))


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_trsm_path_matches_oracle(torch_cuda, case):
    prob = _cases()[case]()
    say("trsm path", case, "nsub", prob.nsub, "m", [s.m for s in prob.subs][:6])
    ref = make_context(prob)
    upload_and_assemble(ref, prob)
    ctx = make_context(prob)
    ctx.set_assembly_path(1)
    upload_and_assemble(ctx, prob)
    assert ctx.info()["trsm_bwd_flops"] > 0
    kap = _kappas(prob)
    _check_F(prob, ctx, "TRSM path", kap, ref)
    Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
    q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
    q_g = gpu_apply(ctx, prob.lam)
    r = q_entry_err(prob, q_g, q_o, Fs)
    say(f"  apply after the TRSM path: every entry max |dq|/s_g {r:.2e}")
    assert r <= max(1e-12, max(kap) * EPS)
    # back to the SYRK path: the same F~ as a context that never left it
    ctx.set_assembly_path(0)
    upload_and_assemble(ctx, prob)
    for i in range(prob.nsub):
        assert np.array_equal(ctx.download_F(i), ref.download_F(i))
    ctx.close()
    ref.close()


@pytest.mark.parametrize("panel", [16, 48, 96])
def test_trsm_path_every_panel_width(torch_cuda, panel):
    """Backward panels of 16..96 columns (1..6 row blocks, partial last
    blocks) on an elasticity case whose supernodes span several panels."""
    from paper_2502_08382_amd.fetif import FetiError
    prob = _cases()["el8"]()
    ref = make_context(prob)
    upload_and_assemble(ref, prob)
    ctx = make_context(prob)
    ctx.set_assembly_path(1)
    ctx.set_assembly(panel, 32)
    upload_and_assemble(ctx, prob)
    kap = _kappas(prob)
    worst = max(elem_err(ctx.download_F(i), ref.download_F(i)) / max(1e-13, 8 * np.sqrt(kap[i]) * EPS)
                for i in range(prob.nsub))
    say(f"trsm path panel {panel}: vs SYRK path, max error / bound {worst:.2e}")
    assert worst <= 1.0
    with pytest.raises(FetiError) as e:
        ctx.factor_assemble([s.Kreg.data for s in prob.subs])
    assert e.value.status == 6
    ctx.close()
    ref.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_trsm_path_reduced_storage_is_rne(torch_cuda, prec):
    prob = _cases()["C2s"]()
    ref = make_context(prob)
    ref.set_assembly_path(1)
    upload_and_assemble(ref, prob)
    ctx = make_context(prob, f_storage=prec)
    ctx.set_assembly_path(1)
    upload_and_assemble(ctx, prob)
    rnd = rne_f32 if prec == "f32" else rne_bf16
    for i in range(prob.nsub):
        assert np.array_equal(ctx.download_F(i), rnd(ref.download_F(i))), i
    say(f"trsm path {prec}: stored F~ equals RNE of the FP64 TRSM-path F~ on all {prob.nsub} subdomains")
    ctx.close()
    ref.close()


@pytest.mark.parametrize("case", ["C5s", "C2s", "el3", "heat2d_ragged", "C2s_tet", "heat1d"])
def test_schur_complement_order_matches_oracle(torch_cuda, case):
    prob = _cases()[case]()
    say("schur-complement order", case)
    ref = make_context(prob)
    upload_and_assemble(ref, prob)
    ctx = make_context(prob, schur_order=1)
    upload_and_assemble(ctx, prob)
    i_sc, i_nd = ctx.info(), ref.info()
    say(f"  flops trsm {i_sc['trsm_flops']:.3g} (nested dissection {i_nd['trsm_flops']:.3g}), "
        f"syrk {i_sc['syrk_flops']:.3g} ({i_nd['syrk_flops']:.3g})")
    kap = _kappas(prob)
    _check_F(prob, ctx, "Schur-complement order", kap)
    Fs = [oracle_F(prob, i) for i in range(prob.nsub)]
    q_o = feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)
    r = q_entry_err(prob, gpu_apply(ctx, prob.lam), q_o, Fs)
    assert r <= max(1e-12, max(kap) * EPS)
    ctx.close()
    ref.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_host_vector_apply_scatter_gather_on_gpu_or_cpu(torch_cuda, prec):
    """fetiF_apply_host with the scatter/gather on the GPU (0) or on host
    threads (1): both equal fetiF_apply bitwise (same band kernels on the
    same values, the same fixed gather order), on two problems in turn."""
    for prob in (config_problem(5, scale=(3, 6)), make_problem(2, "heat", [[7, 13, 5], [9, 11]], 0.5,
                                                                dirichlet_axis=0, seed=9)):
        ctx = make_context(prob, f_storage=prec)
        upload_and_assemble(ctx, prob)
        q_dev = gpu_apply(ctx, prob.lam)
        for sg in (0, 1, 1, 0):
            q_h = ctx.apply_host(prob.lam, cpu_scatter_gather=sg)
            assert np.array_equal(q_h, q_dev), (sg, np.abs(q_h - q_dev).max())
        say(f"host-vector apply {prec}: n_lambda {prob.n_lambda}: GPU and CPU scatter/gather bitwise equal "
            f"to fetiF_apply")
        ctx.close()


def test_read_probe_sums_every_region(torch_cuda):
    """The streaming-read probe (a measurement aid) reads every byte once:
    region sums of a buffer of k = 0, 1, 2, ... equal the closed form, also
    for a ragged last region."""
    t = torch_cuda
    from paper_2502_08382_amd.fetif import read_probe
    n = 3 * (1 << 20) + 4098                 # FP64 values; bytes not a multiple of the region
    buf = t.arange(n, dtype=t.float64, device="cuda")
    for region in (16384, 1 << 20):
        per = region // 8
        ng = -(-n // per)
        out = t.full((ng,), float("nan"), dtype=t.float64, device="cuda")
        read_probe(buf, region, out)
        t.cuda.synchronize()
        lo = np.arange(ng) * per
        hi = np.minimum(lo + per, n)
        expect = (hi * (hi - 1) - lo * (lo - 1)) / 2.0
        got = out.cpu().numpy()
        assert np.allclose(got, expect, rtol=1e-12, atol=0), (region, np.abs(got - expect).max())
