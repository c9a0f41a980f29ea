"""The allocation-free apply (fetiF_apply_static) against fetiF_apply.

fetiF_apply_static runs the same band and gather kernels as fetiF_apply with
the band partials in the library's static device array instead of the
context's buffer, so q must be bitwise the same.  Two calls in a row on one
device, the second on a smaller problem (another context), each checked
against fetiF_apply of its own context and against the oracle's explicit
apply (eq. dualop_apply_expl) at 1e-12; FP32 storage as well.  A plan whose
partials exceed the array is refused with FETIF_ENOTSUP and leaves q as it
was.
"""
import numpy as np
import pytest

from synth import config_problem, make_problem
from oracle import feti
from tests.gpu_common import say, make_context, upload_and_assemble

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def _oracle_q(prob):
    Fs = [feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign) for s in prob.subs]
    return feti.apply_explicit(Fs, [s.dual_map for s in prob.subs], prob.lam, prob.n_lambda)


def _both(t, ctx, lam):
    lam_d = t.tensor(lam, dtype=t.float64, device="cuda")
    q_ref = t.empty_like(lam_d)
    q_st = t.full_like(lam_d, float("nan"))
    ctx.apply(lam_d, q_ref)
    ctx.apply_static(lam_d, q_st)
    t.cuda.synchronize()
    return q_ref.cpu().numpy(), q_st.cpu().numpy()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_static_apply_two_calls_second_smaller(torch_cuda, prec):
    t = torch_cuda
    big = config_problem(5, scale=(3, 6))
    small = make_problem(2, "heat", [[7, 9], [8, 6]], 0.5, dirichlet_axis=0, seed=12)
    assert small.n_lambda < big.n_lambda
    tol = 1e-12 if prec == "f64" else 1e-5
    for label, prob in (("first (larger)", big), ("second (smaller)", small)):
        say(f"static apply {prec}: {label}: {prob.nsub} subdomains, n_lambda {prob.n_lambda}")
        ctx = make_context(prob, f_storage=prec)
        upload_and_assemble(ctx, prob)
        q_ref, q_st = _both(t, ctx, prob.lam)
        q_o = _oracle_q(prob)
        err = np.linalg.norm(q_st - q_o) / np.linalg.norm(q_o)
        say(f"  bitwise equal to fetiF_apply: {np.array_equal(q_st, q_ref)}, rel err vs oracle {err:.2e}")
        assert np.array_equal(q_st, q_ref)
        assert err <= tol
        ctx.close()


def test_static_apply_refuses_partials_beyond_the_array(torch_cuda):
    """One-row bands make the partial vectors as long as the triangles
    (sum m_i (m_i + 1) / 2 FP64 values, 75 MB here, over the 64 MiB array)."""
    t = torch_cuda
    from paper_2502_08382_amd.fetif import FetiError
    prob = config_problem(5)
    ctx = make_context(prob)
    upload_and_assemble(ctx, prob)
    tri = sum(s.m * (s.m + 1) // 2 for s in prob.subs)
    assert tri * 8 > 64 << 20
    ctx.set_apply(1, 0, -1, 0, -1)
    lam_d = t.tensor(prob.lam, dtype=t.float64, device="cuda")
    q = t.full_like(lam_d, 7.0)
    with pytest.raises(FetiError) as ei:
        ctx.apply_static(lam_d, q)
    assert ei.value.status == 6 and "static scratch" in str(ei.value)
    t.cuda.synchronize()
    assert bool((q == 7.0).all())
    # a plan that fits again: back to bitwise agreement
    ctx.set_apply(131072, 0, -1, 0, -1)
    q_ref, q_st = _both(t, ctx, prob.lam)
    assert np.array_equal(q_st, q_ref)
    ctx.close()
