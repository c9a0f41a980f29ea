"""Helpers shared by the GPU parity tests (they only marshal data between the
oracle, the generator and the library)."""
import sys

import numpy as np

from oracle import feti


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def make_context(prob, f_storage="f64", with_elements=False, **opts):
    from paper_2502_08382_amd import FetiContext, subdomain_dict
    subs = [subdomain_dict(s, with_elements) for s in prob.subs]
    return FetiContext(subs, prob.n_lambda, device=0, f_storage=f_storage, **opts)


def upload_and_assemble(ctx, prob):
    import torch
    ctx.factor_upload([s.Kreg.data for s in prob.subs])
    ctx.assemble()
    torch.cuda.synchronize()


def oracle_F(prob, idx):
    s = prob.subs[idx]
    return feti.local_dual_operator(s.Kreg, s.b_dof, s.b_sign)


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_apply(ctx, lam):
    import torch
    lam_d = torch.tensor(lam, dtype=torch.float64, device="cuda")
    q_d = torch.empty_like(lam_d)
    ctx.apply(lam_d, q_d)
    torch.cuda.synchronize()
    return q_d.cpu().numpy()


def elem_err(Fg, Fo):
    """max_ab |Fg[a,b] - Fo[a,b]| / sqrt(Fo[a,a] Fo[b,b]) (element-wise,
    scaled by the Cauchy-Schwarz bound |F_ab| <= sqrt(F_aa F_bb))."""
    d = np.sqrt(np.maximum(np.diag(Fo), 1e-300))
    return float((np.abs(Fg - Fo) / np.outer(d, d)).max())


def q_entry_err(prob, q_g, q_o, Fs, lam=None):
    """max_g |q_g - q_o| / s_g with s_g = sum over the carriers of g of
    ||F~_i||_2 ||lambda_i||_2 (an upper bound of sum_b |F_ab| |lambda_b|)."""
    lam = prob.lam if lam is None else lam
    s = np.zeros(prob.n_lambda)
    for F, sub in zip(Fs, prob.subs):
        s[sub.dual_map] += np.linalg.norm(F, 2) * np.linalg.norm(lam[sub.dual_map])
    return float((np.abs(q_g - q_o) / s).max())


def rne_bf16(x):
    """Round-to-nearest-even of float64 values to bfloat16 (8 significant
    bits), returned as float64; for values in bfloat16's normal range."""
    m, e = np.frexp(x)
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


def rne_f32(x):
    """Round-to-nearest-even of float64 values to float32, as float64."""
    return np.asarray(x).astype(np.float32).astype(np.float64)


def reduced_apply_bound(prec, m_max):
    """Per-entry bound (relative to sum_b |F_ab| |lambda_b|, or any upper
    bound of it) of the FP32-accumulated apply of F~ stored in `prec`:
    storage rounding + lambda rounded to FP32 + FP32 sums no deeper than
    ceil(m_max / 4) + 64 additions."""
    u = 2.0 ** -24
    us = {"f32": u, "bf16": 2.0 ** -8}[prec]
    d = -(-m_max // 4) + 64
    return us + u + d * u / (1 - d * u)
