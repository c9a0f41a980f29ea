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
